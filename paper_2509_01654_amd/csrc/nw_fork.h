// nw_fork.h -- spreading independent launches over concurrent chains.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

namespace nw {

// Independent launches (the per-length launches of one call, which write
// disjoint outputs or commute through atomics) are dealt round-robin to
// kChains chains, so that the tail of one launch overlaps the start of the
// next.  The whole set stays ordered after the caller's earlier work and
// before its later work.  Two forms:
//
// - Eager (the caller's stream is not capturing): chain 0 is the caller's
//   stream, chains 1.. are library streams of the current device.  A library
//   stream waits for an event recorded on the caller's stream at begin(),
//   the first time it is given a launch; end() makes the caller's stream
//   wait for an event recorded on every library stream that took one.  The
//   library streams are created once per device and kept for the process
//   (default priority); calls from several host threads share them, which can
//   serialize those calls against each other but cannot deadlock: every wait
//   binds to an event already recorded, so each dependency points to work
//   enqueued earlier.
//
// - Capture (the caller's stream is being captured into a graph): no stream
//   or event is involved.  Each launch becomes a kernel node added directly to
//   the capture's graph; the first node of a chain depends on the capture's
//   current dependency set, each later one on the chain's previous node, and
//   end() replaces the stream's dependency set by the last node of every
//   chain.  Events recorded into a capture belong to it until the capture
//   ends, and library streams made to wait on them join it; neither can be
//   tied to a caller's capture that ends after this object is gone, so a
//   captured fork uses neither.
#ifndef NW_FORK_STREAMS
#define NW_FORK_STREAMS 3
#endif
constexpr int kForkStreams = NW_FORK_STREAMS;
constexpr int kChains = kForkStreams + 1;

class StreamFork {
  public:
    explicit StreamFork(hipStream_t caller) : caller_(caller) {}
    StreamFork(const StreamFork &) = delete;
    StreamFork &operator=(const StreamFork &) = delete;
    ~StreamFork()
    {
        if (mode_ == kStreams) {
            if (!ended_) (void)end();   // an error path still joins what was launched
            for (hipEvent_t &e : done_)
                if (e) hipEventDestroy(e);
            if (start_) hipEventDestroy(start_);
        }
    }

    // Launches after begin() are spread over the chains; without begin() they
    // all go to the caller's stream in order.
    hipError_t begin()
    {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        unsigned long long id = 0;
        hipGraph_t g = nullptr;
        const hipGraphNode_t *deps = nullptr;
        size_t nd = 0;
        hipError_t e = hipStreamGetCaptureInfo_v2(caller_, &cs, &id, &g, &deps, &nd);
        if (e != hipSuccess) return e;
        if (cs == hipStreamCaptureStatusInvalidated) return hipErrorStreamCaptureInvalidated;
        if (cs == hipStreamCaptureStatusActive) {
            graph_ = g;
            roots_.assign(deps, deps + nd);
            mode_ = kNodes;
            return hipSuccess;
        }
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = library_streams(dev, lib_)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&start_, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventRecord(start_, caller_)) != hipSuccess) return e;
        mode_ = kStreams;
        return hipSuccess;
    }

    // One launch on the next chain.
    hipError_t launch(const void *fn, dim3 grid, dim3 block, size_t lds, void **args)
    {
        const int c = turn_++ % kChains;
        if (mode_ == kNodes) {
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(fn);
            p.gridDim = grid;
            p.blockDim = block;
            p.sharedMemBytes = (unsigned int)lds;
            p.kernelParams = args;   // the values are copied into the node
            p.extra = nullptr;
            const hipGraphNode_t *dep = tail_[c] ? &tail_[c] : roots_.data();
            const size_t nd = tail_[c] ? 1 : roots_.size();
            hipGraphNode_t node = nullptr;
            hipError_t e = hipGraphAddKernelNode(&node, graph_, nd ? dep : nullptr, nd, &p);
            if (e == hipSuccess) tail_[c] = node;
            return e;
        }
        hipStream_t s = caller_;
        if (mode_ == kStreams && c > 0) {
            if (!used_[c - 1]) {
                hipError_t e = hipStreamWaitEvent(lib_[c - 1], start_, 0);
                if (e != hipSuccess) return e;
                used_[c - 1] = true;
            }
            s = lib_[c - 1];
        }
        return hipLaunchKernel(fn, grid, block, args, lds, s);
    }

    // Join every chain back into the caller's stream (its capture's dependency
    // set, or the stream itself); nothing to do for a fork never begun.
    hipError_t end()
    {
        ended_ = true;
        if (mode_ == kNodes) {
            std::vector<hipGraphNode_t> last;
            for (hipGraphNode_t t : tail_)
                if (t) last.push_back(t);
            if (last.empty()) return hipSuccess;   // no launch: the dependency set is unchanged
            return hipStreamUpdateCaptureDependencies(caller_, last.data(), last.size(),
                                                      hipStreamSetCaptureDependencies);
        }
        if (mode_ != kStreams) return hipSuccess;
        for (int i = 0; i < kForkStreams; ++i) {
            if (!used_[i] || done_[i]) continue;
            hipError_t e = hipEventCreateWithFlags(&done_[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(done_[i], lib_[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(caller_, done_[i], 0);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

  private:
    enum Mode { kNone, kStreams, kNodes };
    static hipError_t library_streams(int dev, hipStream_t (&out)[kForkStreams])
    {
        static std::mutex mu;
        static hipStream_t streams[64][kForkStreams] = {};
        if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lock(mu);
        for (int i = 0; i < kForkStreams; ++i) {
            if (!streams[dev][i]) {
                hipError_t e = hipStreamCreateWithFlags(&streams[dev][i], hipStreamNonBlocking);
                if (e != hipSuccess) return e;
            }
            out[i] = streams[dev][i];
        }
        return hipSuccess;
    }
    hipStream_t caller_;
    hipGraph_t graph_ = nullptr;
    Mode mode_ = kNone;
    std::vector<hipGraphNode_t> roots_;        // the capture's dependency set at begin()
    hipGraphNode_t tail_[kChains] = {};        // last node of each chain
    hipStream_t lib_[kForkStreams] = {};
    hipEvent_t start_ = nullptr;
    hipEvent_t done_[kForkStreams] = {};
    bool used_[kForkStreams] = {};             // library stream i waited on start_ and took a launch
    bool ended_ = false;
    int turn_ = 0;
};

}  // namespace nw
