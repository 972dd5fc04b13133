// nw_fork.h -- spreading independent launches over library streams.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

namespace nw {

// Independent launches (the per-length launches of one call, which write
// disjoint outputs or commute through atomics) spread over the caller's
// stream and kForkStreams library streams of the current device, so that the
// tail of one launch overlaps the start of the next.  The library streams
// first wait for the caller's work so far; the caller's stream then waits for
// theirs, so the call stays ordered on the caller's stream.  The library
// streams are created once per device and kept for the process; calls from
// several host threads share them, which can serialize those calls against
// each other but cannot deadlock: every wait binds to an event already
// recorded, so each dependency points to work enqueued earlier.
#ifndef NW_FORK_STREAMS
#define NW_FORK_STREAMS 3
#endif
constexpr int kForkStreams = NW_FORK_STREAMS;

class StreamFork {
  public:
    explicit StreamFork(hipStream_t caller) : caller_(caller) {}
    // Graph mode: every launch becomes a kernel node of `graph` without
    // dependencies, so the nodes of one graph may run side by side on replay
    // (no streams or events are involved; begin and end do nothing).
    explicit StreamFork(hipGraph_t graph) : caller_(nullptr), graph_(graph) {}
    StreamFork(const StreamFork &) = delete;
    StreamFork &operator=(const StreamFork &) = delete;
    ~StreamFork()
    {
        if (begun_ && !ended_) (void)end();   // an error path still joins what was launched
        for (hipEvent_t &e : done_)
            if (e) hipEventDestroy(e);
        if (start_) hipEventDestroy(start_);
    }
    // every launch after begin() goes to next().  A caller's stream that is
    // being captured into a graph is not forked: the launches stay on it, in
    // order (no library streams or events enter a capture).
    hipError_t begin()
    {
        if (graph_) return hipSuccess;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(caller_, &cs);
        if (e != hipSuccess) return e;
        if (cs != hipStreamCaptureStatusNone) return hipSuccess;
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if ((e = library_streams(dev, lib_)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&start_, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventRecord(start_, caller_)) != hipSuccess) return e;
        for (int i = 0; i < kForkStreams; ++i)
            if ((e = hipStreamWaitEvent(lib_[i], start_, 0)) != hipSuccess) return e;
        begun_ = true;
        return hipSuccess;
    }
    hipStream_t next()
    {
        if (!begun_) return caller_;
        const int i = turn_++ % (kForkStreams + 1);
        used_[i] = true;
        return i == 0 ? caller_ : lib_[i - 1];
    }
    // One launch: on next()'s stream, or as a node of the graph.
    hipError_t launch(const void *fn, dim3 grid, dim3 block, size_t lds, void **args)
    {
        if (graph_) {
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(fn);
            p.gridDim = grid;
            p.blockDim = block;
            p.sharedMemBytes = (unsigned int)lds;
            p.kernelParams = args;   // the values are copied into the node
            p.extra = nullptr;
            hipGraphNode_t node;
            return hipGraphAddKernelNode(&node, graph_, nullptr, 0, &p);
        }
        return hipLaunchKernel(fn, grid, block, args, lds, next());
    }
    // the caller's stream waits for every library stream that took a launch
    hipError_t end()
    {
        ended_ = true;
        for (int i = 0; i < kForkStreams; ++i) {
            if (!used_[i + 1]) continue;
            hipError_t e = hipEventCreateWithFlags(&done_[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(done_[i], lib_[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(caller_, done_[i], 0);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

  private:
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
    hipStream_t lib_[kForkStreams] = {};
    hipEvent_t start_ = nullptr;
    hipEvent_t done_[kForkStreams] = {};
    bool used_[kForkStreams + 1] = {};
    bool begun_ = false, ended_ = false;
    int turn_ = 0;
};

}  // namespace nw
