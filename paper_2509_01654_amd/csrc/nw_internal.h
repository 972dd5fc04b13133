// nw_internal.h -- device layout of a loaded dictionary and the launchers the
// C ABI calls.  Shared by the host runtime (nw_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nw_topk.h"

namespace nw {

// Longest word of the register-row kernels (the DP column is unrolled per
// exact length up to this bound); the anti-diagonal kernel takes longer words
// (up to kLongMaxLen) for the triangle calls.
constexpr int kMaxLen = 48;
constexpr int kLongMaxLen = 255;   // lengths are stored as uint8
constexpr uint32_t kMaxLdsBytes = 160u * 1024u;   // LDS of one workgroup (and of one CU)
constexpr int kDiagClasses = 8;    // row-length classes of the anti-diagonal kernel (32 lengths each)
// Threads per workgroup of the tiled kernels (four wave64 wavefronts).
constexpr int kThreads = 256;
// Bytes of a padded word in the blocked layout (kMaxLen symbols, whole 16-byte loads).
constexpr int kWordBytes = 48;
// Profile entry of the sentinel symbol that pads lane words: -2048 in both
// binary16 halves (0xE800 is the binary16 encoding of -2048).
constexpr uint32_t kSentinelPair = 0xE800E800u;

// The dictionary as the kernels see it.  All pointers are device memory inside
// the caller's d_mem.
//
// Caller order: word u has length clen[u] and symbols csym[u*WB .. u*WB+len).
// Blocked order: the words are cut into blocks of CB consecutive caller-order
// words; inside each block they are sorted by length, and words of one
// length lexicographically (ties by caller index).  Sorted slot
// s (global: block*CB + local) holds the word whose caller index is
// block*CB + bcol[s]; its symbols are bsym[s*WB ..] and its length blen[s]
// (0 for the padding slots of the last block).
// Row pairs: for block r and length L, rpairs[rp_off[r*(LMAX+1)+L] .. rp_off[..+1])
// lists pairs of sorted slots of that block whose words both have length L
// (second slot -1 when the count is odd).  gpairs holds the same pairs grouped
// by length only: gpairs[gp_off[L] .. gp_off[L+1]).  dpairs pairs the words of
// a block by class of the anti-diagonal kernel instead (class c: lengths
// 32c+1 .. 32c+32), consecutive in slot order (so of similar lengths):
// dpairs[dp_off[r*kDiagClasses + c] .. dp_off[r*kDiagClasses + c + 1]).
// borig[s] is the caller index of slot s (-1 for padding slots).
// Probe subset (threshold pre-pass of the top-k): nprobe words at caller
// indices floor(i*n/nprobe), sorted by length, as a column set of pslots slots.
struct DevVocab {
    const uint8_t *csym;
    const uint8_t *clen;
    const uint8_t *bsym;
    const uint8_t *blen;
    const uint16_t *bcol;
    const int32_t *rpairs;      // [num_row_pairs][2]
    const uint32_t *rp_off;     // [nb*(LMAX+1)+1]
    const uint16_t *wtab;       // [alphabet*alphabet] binary16 bits of sim(x,y) - 2*gap
    int64_t n;
    int32_t nb;                 // number of blocks
    int32_t CB;                 // block size (multiple of kThreads)
    int32_t WB;                 // bytes per padded word (32 or 48)
    int32_t lmax;               // LMAX of the rp_off table (longest word)
    int32_t alphabet;
    int32_t gap;
    int32_t match, mismatch;    // plain +/- scoring when has_submat == 0
    int32_t has_submat;
    const int8_t *submat;       // [alphabet*alphabet] when has_submat
    const int32_t *borig;       // [nb*CB]
    const int32_t *gpairs;      // [num_row_pairs][2]
    const uint32_t *gp_off;     // [kMaxLen+2]
    const int32_t *dpairs;      // row pairs of the anti-diagonal classes, [.][2]
    const uint32_t *dp_off;     // [nb*kDiagClasses+1]
    const uint8_t *psym;        // probe words [pslots*WB]
    const uint8_t *plen;        // [pslots]
    const int32_t *porig;       // [pslots]
    const uint16_t *prank;      // [pslots] rank i of each probe slot (0 for padding)
    int64_t pslots;
    int32_t nprobe;
    int32_t lo, hi;             // score bounds
};

enum OutKind { OUT_I8 = 1, OUT_I16 = 2, OUT_EDGES = 3 };

// Sink of the threshold edge emitter (graph export, Section 5): every pair
// (i, j), i < j, whose raw score s or normalised weight 100 s / max(len i,
// len j) lies in the closed slice is appended as (i, j, s).  The slice is
// [lo, hi] on s when normalised == 0, and [lo/den, hi/den] on the weight
// otherwise, compared exactly in integers: lo*m <= 100*s*den <= hi*m with
// m = max(len i, len j, 1).  `count` counts every passing pair; only the
// first `cap` appended are stored, in no particular order.
struct EdgeSink {
    int32_t *ei;
    int32_t *ej;
    int16_t *es;
    unsigned long long *count;
    uint64_t cap;
    int32_t normalised;
    int32_t lo, hi, den;
};

// Launchers.  Each enqueues on `stream` and returns the hipError_t of the
// launches.  Launchers with one launch per row length (or class) spread those
// independent launches over `stream` and three library streams of the device,
// forked from `stream` and joined back into it with events, so the work is
// still ordered on `stream` for the caller.

// Triangle scores of pair indices [idx_begin, idx_end); with out_kind ==
// OUT_EDGES the pairs of that range go to the edge sink E instead of d_out.
// h_maxrp[LA] (host) = most row pairs of length LA in one block: sets how
// far tiles are split when the launch has few of them.
// Dictionaries of at most kClassLaunchMaxWords words take one launch per class
// of 8 row lengths (k_tri_class), larger ones one launch per row length.  With
// `shared`, the launches join that fork (begun and ended by the caller)
// instead of one of their own.
constexpr int64_t kClassLaunchMaxWords = 16384;
class StreamFork;
hipError_t launch_triangle_tiled(const DevVocab &V, const uint32_t *h_maxrp, uint64_t idx_begin, uint64_t idx_end,
                                 int out_kind, void *d_out, hipStream_t stream, const EdgeSink *E = nullptr,
                                 StreamFork *shared = nullptr);
hipError_t launch_triangle_naive(const DevVocab &V, uint64_t idx_begin, uint64_t idx_end, int out_kind,
                                 void *d_out, hipStream_t stream, const EdgeSink *E = nullptr);
// Threshold edges of pair indices [idx_begin, idx_end) into E, scored and
// tested in registers (words of at most kMaxLen symbols).
hipError_t launch_edges_tiled(const DevVocab &V, const uint32_t *h_maxrp, uint64_t idx_begin, uint64_t idx_end,
                              const EdgeSink &E, hipStream_t stream);
// Anti-diagonal (16 lanes per pair) kernel, words up to 255 symbols; one
// launch per class of row lengths.  A dictionary whose longest words need a
// profile larger than LDS (diag_fits false) is scored by the naive kernel.
bool diag_fits(const DevVocab &V);
// h_maxrp[0] = most empty row pairs in one block; h_maxdp[c] = most row pairs
// of class c in one block.
hipError_t launch_triangle_diag(const DevVocab &V, const uint32_t *h_maxrp, const uint32_t *h_maxdp,
                                uint64_t idx_begin, uint64_t idx_end, int out_kind, void *d_out, hipStream_t stream,
                                const EdgeSink *E = nullptr);

// Partial lists per row of a query launch over nsplit column splits: the four
// wavefront lists with one split, one merged list per split otherwise.
__host__ __device__ constexpr int query_lists(int nsplit) { return nsplit == 1 ? 4 : nsplit; }

// Per-row top-k lists of the rows R (pairs grouped by length, h_off = host
// copy of R.off) against the column set C, split over nsplit column ranges:
// partial[row][query_lists(nsplit)][k].  Scoring from V.  fork_streams spreads the
// per-length launches over library streams (throughput calls; latency-bound
// callers such as the server keep them on `stream`).
hipError_t launch_query(const DevVocab &V, const RowSet &R, const uint32_t *h_off, const ColSet &C, int k,
                        int nsplit, uint64_t *partial, hipStream_t stream, bool fork_streams = false);

// Merge partial lists [rows][P][kin] into the top kout (scores/indices
// and/or the key of rank `rank`).
hipError_t launch_merge(const uint64_t *partial, int P, int kin, int64_t rows, int kout, int lo, int16_t *score,
                        int32_t *index, uint64_t *thr, int rank, hipStream_t stream);

// The threshold pre-pass of the all-pairs top-k by selection (k_probe.h):
// thr[u] = the key of rank m of every word u of R against V's probe subset.
// Returns hipErrorNotSupported, launching nothing, when probe_thr_applies(V)
// is false.
bool probe_thr_applies(const DevVocab &V);
hipError_t launch_probe_thr(const DevVocab &V, const RowSet &R, const uint32_t *h_off, int m, uint64_t *thr,
                            hipStream_t stream);

// Write recomputed lists: for t < B, the first k entries of (qs, qi)[t][0..kq)
// whose index is not words[t] go to score/index[words[t]][0..k), padded with
// (INT16_MIN, -1).
hipError_t launch_scatter_lists(const int16_t *qs, const int32_t *qi, const int32_t *words, uint32_t B, int kq, int k,
                                int16_t *score, int32_t *index, hipStream_t stream);

// Main pass of the all-pairs top-k: candidates >= thr into per-word lists,
// plus the histogram.
struct TopkArgs;
hipError_t launch_topk_main(const DevVocab &V, const TopkArgs &T, hipStream_t stream);

// Zero n counters (a kernel, so graph capture records no memset node).
hipError_t launch_reset_counters(uint32_t *counters, int n, hipStream_t stream);

// Raise each word's threshold to the k-th best of its candidates so far.
hipError_t launch_tighten(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n, int k, uint64_t *thr,
                          hipStream_t stream);

// Final per-word selection from the candidate lists.
hipError_t launch_select(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n, int k, int lo,
                         int16_t *score, int32_t *index, uint32_t *ovf_count, int32_t *ovf_list, hipStream_t stream);

}  // namespace nw
