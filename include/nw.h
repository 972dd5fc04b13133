/*
 * nw.h -- C ABI of libnw: all-pairs Needleman-Wunsch scoring on MI355X (gfx950).
 *
 * The operation is the global-alignment score of Algorithm 1 of Plein,
 * "Parallel Needleman-Wunsch on CUDA to measure word similarity based on
 * phonetic transcriptions" (2025), Section 2: the maximum, over all global
 * alignments of words A and B, of the sum of similarity(A_x, B_y) over aligned
 * symbol pairs plus the linear gap penalty p for every gap symbol (leading and
 * trailing gaps included).  Words are integer-encoded symbol sequences
 * (Section 3).  Every score is an exact integer.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: NW_OK (0) or a negative status; nw_last_error() then holds a
 *   thread-local message.  Argument errors are detected before anything is
 *   enqueued.  Device errors reported by the HIP runtime surface as NW_EDEVICE.
 * - Pointers named h_* are host memory; d_* are device memory of the current
 *   HIP device; hip_stream is a hipStream_t (NULL = the null stream).
 * - The caller owns every buffer.  The library never allocates device memory:
 *   it works inside the memory (d_mem, d_ws) the caller hands in, whose sizes
 *   the *_bytes queries give.  Host arrays may be reused as soon as a call
 *   returns (the library copies what it needs before returning).
 * - Calls enqueue kernels on hip_stream and return; results are valid once the
 *   stream has been synchronised.  An nw_vocab must outlive every call that
 *   uses it and every kernel those calls enqueued.
 * - Word i is h_symbols[h_offsets[i] .. h_offsets[i+1]).  Lengths may be 0.
 * - Graph capture: the triangle calls (nw_all_pairs_scores and its forms,
 *   nw_all_pairs_scores_batched), nw_all_pairs_edges, nw_batch_run and
 *   nw_ego_network may be enqueued on a stream that is being captured into a
 *   hipGraph; their independent launches become parallel chains of kernel
 *   nodes of the capture, and no memset, event or host callback enters it.
 *   The calls that wait for the device, read results back, copy from
 *   pageable host memory or run host callbacks (nw_load_vocab,
 *   nw_all_pairs_topk, nw_all_pairs_topk_async, nw_topk_finish, nw_query,
 *   nw_export_triangle, nw_graph_csr, nw_batch_autotune) return NW_EINVAL on
 *   a capturing stream, before enqueuing anything.
 */
#ifndef NW_H
#define NW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NW_OK = 0,
    NW_EINVAL = -1,   /* invalid argument (symbol >= alphabet, word too long, gap > 0, ...) */
    NW_ERANGE = -2,   /* scores or DP values do not fit the requested/internal type       */
    NW_ENOMEM = -3,   /* the memory handed in is smaller than the *_bytes query says       */
    NW_EDEVICE = -4,  /* the HIP runtime reported an error                                 */
    NW_ESTOPPED = -5  /* a caller callback asked the call to stop                          */
};

typedef enum { NW_I8 = 1, NW_I16 = 2 } nw_dtype;

/* Scoring of Algorithm 1: the similarity function and the gap penalty p.
 * similarity(x, y) = submat[x * alphabet + y] if submat != NULL (host memory,
 * copied at load), else match when x == y and mismatch otherwise.  x is a
 * symbol of A (the row word), y a symbol of B.  gap is added once per gap
 * symbol and must be <= 0 (Section 2 uses -2 in its examples, Section 4 uses
 * -1 for every run). */
typedef struct {
    int32_t alphabet;        /* 1..255; every symbol must be < alphabet   */
    int32_t match;           /* used when submat == NULL                  */
    int32_t mismatch;        /* used when submat == NULL                  */
    int32_t gap;             /* linear gap penalty p <= 0                 */
    const int8_t *submat;    /* optional alphabet x alphabet, row-major   */
} nw_scoring;

/* Opaque handle to a device-resident dictionary (host-side descriptor). */
typedef struct nw_vocab nw_vocab;

/* Thread-local text of the last error (never NULL). */
const char *nw_last_error(void);

/* Longest word (symbols) the triangle calls accept (255).  The register-row
 * kernels behind top-k, queries, the batched form and the server take words
 * of at most 48 symbols; a dictionary with longer words is scored by the
 * anti-diagonal kernel and is refused (NW_EINVAL) by those calls. */
int nw_max_word_length(void);

/* Device bytes nw_load_vocab needs for n words holding total_symbols symbols,
 * the longest being max_len.  NW_EINVAL if max_len exceeds the maximum. */
int nw_vocab_bytes(uint64_t n, uint64_t total_symbols, uint32_t max_len, uint64_t *dev_bytes);

/* Validate the words and the scoring, bucket the words by length (inside
 * fixed-size blocks of the caller's order, sorted by length and, within a
 * length, lexicographically) and copy the packed layout into d_mem
 * (>= nw_vocab_bytes(...) bytes, 256-byte aligned).  The order is internal:
 * every result is in the caller's word order.
 * Synchronous: returns after the copy has completed on hip_stream.
 * Errors: NW_EINVAL (n >= 2^31, a symbol >= alphabet, a word longer than
 * nw_max_word_length(), gap > 0, alphabet outside 1..255), NW_ERANGE (the
 * scores of these words could leave int16, or the DP could leave the range
 * its 16-bit cells hold exactly), NW_ENOMEM (d_bytes too small).
 * On success *out receives a handle to release with nw_free_vocab. */
int nw_load_vocab(const uint8_t *h_symbols, const uint64_t *h_offsets, uint64_t n,
                  const nw_scoring *sc, void *d_mem, uint64_t d_bytes, void *hip_stream,
                  nw_vocab **out);

/* Every later call on this handle runs on the device that was current at
 * nw_load_vocab: the library makes it current for the call and restores the
 * caller's device before returning.  Streams and buffers passed with the
 * handle must belong to that device. */

/* Release the host descriptor (d_mem stays owned by the caller). */
void nw_free_vocab(nw_vocab *v);

/* n, the longest word, E = n(n-1)/2 unordered pairs and the number of DP
 * cells sum over pairs of len(i)*len(j). Any out pointer may be NULL. */
int nw_vocab_info(const nw_vocab *v, uint64_t *n, uint32_t *max_len, uint64_t *num_pairs,
                  uint64_t *num_cells);

/* Bounds every pair score of this dictionary lies in:
 * lo = L * min(min similarity, p, 0), hi = L * max(max similarity, 0), L = longest word. */
int nw_score_bounds(const nw_vocab *v, int32_t *lo, int32_t *hi);

/* Scores of the unordered pairs (i, j), i < j, in the row-major order of the
 * upper triangle of the adjacency matrix (Section 4.1):
 * idx(i, j) = i(2n-i-1)/2 + (j-i-1), the forward form of the paper's S_{r-1}
 * (Section 4.2).  Writes d_out[idx - idx_begin] = score(word i, word j) for
 * every idx in [idx_begin, idx_end) -- the restartable chunk the paper
 * proposes for going past device memory (Section 5).  d_out holds
 * (idx_end - idx_begin) elements of dt (int8 or int16), row-major triangle
 * order, in the caller's word order.
 * Errors: NW_EINVAL (NULL vocab, idx_begin > idx_end or idx_end > E, bad
 * dtype, NULL d_out with a non-empty range, a similarity matrix that is not
 * symmetric -- the unordered pairs need score(i, j) = score(j, i)),
 * NW_ERANGE (the score bounds do not fit dt), NW_EDEVICE. */
int nw_all_pairs_scores(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt,
                        void *d_out, void *hip_stream);

/* The whole triangles of nv dictionaries in one call: d_outs[i] receives
 * dictionary v[i]'s scores exactly as nw_all_pairs_scores with the range
 * [0, E_i) writes them (row-major, dtype dt).  The register-row launches of
 * all dictionaries are enqueued as one set of concurrent chains, so one
 * dictionary's tail overlaps the next one's start; dictionaries with words
 * longer than 48 take the anti-diagonal kernel.  Needs no workspace.  This is
 * the one-call batched form; the nw_batch_* calls below plan the same work
 * once (persistent work queues or these launches, optionally as a replayed
 * hipGraph) and let the autotuner choose.  Every dictionary must live on the
 * same device.  Errors: those of nw_all_pairs_scores for any dictionary
 * (the message names it), NW_EINVAL (NULL arrays, dictionaries on different
 * devices), NW_EDEVICE. */
int nw_all_pairs_scores_batched(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt,
                                void *hip_stream);

/* The same scores computed by the intra-pair anti-diagonal kernel: 16 lanes
 * per pair walk the score matrix by anti-diagonals (the stencil
 * parallelisation the paper proposes in Section 6).  nw_all_pairs_scores uses
 * it by itself for words longer than 48; this entry point forces it (for
 * comparison with the register-row kernel).  A dictionary whose longest words
 * need a similarity profile larger than LDS (e.g. more than 125 symbols with
 * words over 192) is scored by the one-thread-per-pair kernel instead.  Same
 * arguments and errors. */
int nw_all_pairs_scores_diag(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt,
                             void *d_out, void *hip_stream);

/* The same scores computed by the one-thread-per-pair scheme of Section 4.2
 * (1-D grid, idx -> (row, column), one DP per thread).  Kept as the plain
 * comparison point for the tiled kernels; same arguments and errors. */
int nw_all_pairs_scores_naive(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt,
                              void *d_out, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Streamed triangle export.  Section 5 stops at about 107,000 words because
 * the whole i8 edge-weight array must fit the GPU, and proposes copying parts
 * of it to the host and continuing with the index shifted back to 0.  This
 * call does that for any range of pair indices: the triangle is computed in
 * chunks of chunk_pairs pairs into two alternating device buffers while the
 * previous chunk is copied to the host on a second stream, and each chunk
 * is handed to the caller in index order.
 * ------------------------------------------------------------------------- */

/* Receives the scores of pair indices [idx_begin, idx_begin + count) in the
 * export's dtype.  h_chunk is valid only during the call.  Return 0 to go on,
 * anything else to stop the export. */
typedef int (*nw_chunk_fn)(void *user, uint64_t idx_begin, uint64_t count, const void *h_chunk);

/* Scores of pair indices [idx_begin, idx_end), the same values and order as
 * nw_all_pairs_scores, delivered through fn (called on the calling thread,
 * once per chunk, in index order; the last chunk may be shorter).
 * d_ws: device memory of 2 * chunk_pairs * sizeof(dt) bytes, 256-byte aligned.
 * h_buf: host memory of the same size; page-locked memory (hipHostMalloc)
 * gives the full transfer rate.  Both are caller-owned and reused in turn.
 * Work is enqueued on hip_stream (kernels) and on a stream the call creates
 * and destroys (copies).  Synchronous: returns once the last chunk has been
 * delivered, or after a stop with every enqueued step finished.
 * Errors: NW_EINVAL (as nw_all_pairs_scores, NULL fn, d_ws or h_buf with a
 * non-empty range, chunk_pairs == 0, misaligned d_ws), NW_ERANGE (scores do
 * not fit int8), NW_ESTOPPED (fn returned non-zero), NW_EDEVICE. */
int nw_export_triangle(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, uint64_t chunk_pairs,
                       void *d_ws, void *h_buf, nw_chunk_fn fn, void *user, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Threshold edges (graph export).  Section 5 slices the word graph by edge
 * weight before drawing it: raw alignment scores, or scores normalised by the
 * longer word, weight(i, j) = 100 * score(i, j) / max(len i, len j).
 * ------------------------------------------------------------------------- */

typedef enum { NW_EDGE_RAW = 0, NW_EDGE_NORMALISED = 1 } nw_edge_mode;

/* A closed slice of edge weights.  NW_EDGE_RAW: lo <= score <= hi (den is
 * ignored).  NW_EDGE_NORMALISED: lo/den <= weight <= hi/den, decided exactly
 * in integers as lo*m <= 100*score*den <= hi*m, m = max(len i, len j, 1)
 * (a pair of two empty words has weight 0).  den in 1..1000000 lets a slice
 * end between integers (200/3 is lo = hi = 200, den = 3). */
typedef struct {
    int32_t mode;
    int32_t lo, hi;
    int32_t den;
} nw_edge_filter;

/* Every unordered pair (i, j), i < j, with pair index in [idx_begin, idx_end)
 * (the row-major order of nw_all_pairs_scores) whose weight lies in the slice
 * *f is appended as (d_i[q], d_j[q], d_score[q]) = (i, j, score(i, j)),
 * q = 0, 1, ...  in no particular order (one run may order the edges
 * differently from the next; the set is exact).  *d_count (device uint64,
 * set by this call) receives the number of pairs that passed; when it exceeds
 * cap only cap of them are stored and the caller repeats with a larger cap
 * or a smaller index range.  d_i, d_j (int32) and d_score (int16) hold cap
 * entries each (they may be NULL when cap == 0, to count only).  Enqueued
 * on hip_stream; the results are valid once it has synchronised.
 * Errors: NW_EINVAL (NULL vocab, filter or d_count, d_count not 8-byte or
 * the arrays not naturally aligned, mode not one of nw_edge_mode, lo > hi,
 * den outside 1..1000000 for the normalised mode, a range outside
 * [0, n(n-1)/2], an asymmetric similarity), NW_EDEVICE. */
int nw_all_pairs_edges(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, const nw_edge_filter *f,
                       int32_t *d_i, int32_t *d_j, int16_t *d_score, uint64_t cap, uint64_t *d_count,
                       void *hip_stream);


/* ---------------------------------------------------------------------------
 * Neighbour lists.  A neighbour of word i is ranked by (score descending,
 * index ascending); identical words at different indices are distinct
 * neighbours.  Lists shorter than k are padded with (INT16_MIN, -1).
 * ------------------------------------------------------------------------- */

/* Workspace bytes nw_all_pairs_topk needs for this dictionary and k. */
int nw_topk_workspace_bytes(const nw_vocab *v, uint32_t k, uint64_t *bytes);

/* For every word i, its k best neighbours over all j != i (the self-loops the
 * paper leaves out of the adjacency matrix, Section 4.1, are excluded here
 * too): d_score[i*k + r] (int16) and d_index[i*k + r] (int32), r = 0..k-1.
 * If d_hist != NULL it receives hi-lo+1 uint64 counts, bin b = number of
 * unordered pairs {i, j} with score lo + b (bounds from nw_score_bounds): the
 * histogram of raw edge weights of Section 5.  Every unordered pair is scored
 * once.  d_ws: nw_topk_workspace_bytes() bytes, 256-byte aligned, caller-owned.
 * Synchronous: returns once the results are complete on hip_stream.  It has
 * to wait: a word's candidates are gathered into a list of fixed capacity,
 * and the few words whose list overflowed are recomputed exactly by a second
 * pass whose size (the number of such words and their ids) only the device
 * knows after the main pass.  nw_all_pairs_topk = nw_all_pairs_topk_async
 * followed by nw_topk_finish.
 * Errors: NW_EINVAL (k outside 1..63, asymmetric similarity, words longer
 * than 48 symbols, NULL or misaligned buffers, a capturing stream), NW_ENOMEM
 * (workspace too small), NW_EDEVICE. */
int nw_all_pairs_topk(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, uint64_t *d_hist,
                      void *d_ws, uint64_t ws_bytes, void *hip_stream);

/* Enqueue-only form: the threshold pre-pass, the main pass (histogram
 * included) and the selection are enqueued on hip_stream and the call
 * returns.  Once the stream has synchronised, d_hist is complete and every
 * list is exact except those of words whose candidate list overflowed;
 * nw_topk_finish, called next with the same dictionary, k, outputs and
 * workspace, recomputes those and must precede any use of the lists.  One
 * pass per dictionary may be pending at a time.  Same arguments and errors
 * as nw_all_pairs_topk. */
int nw_all_pairs_topk_async(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, uint64_t *d_hist,
                            void *d_ws, uint64_t ws_bytes, void *hip_stream);

/* Complete the pass nw_all_pairs_topk_async enqueued: waits for hip_stream,
 * reads the overflow count, recomputes the overflowed words' lists exactly
 * (blocking) and records the phase times.  NW_EINVAL if no pass is pending
 * on this dictionary; otherwise the errors of nw_all_pairs_topk. */
int nw_topk_finish(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, void *d_ws, uint64_t ws_bytes,
                   void *hip_stream);

/* GPU time of the three phases of the last completed nw_all_pairs_topk call
 * on this dictionary, from HIP events recorded on its stream: the probe
 * threshold pre-pass, the all-pairs main pass, and the per-word selection
 * (milliseconds; any pointer may be NULL). */
int nw_topk_phase_times(const nw_vocab *v, float *prepass_ms, float *main_ms, float *select_ms);

/* Number of words whose candidate list overflowed in the last completed
 * nw_all_pairs_topk call on this dictionary and were recomputed exactly
 * (their lists are exact either way). */
int nw_topk_overflow_words(const nw_vocab *v, uint32_t *words);

/* Workspace bytes nw_query needs for n_q query words (q_symbols is unused). */
int nw_query_workspace_bytes(const nw_vocab *v, uint64_t n_q, uint64_t q_symbols, uint32_t k, uint64_t *bytes);

/* For every query word q (host arrays in the same format as the dictionary),
 * its k best dictionary neighbours over all dictionary words d (no
 * self-exclusion), A = the query word: d_score[q*k + r], d_index[q*k + r].
 * The similar-word lookup the paper envisions (Section 6).  Enqueued on
 * hip_stream; the host arrays may be reused when the call returns (the
 * library's host image of the batch is released by a host callback on the
 * stream once its copy is done, which is why the call refuses a capturing
 * stream).
 * Errors: NW_EINVAL (k outside 1..64, bad query words, a capturing stream),
 * NW_ERANGE (query scores could leave int16), NW_ENOMEM (workspace too
 * small). */
int nw_query(const nw_vocab *v, const uint8_t *h_q_symbols, const uint64_t *h_q_offsets, uint64_t n_q, uint32_t k,
             int16_t *d_score, int32_t *d_index, void *d_ws, uint64_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): nw_query without a workspace
 * argument.  Same results, arguments and errors as nw_query for the same
 * queries and k, but the query workspace is a fixed 4 MiB device array of the
 * library (one per device, kept until the process ends), so at most 256
 * queries per call (NW_EINVAL beyond); the host image is built on the stack
 * and uploaded as kernel arguments, so nothing is allocated on the device or
 * the host, and the host arrays may be reused when the call returns.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (two streams, two threads) race and must be serialised by the
 * caller. */
int nw_query_noalloc(const nw_vocab *v, const uint8_t *h_q_symbols, const uint64_t *h_q_offsets, uint64_t n_q,
                     uint32_t k, int16_t *d_score, int32_t *d_index, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Query server: continuous batching over a resident dictionary, admitted by
 * memory.  A scheduler thread admits the oldest waiting queries (up to
 * max_batch) into any free slot; each slot has its own stream and pinned
 * buffers, so batches overlap on the device and requests arriving meanwhile
 * start as soon as a slot and memory free up.  The device workspace is a pool:
 * a batch of q queries reserves the bytes its own query workspace and results
 * need and returns them on completion; a batch is shrunk to what the largest
 * free range holds, and when not even one query fits, admission waits for a
 * running batch (back-pressure).  A query's result is the one nw_query gives
 * for it alone, whatever batch or memory it ran in.  Serving is the online
 * similar-word lookup the paper envisions (Section 6).
 * ------------------------------------------------------------------------- */
typedef struct nw_server nw_server;

/* Device workspace bytes at which no admission ever waits for memory:
 * num_slots times the largest batch (of 1..max_batch queries).  k 1..64,
 * max_batch 1..4096, num_slots 1..16. */
int nw_server_workspace_bytes(const nw_vocab *v, uint32_t k, uint32_t max_batch, uint32_t num_slots,
                              uint64_t *bytes);

/* The smallest workspace a server accepts: one batch of one query. */
int nw_server_min_workspace_bytes(const nw_vocab *v, uint32_t k, uint64_t *bytes);

/* Start a server.  d_ws (caller-owned, 256-byte aligned, ws_bytes between
 * nw_server_min_workspace_bytes and nw_server_workspace_bytes; more is not
 * used) is the memory pool; it must stay valid, like v, until
 * nw_server_destroy returns.  The server creates its own streams, events and
 * pinned host buffers.  Errors: NW_EINVAL, NW_ENOMEM (ws_bytes below the
 * minimum), NW_EDEVICE. */
int nw_server_create(const nw_vocab *v, uint32_t k, uint32_t max_batch, uint32_t num_slots, void *d_ws,
                     uint64_t ws_bytes, nw_server **out);

/* Queue one query word (len symbols, copied).  tag is returned with the
 * result; t_arrival_ns (nw_clock_ns() time base, 0 = now) is the time the
 * latency is measured from.  Thread-safe. */
int nw_server_submit(nw_server *s, const uint8_t *h_symbols, uint32_t len, uint64_t tag, int64_t t_arrival_ns);

/* Collect up to max_results finished queries, waiting up to timeout_us for
 * the first: tags[r], scores[r*k ..], indices[r*k ..], latency_ns[r]
 * (completion - arrival).  *n_out receives the count.  Any output array may
 * be NULL. */
int nw_server_poll(nw_server *s, uint32_t max_results, int32_t timeout_us, uint64_t *tags, int16_t *scores,
                   int32_t *indices, int64_t *latency_ns, uint32_t *n_out);

/* Open-loop replay: submit query q at arrival_s[q] seconds after the start
 * (from a submitter thread), collect every result into scores[q*k ..],
 * indices[q*k ..] and latency_s[q] (completion - scheduled arrival). */
int nw_server_replay(nw_server *s, const uint8_t *h_symbols, const uint64_t *h_offsets, uint64_t n_q,
                     const double *arrival_s, int16_t *scores, int32_t *indices, double *latency_s);

/* Batches and queries completed so far. */
int nw_server_stats(nw_server *s, uint64_t *batches, uint64_t *queries);

/* Memory admission so far: the pool size in use, the most bytes reserved at
 * once, and how many admitted batches had waited or were shrunk because the
 * pool was short.  Any pointer may be NULL. */
int nw_server_memory_stats(nw_server *s, uint64_t *pool_bytes, uint64_t *peak_bytes, uint64_t *waits);

/* Test hook: the next batch the scheduler admits fails on the host before
 * anything of it is enqueued, as a failed launch would.  The server then
 * admits nothing more: queued queries are dropped, submit and poll return
 * NW_EDEVICE, and nw_server_destroy still returns once the batches in flight
 * have drained. */
int nw_server_inject_failure(nw_server *s);

/* Finish the queued and running batches and release the server (after an
 * error: the running batches only). */
void nw_server_destroy(nw_server *s);

/* The server clock (steady, nanoseconds). */
int64_t nw_clock_ns(void);

/* ---------------------------------------------------------------------------
 * Batched form, planned: the triangles of many dictionaries (each with its own
 * words; every dictionary symmetric) in one graph-captured sequence of
 * launches.  nw_batch_create plans once and nw_batch_run replays; together
 * they take the place of the one-call nw_all_pairs_scores_batched above when
 * the same dictionaries are scored repeatedly (the persistent form needs a
 * workspace for its work queues, which the one-call form does without).
 * Persistent form: work items (dictionary, block pair, row length, chunk of
 * row pairs) are ordered heaviest first inside row-length classes; one
 * persistent kernel per class drains its queue.  Tiled form (class_width 0):
 * every dictionary's per-length tiled launches, as nw_all_pairs_scores issues
 * them, spread over concurrent chains (library streams when eager, chains of
 * kernel nodes in the graph).  nw_batch_autotune times both.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t class_width;     /* 1: one persistent kernel per row length; 8: classes of 8 lengths;
                                 0: no persistent kernels -- every dictionary's per-length tiled
                                 launches, spread over concurrent chains (wg_per_cu and
                                 pairs_per_item unused) */
    uint32_t wg_per_cu;       /* persistent workgroups per compute unit (>= 1) */
    uint32_t pairs_per_item;  /* row pairs per work item (0 = all of a block and length) */
    uint32_t use_graph;       /* 1: capture once into a hipGraph and replay; 0: launch eagerly */
} nw_batch_options;

typedef struct nw_batch nw_batch;

/* Device workspace bytes of a batch plan. */
int nw_batch_workspace_bytes(const nw_vocab *const *v, uint32_t nv, const nw_batch_options *opt, uint64_t *bytes);

/* Plan the batch: dictionary v[i] writes its whole triangle (row-major, as
 * nw_all_pairs_scores with [0, E_i)) to d_outs[i] (dtype dt).  The plan, the
 * dictionaries, the outputs and d_ws must stay valid until nw_batch_destroy.
 * Synchronous (uploads the plan; captures the graph).
 * Errors: NW_EINVAL, NW_ERANGE (bounds do not fit dt), NW_ENOMEM. */
int nw_batch_create(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt,
                    const nw_batch_options *opt, void *d_ws, uint64_t ws_bytes, nw_batch **out);

/* Enqueue one run of the batch on hip_stream (a graph launch when captured). */
int nw_batch_run(nw_batch *b, void *hip_stream);

/* Number of work items and of persistent launches per run. */
int nw_batch_info(const nw_batch *b, uint64_t *items, uint32_t *launches);

void nw_batch_destroy(nw_batch *b);

/* Choose nw_batch_options for this batch by timing candidates on it
 * (the tiled form launched eagerly, then a coordinate search over class
 * width, workgroups per CU and pairs per item with graphs;
 * the workspace must hold the largest candidate plan, see
 * nw_batch_workspace_bytes with pairs_per_item = 16).  With cache_path, a
 * result cached for the same device and workload signature is returned
 * without timing, and new results are appended (one JSON object per line).
 * Overwrites the outputs. */
int nw_batch_autotune(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt, void *d_ws,
                      uint64_t ws_bytes, void *hip_stream, const char *cache_path, nw_batch_options *best,
                      float *best_ms);

/* ---------------------------------------------------------------------------
 * Ego networks on the word graph.  Section 5 reads the graph through
 * ego networks: the words within a few hops (depth 3 in its figures) of a
 * chosen word, in a slice of edge weights.  These calls take an edge list
 * (for instance from nw_all_pairs_edges) as an undirected graph on n words.
 * ------------------------------------------------------------------------- */

/* Workspace bytes of nw_graph_csr for n nodes. */
int nw_graph_workspace_bytes(uint64_t n, uint64_t *bytes);

/* Compressed rows of the undirected graph with the m edges {d_i[e], d_j[e]}:
 * the neighbours of node v are d_adj[d_row_ptr[v] .. d_row_ptr[v+1]), each
 * edge listed from both ends (a self-loop twice at its node, a repeated edge
 * as often as it is given), in no particular order within a row.
 * d_row_ptr: n+1 int64; d_adj: 2m int32; d_ws: nw_graph_workspace_bytes,
 * 256-byte aligned.  All device memory, caller-owned.  Synchronous (it reads
 * back the endpoint check).
 * Errors: NW_EINVAL (n >= 2^31, NULL or misaligned arguments, an endpoint
 * outside [0, n)), NW_ENOMEM (ws_bytes too small), NW_EDEVICE. */
int nw_graph_csr(uint64_t n, const int32_t *d_i, const int32_t *d_j, uint64_t m, int64_t *d_row_ptr, int32_t *d_adj,
                 void *d_ws, uint64_t ws_bytes, void *hip_stream);

/* Hop distances from a seed set, breadth first, up to `depth` hops:
 * d_dist[v] (int32, n entries, device) = the fewest edges on a path from any
 * seed to v if that is <= depth (0 for the seeds), else -1.  The nodes with
 * d_dist >= 0 are the ego network of the seeds.  h_seeds: host array of
 * n_seeds node ids (repeats allowed).  Enqueued on hip_stream.
 * Errors: NW_EINVAL (NULL arguments, n >= 2^31, a seed outside [0, n),
 * depth > 1000000), NW_EDEVICE. */
int nw_ego_network(uint64_t n, const int64_t *d_row_ptr, const int32_t *d_adj, const int32_t *h_seeds,
                   uint32_t n_seeds, uint32_t depth, int32_t *d_dist, void *hip_stream);

/* Issue-rate microbenchmark of the DP's instruction pair (one packed add and
 * one packed three-input max per two cells): `blocks` workgroups of 256
 * threads each issue trips x 64 packed instructions in eight independent
 * chains per lane, touching no memory.  Enqueued on hip_stream; the caller
 * times it (events on that stream).  *lane_instructions receives the number
 * of lane-instructions the launch issues, so instructions per second is the
 * packed issue rate the chip sustains at its running clock, and twice that
 * the 16-bit operation rate (two halves per instruction): the measured
 * counterpart of the nominal 256 CUs x 64 lanes x clock.  Errors: NW_EINVAL
 * (blocks or trips 0, NULL out), NW_EDEVICE. */
int nw_packed_issue_rate(uint32_t blocks, uint32_t trips, uint64_t *lane_instructions, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* NW_H */
