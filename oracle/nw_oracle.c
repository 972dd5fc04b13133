/*
 * nw_oracle.c -- plain CPU oracle for all-pairs Needleman-Wunsch scoring.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 *
 * Everything here is written to be checked by eye against the paper
 * (Plein, "Parallel Needleman-Wunsch on CUDA to measure word similarity based
 * on phonetic transcriptions", 2025):
 *
 *   - orc_score: the global-alignment score of Section 2 from its prefix
 *     recurrence (the table Algorithm 1 fills), one int32 row at a time;
 *     orc_matrix returns the whole table for the worked examples.
 *   - orc_triangle: the upper triangle of the adjacency matrix traversed in
 *     row-major order (0,1),(0,2),...,(n-2,n-1) (Section 4.1), with
 *     A = word i (row) and B = word j (column).
 *   - orc_topk_rows / orc_query: for each word, score it against every other
 *     word (every dictionary word for a query) and keep the k first under the
 *     order (score descending, index ascending), offered one by one to a
 *     sorted list of at most k entries.  Not in the paper; this is the plain
 *     definition of a per-word neighbour list.
 *   - histogram: a count of unordered pairs (i < j) per integer score.
 *
 * Threads (POSIX) only split rows, like the paper's Rayon loop over the outer
 * word (Section 4.1); every thread writes disjoint output slots.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* The score of one pair (Section 2).                                        */
/*                                                                           */
/* V(i, j) is the best score of a global alignment of the first i symbols   */
/* of A with the first j symbols of B.  The last column of such an          */
/* alignment pairs A_i with B_j, or sets A_i against a gap, or B_j against  */
/* a gap, so                                                                 */
/*   V(i, 0) = i p,   V(0, j) = j p,                                         */
/*   V(i, j) = max(V(i-1, j-1) + sim(A_i, B_j), V(i-1, j) + p, V(i, j-1) + p) */
/* and score(A, B) = V(len A, len B): the table Algorithm 1 fills.           */
/*   sim[x * alphabet + y] is the similarity of symbol x of A and y of B;    */
/*   gap is the linear penalty p, added once per gap symbol.                 */
/*                                                                           */
/* Only one row of V is kept: `line` (lb+1 int32) holds V(i-1, .) before     */
/* row i is computed over it, left to right.  When `table` is non-NULL,      */
/* every finished row i is also copied to table[i*(lb+1) ..], which gives    */
/* the whole (la+1) x (lb+1) table in row-major order.                       */
/* ------------------------------------------------------------------------ */
static int32_t prefix_scores(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                             const int32_t *sim, int32_t alphabet, int32_t gap,
                             int32_t *line, int32_t *table)
{
    const size_t row_bytes = sizeof(int32_t) * (size_t)(lb + 1);
    for (int64_t j = 0; j <= lb; ++j) line[j] = (int32_t)j * gap;
    if (table) memcpy(table, line, row_bytes);
    for (int64_t i = 1; i <= la; ++i) {
        int32_t corner = line[0];              /* V(i-1, j-1) for j = 1 */
        int32_t left = (int32_t)i * gap;       /* V(i, j-1) for j = 1 */
        line[0] = left;
        for (int64_t j = 1; j <= lb; ++j) {
            const int32_t above = line[j];     /* V(i-1, j) */
            int32_t v = corner + sim[(int64_t)A[i - 1] * alphabet + B[j - 1]];
            const int32_t a_gapped = above + gap;
            const int32_t b_gapped = left + gap;
            if (a_gapped > v) v = a_gapped;
            if (b_gapped > v) v = b_gapped;
            line[j] = v;
            corner = above;
            left = v;
        }
        if (table) memcpy(table + i * (lb + 1), line, row_bytes);
    }
    return line[lb];
}

/* score(A, B); `line` needs lb+1 int32. */
int32_t orc_score(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                  const int32_t *sim, int32_t alphabet, int32_t gap, int32_t *line)
{
    return prefix_scores(A, la, B, lb, sim, alphabet, gap, line, NULL);
}

/* score(A, B) with its own row buffer. */
int32_t orc_score1(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                   const int32_t *sim, int32_t alphabet, int32_t gap)
{
    int32_t *line = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    if (!line) return INT32_MIN;
    int32_t s = orc_score(A, la, B, lb, sim, alphabet, gap, line);
    free(line);
    return s;
}

/* The whole table V for one pair (to check worked examples cell by cell);
 * M holds (la+1)*(lb+1) int32, row-major. */
void orc_matrix(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                const int32_t *sim, int32_t alphabet, int32_t gap, int32_t *M)
{
    int32_t *line = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    if (!line) return;
    (void)prefix_scores(A, la, B, lb, sim, alphabet, gap, line, M);
    free(line);
}

/* ------------------------------------------------------------------------ */
/* Shared worker plumbing                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *sym;      /* dictionary symbols                    */
    const uint64_t *off;     /* dictionary offsets [n+1]              */
    int64_t n;
    const int32_t *sim;
    int32_t alphabet, gap;
    int64_t max_len;         /* longest word over everything scored   */
    int nthreads, tid;
    /* job-specific */
    int kind;
    uint64_t idx_begin, idx_end;
    int32_t *out;
    const int64_t *pi, *pj;
    int64_t m;
    int32_t k;
    int64_t r0, r1;
    int32_t *score_out, *index_out;
    uint64_t *hist;          /* per-thread private histogram           */
    int32_t hist_lo, hist_nbins;
    const uint8_t *qsym;
    const uint64_t *qoff;
    int64_t nq;
    int failed;
} job_t;

static const uint8_t *word_ptr(const uint8_t *sym, const uint64_t *off, int64_t i, int64_t *len)
{
    *len = (int64_t)(off[i + 1] - off[i]);
    return sym + off[i];
}

/* Number of pairs traversed before row r starts: S_{r-1} of the paper's
 * Eq. for S_r (Section 4.2, "Row & Column"), S_r = (n-1)(r+1) - r(r+1)/2. */
static uint64_t row_start(int64_t n, int64_t r)
{
    /* S_{r-1} = (n-1) r - (r-1) r / 2 */
    return (uint64_t)(n - 1) * (uint64_t)r - (uint64_t)(r - 1) * (uint64_t)r / 2u;
}

typedef struct { int32_t score; int32_t index; } entry_t;

/* Does (s, j) come before entry e in a neighbour list?  Higher score first;
 * on equal scores the lower index first. */
static int comes_before(int32_t s, int32_t j, const entry_t *e)
{
    if (s != e->score) return s > e->score;
    return j < e->index;
}

/* Offer (s, j) to `list`, which holds the *len best entries offered so far in
 * list order (at most k).  A full list keeps (s, j) only if it comes before
 * the last entry, which then drops out. */
static void list_offer(entry_t *list, int32_t k, int32_t *len, int32_t s, int32_t j)
{
    int32_t p;
    if (*len < k) {
        p = (*len)++;
    } else {
        if (k == 0 || !comes_before(s, j, &list[k - 1])) return;
        p = k - 1;
    }
    while (p > 0 && comes_before(s, j, &list[p - 1])) {
        list[p] = list[p - 1];
        --p;
    }
    list[p].score = s;
    list[p].index = j;
}

enum { JOB_TRIANGLE = 1, JOB_PAIRS = 2, JOB_TOPK = 3, JOB_QUERY = 4 };

static void *worker(void *arg)
{
    job_t *J = (job_t *)arg;
    int32_t *M = (int32_t *)malloc(sizeof(int32_t) * (size_t)(J->max_len + 1));
    entry_t *list = NULL;
    if (!M) { J->failed = 1; return NULL; }

    if (J->kind == JOB_TRIANGLE) {
        /* rows i = tid, tid+T, ...; columns j = i+1 .. n-1 */
        for (int64_t i = J->tid; i < J->n - 1; i += J->nthreads) {
            uint64_t s = row_start(J->n, i);
            uint64_t e = s + (uint64_t)(J->n - 1 - i);
            if (e <= J->idx_begin || s >= J->idx_end) continue;
            int64_t la; const uint8_t *A = word_ptr(J->sym, J->off, i, &la);
            for (int64_t j = i + 1; j < J->n; ++j) {
                uint64_t idx = s + (uint64_t)(j - i - 1);
                if (idx < J->idx_begin || idx >= J->idx_end) continue;
                int64_t lb; const uint8_t *B = word_ptr(J->sym, J->off, j, &lb);
                J->out[idx - J->idx_begin] = orc_score(A, la, B, lb, J->sim, J->alphabet, J->gap, M);
            }
        }
    } else if (J->kind == JOB_PAIRS) {
        for (int64_t t = J->tid; t < J->m; t += J->nthreads) {
            int64_t la, lb;
            const uint8_t *A = word_ptr(J->sym, J->off, J->pi[t], &la);
            const uint8_t *B = word_ptr(J->sym, J->off, J->pj[t], &lb);
            J->out[t] = orc_score(A, la, B, lb, J->sim, J->alphabet, J->gap, M);
        }
    } else if (J->kind == JOB_TOPK || J->kind == JOB_QUERY) {
        int64_t rows = J->kind == JOB_TOPK ? J->r1 - J->r0 : J->nq;
        list = (entry_t *)malloc(sizeof(entry_t) * (size_t)(J->k > 0 ? J->k : 1));
        if (!list) { J->failed = 1; free(M); return NULL; }
        for (int64_t t = J->tid; t < rows; t += J->nthreads) {
            int64_t i = J->kind == JOB_TOPK ? J->r0 + t : t;
            int64_t la; const uint8_t *A;
            if (J->kind == JOB_TOPK) A = word_ptr(J->sym, J->off, i, &la);
            else A = word_ptr(J->qsym, J->qoff, i, &la);
            int32_t len = 0;
            for (int64_t j = 0; j < J->n; ++j) {
                if (J->kind == JOB_TOPK && j == i) continue;   /* no self-loops */
                int64_t lb; const uint8_t *B = word_ptr(J->sym, J->off, j, &lb);
                int32_t s = orc_score(A, la, B, lb, J->sim, J->alphabet, J->gap, M);
                list_offer(list, J->k, &len, s, (int32_t)j);
                if (J->hist && J->kind == JOB_TOPK && j > i) {
                    int64_t b = (int64_t)s - J->hist_lo;
                    if (b >= 0 && b < J->hist_nbins) J->hist[b] += 1;
                }
            }
            for (int32_t r = 0; r < J->k; ++r) {
                int64_t o = t * (int64_t)J->k + r;
                if (r < len) { J->score_out[o] = list[r].score; J->index_out[o] = list[r].index; }
                else { J->score_out[o] = INT16_MIN; J->index_out[o] = -1; }
            }
        }
    }
    free(list);
    free(M);
    return NULL;
}

static int64_t max_len_of(const uint64_t *off, int64_t n)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = (int64_t)(off[i + 1] - off[i]);
        if (l > m) m = l;
    }
    return m;
}

static int run_jobs(job_t *base, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t *hists = NULL;
    int failed = 0;
    if (!jobs || !th) { free(jobs); free(th); return -1; }
    if (base->hist) {
        hists = (uint64_t *)calloc((size_t)nthreads * (size_t)base->hist_nbins, sizeof(uint64_t));
        if (!hists) { free(jobs); free(th); return -1; }
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        if (hists) jobs[t].hist = hists + (size_t)t * (size_t)base->hist_nbins;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        failed |= jobs[t].failed;
        if (hists)
            for (int b = 0; b < base->hist_nbins; ++b) base->hist[b] += jobs[t].hist[b];
    }
    free(hists); free(jobs); free(th);
    return failed ? -1 : 0;
}

/* Scores of pairs idx in [idx_begin, idx_end) of the row-major upper
 * triangle (Section 4.1): out[idx - idx_begin] = score(word i, word j). */
int orc_triangle(const uint8_t *sym, const uint64_t *off, int64_t n,
                 const int32_t *sim, int32_t alphabet, int32_t gap,
                 uint64_t idx_begin, uint64_t idx_end, int32_t *out, int nthreads)
{
    job_t J; memset(&J, 0, sizeof J);
    J.sym = sym; J.off = off; J.n = n; J.sim = sim; J.alphabet = alphabet; J.gap = gap;
    J.max_len = max_len_of(off, n); J.kind = JOB_TRIANGLE;
    J.idx_begin = idx_begin; J.idx_end = idx_end; J.out = out;
    return run_jobs(&J, nthreads);
}

/* out[t] = score(word pi[t], word pj[t]) with A = word pi[t]. */
int orc_pairs(const uint8_t *sym, const uint64_t *off, int64_t n,
              const int32_t *sim, int32_t alphabet, int32_t gap,
              const int64_t *pi, const int64_t *pj, int64_t m, int32_t *out, int nthreads)
{
    job_t J; memset(&J, 0, sizeof J);
    J.sym = sym; J.off = off; J.n = n; J.sim = sim; J.alphabet = alphabet; J.gap = gap;
    J.max_len = max_len_of(off, n); J.kind = JOB_PAIRS;
    J.pi = pi; J.pj = pj; J.m = m; J.out = out;
    return run_jobs(&J, nthreads);
}

/* For rows i in [r0, r1): the first k of {(score(i,j), j) : j != i} sorted
 * by (score desc, j asc); missing entries are (INT16_MIN, -1).
 * If hist != NULL, hist[s - hist_lo] also counts pairs (i, j) with j > i. */
int orc_topk_rows(const uint8_t *sym, const uint64_t *off, int64_t n,
                  const int32_t *sim, int32_t alphabet, int32_t gap, int32_t k,
                  int64_t r0, int64_t r1, int32_t *score_out, int32_t *index_out,
                  uint64_t *hist, int32_t hist_lo, int32_t hist_nbins, int nthreads)
{
    job_t J; memset(&J, 0, sizeof J);
    J.sym = sym; J.off = off; J.n = n; J.sim = sim; J.alphabet = alphabet; J.gap = gap;
    J.max_len = max_len_of(off, n); J.kind = JOB_TOPK; J.k = k; J.r0 = r0; J.r1 = r1;
    J.score_out = score_out; J.index_out = index_out;
    J.hist = hist; J.hist_lo = hist_lo; J.hist_nbins = hist_nbins;
    return run_jobs(&J, nthreads);
}

/* For each query q: the first k of {(score(q, d), d) : d in dictionary},
 * sorted by (score desc, d asc); A = the query word; no self-exclusion. */
int orc_query(const uint8_t *sym, const uint64_t *off, int64_t n,
              const int32_t *sim, int32_t alphabet, int32_t gap,
              const uint8_t *qsym, const uint64_t *qoff, int64_t nq, int32_t k,
              int32_t *score_out, int32_t *index_out, int nthreads)
{
    job_t J; memset(&J, 0, sizeof J);
    J.sym = sym; J.off = off; J.n = n; J.sim = sim; J.alphabet = alphabet; J.gap = gap;
    int64_t a = max_len_of(off, n), b = max_len_of(qoff, nq);
    J.max_len = a > b ? a : b; J.kind = JOB_QUERY;
    J.qsym = qsym; J.qoff = qoff; J.nq = nq; J.k = k;
    J.score_out = score_out; J.index_out = index_out;
    return run_jobs(&J, nthreads);
}
