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
 *   - orc_score: Algorithm 1 ("Needleman-Wunsch", Section 2) step by step, with
 *     the full (len(A)+1) x (len(B)+1) score matrix held in int32.
 *   - orc_triangle: the upper triangle of the adjacency matrix traversed in
 *     row-major order (0,1),(0,2),...,(n-2,n-1) (Section 4.1), with
 *     A = word i (row) and B = word j (column).
 *   - orc_topk_rows / orc_query: for each word, score it against every other
 *     word (every dictionary word for a query), sort all results by
 *     (score descending, index ascending) and keep the first k.  Not in the
 *     paper; this is the plain definition of a per-word neighbour list.
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
/* Algorithm 1 (Section 2).                                                  */
/*   sim[x * alphabet + y] is similarity(x, y) for symbol x of A, y of B.    */
/*   gap is the linear gap penalty p, added once per gap symbol.             */
/*   M must hold (la+1)*(lb+1) int32; cell (i,j) lives at i*(lb+1)+j, which  */
/*   is the paper's row-major layout of the score matrix.                    */
/* ------------------------------------------------------------------------ */
int32_t orc_score(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                  const int32_t *sim, int32_t alphabet, int32_t gap, int32_t *M)
{
    const int64_t W = lb + 1;
    /* first column: scoreMatrix[i][0] = p * i */
    for (int64_t i = 0; i <= la; ++i) M[i * W + 0] = gap * (int32_t)i;
    /* first row: scoreMatrix[0][j] = p * j */
    for (int64_t j = 0; j <= lb; ++j) M[0 * W + j] = gap * (int32_t)j;
    /* nested loops, row-wise, indices from 1 */
    for (int64_t i = 1; i <= la; ++i) {
        for (int64_t j = 1; j <= lb; ++j) {
            int32_t cost = sim[(int64_t)A[i - 1] * alphabet + B[j - 1]];
            int32_t matchScore = M[(i - 1) * W + (j - 1)] + cost;
            int32_t deleteScore = M[(i - 1) * W + j] + gap;
            int32_t insertScore = M[i * W + (j - 1)] + gap;
            int32_t best = matchScore;
            if (deleteScore > best) best = deleteScore;
            if (insertScore > best) best = insertScore;
            M[i * W + j] = best;
        }
    }
    /* the bottom-right field holds the optimal score */
    return M[la * W + lb];
}

/* Convenience wrapper that allocates its own matrix. */
int32_t orc_score1(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                   const int32_t *sim, int32_t alphabet, int32_t gap)
{
    int32_t *M = (int32_t *)malloc(sizeof(int32_t) * (size_t)((la + 1) * (lb + 1)));
    if (!M) return INT32_MIN;
    int32_t s = orc_score(A, la, B, lb, sim, alphabet, gap, M);
    free(M);
    return s;
}

/* Full score matrix for one pair (for checking worked examples). */
void orc_matrix(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
                const int32_t *sim, int32_t alphabet, int32_t gap, int32_t *M)
{
    (void)orc_score(A, la, B, lb, sim, alphabet, gap, M);
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

/* (score descending, index ascending) */
static int entry_cmp(const void *x, const void *y)
{
    const entry_t *a = (const entry_t *)x, *b = (const entry_t *)y;
    if (a->score != b->score) return a->score > b->score ? -1 : 1;
    if (a->index != b->index) return a->index < b->index ? -1 : 1;
    return 0;
}

enum { JOB_TRIANGLE = 1, JOB_PAIRS = 2, JOB_TOPK = 3, JOB_QUERY = 4 };

static void *worker(void *arg)
{
    job_t *J = (job_t *)arg;
    int64_t L = J->max_len + 1;
    int32_t *M = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L * L));
    entry_t *all = NULL;
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
        all = (entry_t *)malloc(sizeof(entry_t) * (size_t)(J->n > 0 ? J->n : 1));
        if (!all) { J->failed = 1; free(M); return NULL; }
        for (int64_t t = J->tid; t < rows; t += J->nthreads) {
            int64_t i = J->kind == JOB_TOPK ? J->r0 + t : t;
            int64_t la; const uint8_t *A;
            if (J->kind == JOB_TOPK) A = word_ptr(J->sym, J->off, i, &la);
            else A = word_ptr(J->qsym, J->qoff, i, &la);
            int64_t cnt = 0;
            for (int64_t j = 0; j < J->n; ++j) {
                if (J->kind == JOB_TOPK && j == i) continue;   /* no self-loops */
                int64_t lb; const uint8_t *B = word_ptr(J->sym, J->off, j, &lb);
                int32_t s = orc_score(A, la, B, lb, J->sim, J->alphabet, J->gap, M);
                all[cnt].score = s; all[cnt].index = (int32_t)j; ++cnt;
                if (J->hist && J->kind == JOB_TOPK && j > i) {
                    int64_t b = (int64_t)s - J->hist_lo;
                    if (b >= 0 && b < J->hist_nbins) J->hist[b] += 1;
                }
            }
            qsort(all, (size_t)cnt, sizeof(entry_t), entry_cmp);
            for (int32_t r = 0; r < J->k; ++r) {
                int64_t o = t * (int64_t)J->k + r;
                if (r < cnt) { J->score_out[o] = all[r].score; J->index_out[o] = all[r].index; }
                else { J->score_out[o] = INT16_MIN; J->index_out[o] = -1; }
            }
        }
    }
    free(all);
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
