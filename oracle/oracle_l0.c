/*
 * CPU FP64 oracle for the SISSO l0 step.  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the benchmark's CPU-baseline leg call it; the
 * GPU library never does, and the two share no code.
 *
 * What it computes (paper, section "l0-regularization"): for every D-tuple of
 * the m SIS-selected features, the descriptor matrix is assembled in scratch
 * space, factorised by Householder QR, the least-squares fit of the target is
 * taken from the factors, and the tuple is scored by its squared deviation.
 * The paper scores by the mean squared deviation; for a fixed problem that is
 * the sum of squared errors (SSE) divided by the sample count, so this oracle
 * ranks by SSE and reports SSE.
 *
 * Readings of points the paper leaves open:
 *  - the descriptor matrix of task t is X = [1, F_t[:, i_1], ..., F_t[:, i_D]],
 *    i.e. every task gets its own intercept;
 *  - multi-task SISSO (section "Test Cases": same descriptor, different
 *    coefficients per task) scores a tuple by the sum over tasks of SSE_t;
 *  - SSE_t is the squared norm of the tail (rows D+1..n_t-1) of Q^T y, never
 *    |y|^2 minus the head;
 *  - a tuple is rank-deficient, and gets SSE = +inf, when for some feature
 *    column m (in increasing index order) of some task the ratio
 *    R_mm^2 / |x_m - mean(x_m)|^2 is <= 1e-10 (one minus the R^2 of x_m on
 *    the intercept and the earlier columns), or when x_m is constant on the
 *    task to that same 1e-10: |x_m - mean(x_m)|^2 <= 1e-10 |x_m|^2 (one minus
 *    the uncentred R^2 of x_m on the intercept alone).  The second rule keeps
 *    a column that is constant on a task up to rounding, whose centred values
 *    are rounding noise, from passing the first rule on that noise;
 *  - a task with n_t < D+1 rows cannot determine D+1 coefficients: +inf;
 *  - Householder vectors use the LAPACK sign choice v = x + sign(x_1)|x| e_1;
 *  - the top-k is ordered by (SSE ascending, index tuple lexicographically
 *    ascending); tuples are enumerated by plain nested loops in lex order.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -fPIC -shared.
 * No FMA contraction, so every product and sum is rounded as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_D 8
#define ORACLE_RANK_EPS 1e-10

/* Least squares of one task for one tuple.
 * F is n_total x S column-major: column j at F + j*n_total.
 * Rows [r0, r1) belong to the task.  work holds (D+2)*(r1-r0) doubles.
 * On return *sse is SSE_t (or +inf) and, when coef != NULL, coef[0..D] are
 * (intercept, beta_1..beta_D) in the units of F and y (NaN when rank-deficient).
 */
static void task_fit(const double *F, const double *y, int64_t n_total,
                     int64_t r0, int64_t r1, const int32_t *tup, int D,
                     double *work, double *sse, double *coef)
{
    const int64_t nt = r1 - r0;
    const int ncol = D + 1;            /* intercept + D features */
    double *A = work;                  /* nt x ncol, column-major */
    double *b = work + (int64_t)ncol * nt;
    double Rdiag[ORACLE_MAX_D + 1];
    double cnorm2[ORACLE_MAX_D + 1];
    double rnorm2[ORACLE_MAX_D + 1];
    int64_t i;
    int j, c;

    if (coef)
        for (j = 0; j <= D; ++j) coef[j] = NAN;
    if (nt < ncol) { *sse = INFINITY; return; }

    /* 1. assemble the descriptor matrix and right-hand side in scratch */
    for (i = 0; i < nt; ++i) A[i] = 1.0;
    for (j = 0; j < D; ++j) {
        const double *col = F + (int64_t)tup[j] * n_total + r0;
        double *dst = A + (int64_t)(j + 1) * nt;
        double mean = 0.0, s2 = 0.0, r2 = 0.0;
        for (i = 0; i < nt; ++i) { dst[i] = col[i]; mean += col[i]; r2 += col[i] * col[i]; }
        mean /= (double)nt;
        for (i = 0; i < nt; ++i) { double d = col[i] - mean; s2 += d * d; }
        cnorm2[j + 1] = s2;
        rnorm2[j + 1] = r2;
    }
    for (i = 0; i < nt; ++i) b[i] = y[r0 + i];

    /* 2. Householder QR of A, applying each reflector to b as it is formed */
    for (c = 0; c < ncol; ++c) {
        double *x = A + (int64_t)c * nt;
        double norm2 = 0.0, alpha, vtv, x0;
        for (i = c; i < nt; ++i) norm2 += x[i] * x[i];
        if (norm2 == 0.0) { *sse = INFINITY; return; }
        x0 = x[c];
        alpha = (x0 >= 0.0) ? -sqrt(norm2) : sqrt(norm2);   /* R_cc */
        /* v = x - alpha e_c stored in place of x[c..]; v^T v = 2(norm2 - alpha x0) */
        x[c] = x0 - alpha;
        vtv = 2.0 * (norm2 - alpha * x0);
        /* apply H = I - 2 v v^T / (v^T v) to the remaining columns and to b */
        for (j = c + 1; j < ncol; ++j) {
            double *z = A + (int64_t)j * nt;
            double dot = 0.0, f;
            for (i = c; i < nt; ++i) dot += x[i] * z[i];
            f = 2.0 * dot / vtv;
            for (i = c; i < nt; ++i) z[i] -= f * x[i];
        }
        {
            double dot = 0.0, f;
            for (i = c; i < nt; ++i) dot += x[i] * b[i];
            f = 2.0 * dot / vtv;
            for (i = c; i < nt; ++i) b[i] -= f * x[i];
        }
        Rdiag[c] = alpha;
        /* rank test on the feature columns, in increasing index order */
        if (c >= 1) {
            if (cnorm2[c] <= ORACLE_RANK_EPS * rnorm2[c] ||
                (alpha * alpha) / cnorm2[c] <= ORACLE_RANK_EPS) {
                *sse = INFINITY;
                return;
            }
        }
    }

    /* 3. least-squares fit: back substitution R c = (Q^T b)[0..D] */
    if (coef) {
        double x[ORACLE_MAX_D + 1];
        for (j = ncol - 1; j >= 0; --j) {
            double s = b[j];
            for (c = j + 1; c < ncol; ++c) s -= A[(int64_t)c * nt + j] * x[c];
            x[j] = s / Rdiag[j];
        }
        for (j = 0; j <= D; ++j) coef[j] = x[j];
    }

    /* 4. score: squared norm of the residual part of Q^T b */
    {
        double s = 0.0;
        for (i = ncol; i < nt; ++i) s += b[i] * b[i];
        *sse = s;
    }
}

static int64_t max_task_rows(const int64_t *off, int T)
{
    int64_t m = 0;
    int t;
    for (t = 0; t < T; ++t)
        if (off[t + 1] - off[t] > m) m = off[t + 1] - off[t];
    return m;
}

static int check_args(const double *F, const double *y, const int64_t *off,
                      int T, int64_t n, int64_t S, int D)
{
    int t;
    if (!F || !y || !off || T < 1 || n < 1 || S < 1 || D < 1 || D > ORACLE_MAX_D || S < D)
        return -1;
    if (off[0] != 0 || off[T] != n) return -1;
    for (t = 0; t < T; ++t)
        if (off[t + 1] < off[t]) return -1;
    return 0;
}

/* SSE (sum over tasks) of one tuple; coef (optional) gets T*(D+1) values,
 * task-major: [t*(D+1) + 0] is the intercept of task t. Returns 0 or -1. */
int oracle_tuple_sse(const double *F, const double *y, const int64_t *off, int T,
                     int64_t n, int64_t S, int D, const int32_t *tup,
                     double *sse_out, double *coef)
{
    double *work, total = 0.0;
    int t, j;
    if (check_args(F, y, off, T, n, S, D) || !tup || !sse_out) return -1;
    for (j = 0; j < D; ++j) {
        if (tup[j] < 0 || tup[j] >= S) return -1;
        if (j > 0 && tup[j] <= tup[j - 1]) return -1;
    }
    work = (double *)malloc(sizeof(double) * (size_t)(D + 2) * (size_t)max_task_rows(off, T));
    if (!work) return -1;
    for (t = 0; t < T; ++t) {
        double s;
        task_fit(F, y, n, off[t], off[t + 1], tup, D, work, &s, coef ? coef + (int64_t)t * (D + 1) : NULL);
        total += s;
    }
    free(work);
    *sse_out = total;
    return 0;
}

/* ---------------- top-k by (SSE, lex tuple) ---------------- */

typedef struct {
    double sse;
    int32_t tup[ORACLE_MAX_D];
} cand_t;

static int g_cmp_D;  /* tuple length for qsort comparisons (set before use) */

/* <0 if a ranks before b */
static int cand_cmp(const cand_t *a, const cand_t *b, int D)
{
    int j;
    if (a->sse < b->sse) return -1;
    if (a->sse > b->sse) return 1;
    for (j = 0; j < D; ++j) {
        if (a->tup[j] < b->tup[j]) return -1;
        if (a->tup[j] > b->tup[j]) return 1;
    }
    return 0;
}

static int cand_qsort_cmp(const void *x, const void *y)
{
    return cand_cmp((const cand_t *)x, (const cand_t *)y, g_cmp_D);
}

/* bounded max-heap: heap[0] is the worst kept candidate */
typedef struct {
    cand_t *h;
    int size, cap, D;
} heap_t;

static void heap_sift_down(heap_t *hp, int i)
{
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < hp->size && cand_cmp(&hp->h[l], &hp->h[m], hp->D) > 0) m = l;
        if (r < hp->size && cand_cmp(&hp->h[r], &hp->h[m], hp->D) > 0) m = r;
        if (m == i) return;
        { cand_t tmp = hp->h[i]; hp->h[i] = hp->h[m]; hp->h[m] = tmp; }
        i = m;
    }
}

static void heap_offer(heap_t *hp, const cand_t *c)
{
    if (hp->size < hp->cap) {
        int i = hp->size++;
        hp->h[i] = *c;
        while (i > 0) {
            int p = (i - 1) / 2;
            if (cand_cmp(&hp->h[i], &hp->h[p], hp->D) <= 0) break;
            { cand_t tmp = hp->h[i]; hp->h[i] = hp->h[p]; hp->h[p] = tmp; }
            i = p;
        }
        return;
    }
    if (cand_cmp(c, &hp->h[0], hp->D) < 0) {
        hp->h[0] = *c;
        heap_sift_down(hp, 0);
    }
}

/* Enumerate every tuple whose first index lies in [i1_lo, i1_hi) in lex
 * order, score it, and keep the k best by (SSE, lex tuple).  Rank-deficient
 * tuples (SSE = +inf) are never kept.  Outputs are sorted; unused slots get
 * idx = -1 and sse = +inf.  Returns the number of tuples scored, or -1. */
int64_t oracle_l0_topk(const double *F, const double *y, const int64_t *off, int T,
                       int64_t n, int64_t S, int D, int k, int64_t i1_lo, int64_t i1_hi,
                       int32_t *idx_out, double *sse_out, int nthreads)
{
    int64_t total = 0;
    int nth = 1, th, j;
    heap_t *heaps;
    cand_t *all;
    int nall = 0;
    if (check_args(F, y, off, T, n, S, D) || k < 1 || !idx_out || !sse_out) return -1;
    if (i1_lo < 0) i1_lo = 0;
    if (i1_hi > S) i1_hi = S;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    heaps = (heap_t *)calloc((size_t)nth, sizeof(heap_t));
    if (!heaps) return -1;
    for (th = 0; th < nth; ++th) {
        heaps[th].h = (cand_t *)malloc(sizeof(cand_t) * (size_t)k);
        heaps[th].cap = k;
        heaps[th].D = D;
    }

#ifdef _OPENMP
#pragma omp parallel num_threads(nth) reduction(+:total)
#endif
    {
        int me = 0;
        double *work;
        int32_t tup[ORACLE_MAX_D];
        int64_t u, nunits;
#ifdef _OPENMP
        me = omp_get_thread_num();
#endif
        work = (double *)malloc(sizeof(double) * (size_t)(D + 2) * (size_t)max_task_rows(off, T));
        /* A unit of parallel work is one first index (D = 1) or one pair of
         * leading indices (i1, i2) (D >= 2), so that a range of a few first
         * indices still keeps every thread busy.  The scheduling changes no
         * result: every tuple is scored by the same per-tuple QR and the
         * per-thread heaps are merged by (SSE, lex tuple). */
        nunits = D == 1 ? i1_hi - i1_lo : (i1_hi - i1_lo) * S;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (u = 0; u < nunits; ++u) {
            /* nested loops over i_3 < ... < i_D, written as an odometer */
            int m, lead;
            const int64_t i1 = i1_lo + (D == 1 ? u : u / S);
            if (S - i1 < D) continue;
            tup[0] = (int32_t)i1;
            lead = 1;
            if (D >= 2) {
                const int64_t i2 = u % S;
                if (i2 <= i1 || S - i2 < D - 1) continue;
                tup[1] = (int32_t)i2;
                lead = 2;
            }
            for (m = lead; m < D; ++m) tup[m] = tup[m - 1] + 1;
            for (;;) {
                cand_t c;
                int t;
                double s = 0.0;
                for (t = 0; t < T; ++t) {
                    double st;
                    task_fit(F, y, n, off[t], off[t + 1], tup, D, work, &st, NULL);
                    s += st;
                }
                ++total;
                if (s < INFINITY) {
                    c.sse = s;
                    for (m = 0; m < D; ++m) c.tup[m] = tup[m];
                    heap_offer(&heaps[me], &c);
                }
                /* advance the odometer over positions lead..D-1 */
                m = D - 1;
                while (m >= lead && tup[m] == S - D + m) --m;
                if (m < lead) break;
                ++tup[m];
                for (++m; m < D; ++m) tup[m] = tup[m - 1] + 1;
            }
        }
        free(work);
    }

    all = (cand_t *)malloc(sizeof(cand_t) * (size_t)nth * (size_t)k);
    for (th = 0; th < nth; ++th) {
        int i;
        for (i = 0; i < heaps[th].size; ++i) all[nall++] = heaps[th].h[i];
        free(heaps[th].h);
    }
    free(heaps);
    g_cmp_D = D;
    qsort(all, (size_t)nall, sizeof(cand_t), cand_qsort_cmp);
    for (th = 0; th < k; ++th) {
        if (th < nall) {
            sse_out[th] = all[th].sse;
            for (j = 0; j < D; ++j) idx_out[(int64_t)th * D + j] = all[th].tup[j];
        } else {
            sse_out[th] = INFINITY;
            for (j = 0; j < D; ++j) idx_out[(int64_t)th * D + j] = -1;
        }
    }
    free(all);
    return total;
}

/* SSE of every tuple in lex order (for small problems); out has C(S,D)
 * entries.  Returns the number written, or -1. */
int64_t oracle_all_sse(const double *F, const double *y, const int64_t *off, int T,
                       int64_t n, int64_t S, int D, double *out, int64_t out_len)
{
    int32_t tup[ORACLE_MAX_D];
    double *work;
    int64_t cnt = 0;
    int m;
    if (check_args(F, y, off, T, n, S, D) || !out) return -1;
    work = (double *)malloc(sizeof(double) * (size_t)(D + 2) * (size_t)max_task_rows(off, T));
    for (m = 0; m < D; ++m) tup[m] = m;
    for (;;) {
        int t;
        double s = 0.0;
        if (cnt >= out_len) { free(work); return -1; }
        for (t = 0; t < T; ++t) {
            double st;
            task_fit(F, y, n, off[t], off[t + 1], tup, D, work, &st, NULL);
            s += st;
        }
        out[cnt++] = s;
        m = D - 1;
        while (m >= 0 && tup[m] == S - D + m) --m;
        if (m < 0) break;
        ++tup[m];
        for (++m; m < D; ++m) tup[m] = tup[m - 1] + 1;
    }
    free(work);
    return cnt;
}

int oracle_max_d(void) { return ORACLE_MAX_D; }

/* Threads an OpenMP region of the oracle uses by default. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
