/*
 * sisso_l0.h -- C ABI of an MI355X (gfx950) library for the l0 step of SISSO.
 *
 * The operation (paper, section "l0-regularization"): given the m features
 * that sure-independence screening selected and a target property, score
 * every D-tuple of features by a least-squares fit of the target and keep the
 * best.  The paper scores by the mean squared deviation; here tuples are
 * ranked by the sum of squared errors (SSE), which orders them identically
 * for a fixed problem (MSD = SSE / n_total).  Each task of a multi-task
 * problem (section "Test Cases": one descriptor, coefficients per task) has
 * its own intercept and coefficients, and a tuple's SSE is the sum over tasks.
 *
 * Call sequence:  sisso_l0_workspace_bytes -> sisso_l0_create -> sisso_gram
 *                 -> sisso_l0_search (any number of times, any D <= D_max)
 *                 -> sisso_l0_topk -> sisso_l0_destroy.
 *
 * Conventions
 *  - Every function returns SISSO_OK (0) or a negative SISSO_E* code; no
 *    exception crosses the ABI.  sisso_l0_last_error(h) gives a message.
 *  - Device pointers are HIP device memory owned by the caller.  The library
 *    never allocates device memory: it carves everything it needs out of the
 *    caller's workspace, which must stay alive until sisso_l0_destroy.
 *  - All device work is enqueued on desc.stream (a hipStream_t; NULL = the
 *    default stream) and is asynchronous, except sisso_l0_topk, which
 *    synchronises that stream.  Calls on one handle must not overlap in time
 *    from several host threads.
 *  - Results are deterministic: they do not depend on launch configuration,
 *    scheduling or the order in which the GPU visits tuples.
 */
#ifndef SISSO_L0_H
#define SISSO_L0_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sisso_l0 sisso_l0; /* opaque handle, owned by the library */

enum {
    SISSO_OK = 0,
    SISSO_EINVAL = -1,  /* bad argument (null pointer, size, index, non-finite input) */
    SISSO_ESTATE = -2,  /* call out of order (search before gram, topk before search) */
    SISSO_ENOMEM = -3,  /* caller's workspace smaller than sisso_l0_workspace_bytes */
    SISSO_EDEVICE = -4, /* a HIP runtime call failed; see sisso_l0_last_error */
    SISSO_ENOTSUP = -5  /* a valid request the library does not implement (e.g. D > SISSO_MAX_D) */
};

enum {
    SISSO_PREC_FP64 = 0,       /* Gram, fits and scores in FP64 */
    /* Precision form of the Gram (the search, F^T y, |y|^2 and the re-score
     * stay FP64): every centred column is cut, per chunk of 256 samples, into
     * BF16 slices of small integers with a shared power-of-two scale; the
     * slice cross products run on BF16 MFMA with FP32 accumulation, exact
     * within a chunk, and the chunk sums are scaled and accumulated in FP64.
     * Three slices keep ~23 bits of each centred value.  The error this
     * leaves in the correlation matrix is measured by
     * sisso_l0_precision_report. */
    SISSO_PREC_BF16_COMP = 1,
    /* The same with two FP16 slices of 11 significant bits (22 bits of each
     * centred value) and three slice products instead of six: half the MFMA
     * work of the BF16 form.  FP16 products of these integers reach 2^20, so
     * the FP32 chunk sums round (they are not exact as in the BF16 form);
     * the FP64 accumulation of the chunk sums compensates across chunks.
     * Gram error ~4x that of the BF16 form, reported the same way. */
    SISSO_PREC_FP16_COMP = 2,
    /* FP32 per-tuple solve (the precision option of section
     * "l0-regularization"): the Gram is the FP64 one; the search's solves --
     * prefix factors, records, the incremental last-index terms, the filter
     * and the candidate SSEs -- run in FP32 from the FP64 correlations
     * rounded to FP32, and the 2 (k + 16) best candidates by FP32 SSE are
     * re-scored exactly in FP64 from F, so the returned SSEs are the FP64
     * ones.  FP32 resolves pivot ratios only down to ~1e-5 (below that a
     * tuple counts as rank deficient here, against 1e-10 in FP64), and the
     * filter bound is widened by 1e-5 sum_t c_t.  sisso_l0_precision_report's
     * out[2] gives the FP32 SSEs' error over the returned tuples.  Runs the
     * general search kernels for every D >= 2 (not the FP64 record-table
     * sweeps); D = 1 is solved in FP64. */
    SISSO_PREC_FP32_SOLVE = 3
};

#define SISSO_MAX_D 4      /* largest descriptor dimension compiled in */
#define SISSO_MAX_T 64     /* largest number of tasks */
#define SISSO_MAX_K 496    /* largest top-k */

typedef struct {
    /* F: device, n_total x S, column-major ("feature-major"): sample i of
     * feature j is F[j * n_total + i].  Must be finite. */
    const double *F;
    /* y: device, n_total target values, rows in the same order as F. */
    const double *y;
    /* task_offsets: HOST array of T+1 nondecreasing row offsets with
     * task_offsets[0] = 0 and task_offsets[T] = n_total; task t owns rows
     * [task_offsets[t], task_offsets[t+1]).  Copied at create. */
    const int64_t *task_offsets;
    int64_t n_total;  /* rows (samples) */
    int64_t S;        /* features (columns) */
    int32_t T;        /* tasks, 1..SISSO_MAX_T */
    int32_t D_max;    /* largest D that will be searched, 1..SISSO_MAX_D */
    int32_t k_max;    /* largest k that will be requested, 1..SISSO_MAX_K */
    int32_t precision;/* SISSO_PREC_* */
    void *workspace;  /* device, >= sisso_l0_workspace_bytes(desc) bytes, 256-B aligned */
    size_t workspace_bytes;
    void *stream;     /* hipStream_t on which all work is enqueued */
} sisso_l0_desc;

/* Device bytes the caller must provide in desc->workspace for this problem
 * shape (pure function of n_total, S, T, D_max, k_max and precision; reads
 * no pointer).  With several tasks and D_max >= 3 it includes the filter
 * task's matrix (S^2 doubles) and the D = 3 step queue (24 bytes per sweep
 * step, at most 8 GiB: about 2 GB at S = 5000).  Returns 0 if the shape is
 * invalid. */
size_t sisso_l0_workspace_bytes(const sisso_l0_desc *desc);

/* Validate the descriptor and create a handle in *out.  Errors: EINVAL for
 * null pointers, S < 1, T outside 1..SISSO_MAX_T, offsets not covering
 * [0, n_total) in order, D_max/k_max out of range; ENOMEM if the workspace is
 * too small; ENOTSUP for an unknown precision; EDEVICE if the device cannot
 * be queried.  *out is set only on success. */
int32_t sisso_l0_create(const sisso_l0_desc *desc, sisso_l0 **out);

/* Enqueue the per-task statistics and the Gram precompute: column means,
 * centred cross-products F_t^T F_t (as a correlation matrix), F_t^T y_t and
 * |y_t - mean|^2 for every task.  This replaces the per-tuple assembly of the
 * descriptor matrix: every least-squares system of the search is a
 * sub-matrix of these products.  Non-finite entries of F or y are detected
 * here and reported (EINVAL) by the next sisso_l0_topk. */
int32_t sisso_gram(sisso_l0 *h);

/* Enqueue an exhaustive search over all C(S, D) tuples and keep the k best by
 * (SSE ascending, lexicographic rank ascending).  Rank-deficient tuples (a
 * feature whose 1 - R^2 on the intercept and the earlier features of the
 * tuple is <= 1e-10 in some task, or which is constant on some task to the
 * same 1e-10: |x - mean|^2 <= 1e-10 |x|^2 over the task's rows) are never
 * returned.  Errors: ESTATE before
 * sisso_gram; ENOTSUP for D > D_max or D > SISSO_MAX_D; EINVAL for D < 1,
 * S < D, k < 1, k > k_max, k > C(S, D), or a task with fewer than D + 2 rows. */
int32_t sisso_l0_search(sisso_l0 *h, int32_t D, int32_t k);

/* As sisso_l0_search, restricted to tuples whose lexicographic rank r
 * (0-based, among all C(S, D) tuples of sorted indices) satisfies
 * r0 <= r < r1.  Disjoint ranges merged by (SSE, rank) give the full search,
 * which makes the search resumable and splittable.  EINVAL if r0 >= r1 or
 * r1 > C(S, D). */
int32_t sisso_l0_search_range(sisso_l0 *h, int32_t D, int32_t k, uint64_t r0, uint64_t r1);

/* Batched form (many independent problems, e.g. several SIS subspaces or
 * the problems of a parameter scan; the paper's multi-task case is one
 * handle with T > 1).  A batch holds a HIP graph in which every handle's
 * sisso_gram + sisso_l0_search(D, k) run as one chain, the chains on up to 16
 * concurrent branches.  The graph is captured once by sisso_l0_batch_create
 * and launched by sisso_l0_batch_launch (asynchronous, ordered after prior
 * work on the handles' stream, which all handles must share); afterwards
 * sisso_l0_topk on each handle returns exactly what an unbatched gram +
 * search would.  Errors: EINVAL for null/duplicate handles, handles on
 * different streams, or a (D, k) that some handle rejects (same rules as
 * sisso_l0_search, except that sisso_gram need not have run); EDEVICE if
 * capture fails.  Messages: sisso_l0_batch_last_error(). */
typedef struct sisso_l0_batch sisso_l0_batch;
int32_t sisso_l0_batch_create(sisso_l0 *const *hs, int32_t P, int32_t D, int32_t k, sisso_l0_batch **out);
int32_t sisso_l0_batch_launch(sisso_l0_batch *b);
void sisso_l0_batch_destroy(sisso_l0_batch *b); /* waits for the batch's last launch; NULL-safe */
const char *sisso_l0_batch_last_error(void);
/* One-shot convenience: create, launch, destroy (so it returns after the
 * GPU work has finished). */
int32_t sisso_l0_search_batch(sisso_l0 *const *hs, int32_t P, int32_t D, int32_t k);

/* Prefix-list evaluation (the exact half of a learned proposal; see
 * include/sisso_mlp.h).  prefixes: DEVICE int32 [n][m], each row strictly
 * increasing indices in [0, S).  Every tuple P + {j} (j not in P) is scored
 * exactly like the exhaustive search scores it (normal equations on the
 * correlation matrices, sorted-index Cholesky, the same rank rule), so a
 * tuple reached from several prefixes gets one SSE.  Asynchronous; ESTATE
 * before sisso_gram; EINVAL for bad sizes or null pointers.
 *  - sisso_l0_prefix_best: best[p] (DEVICE double [n]) = min over j of
 *    SSE(P + {j}), +inf if no extension is full rank, NaN for a malformed
 *    row.  1 <= m <= SISSO_MAX_D - 1 (ENOTSUP above).  Exhaustive over the
 *    extensions, so a list of all m-subsets gives per-prefix minima of an
 *    exhaustive (m+1)-search.
 *  - sisso_l0_prefix_features: feat (DEVICE float [n][8]) = R^2 of P's own
 *    fit, max/min/mean squared correlation with y of P's features, max/mean
 *    |G| among them, R^2 minus the best single squared correlation, 1/m.
 *    Malformed rows give NaN.  1 <= m <= SISSO_MAX_D.
 *  - sisso_l0_search_list: the k best distinct D-tuples among all extensions
 *    of the list (D = m + 1, same rules as sisso_l0_search on D and k),
 *    exactly re-scored and read with sisso_l0_topk; malformed rows are
 *    skipped.  sisso_l0_scored reports n (S - D + 1). */
int32_t sisso_l0_prefix_best(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, double *best);
int32_t sisso_l0_prefix_features(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, float *feat);
int32_t sisso_l0_search_list(sisso_l0 *h, int32_t D, int32_t k, const int32_t *prefixes, int64_t n);
/* Training target of each prefix (the label a learned proposal is fitted
 * to): runs sisso_l0_prefix_best into best (DEVICE double [n]) and then sets
 * target[p] (DEVICE float [n]) = -log10(best[p] / c), c = sum over tasks of
 * |y_t - mean(y_t)|^2, with the fraction clamped to [1e-12, 1]; a prefix
 * with no full-rank extension, or a malformed row, gets 0.  Same arguments,
 * rules and errors as sisso_l0_prefix_best, plus EINVAL for a null target. */
int32_t sisso_l0_prefix_target(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, double *best,
                               float *target);
/* Every one-index extension of each listed prefix, for a proposal that
 * scores short prefixes first and only the extensions of the best ones
 * (sub-enumeration): out (DEVICE int32 [n (S - m)][m + 1]) row p (S - m) + t
 * is the sorted tuple P_p + {j}, j the t-th index in {0..S-1} not in P_p,
 * ascending; a malformed row of prefixes (not strictly increasing indices in
 * [0, S)) gives rows of -1, which sisso_l0_prefix_features and
 * sisso_l0_search_list treat as malformed.  1 <= m <= SISSO_MAX_D - 1
 * (ENOTSUP above); asynchronous; ESTATE before sisso_gram, EINVAL for null
 * pointers, a negative count or more than 2^40 output rows. */
int32_t sisso_l0_prefix_extend(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, int32_t *out);
/* Features (as sisso_l0_prefix_features) of the m-subsets of {0..S-1}
 * (1 <= m <= 3) with colexicographic ranks r0 .. r0 + n - 1, i.e. ordered
 * by largest element, then by the rest in the same order; feat: DEVICE
 * float [n][8].  EINVAL if the range exceeds C(S, m). */
int32_t sisso_l0_prefix_features_range(sisso_l0 *h, int32_t m, uint64_t r0, int64_t n, float *feat);

/* Launch tuning.  The persistent search kernel runs on a grid of
 * workgroups (default 1024) whose best size depends on the problem; it
 * changes no arithmetic, so every size gives bit-identical results.  (The
 * paper auto-tunes its launch configuration by timing a predefined set on
 * the first batch of each run, section "l0-regularization".)  sisso_l0_set_search_grid sets it (EINVAL
 * outside 1..2048); sisso_l0_search_grid reads it (0 for NULL).
 * sisso_l0_autotune times the candidates 256, 512, ..., 2048 on a full
 * search of (D, k) (same argument rules as sisso_l0_search), keeps the
 * fastest and writes it to *chosen (may be NULL).  With cache_path (may be
 * NULL) it first looks up, and afterwards stores, the choice in a JSON file
 * keyed by GPU architecture, D, S rounded up to a power of two, T and the
 * precision mode; a cache hit runs nothing.  After a tuning run the handle
 * holds the result of a search of (D, k), as after sisso_l0_search.
 * Synchronises the stream; EINVAL if the cache cannot be written. */
int32_t sisso_l0_set_search_grid(sisso_l0 *h, int32_t workgroups);
int32_t sisso_l0_search_grid(const sisso_l0 *h);
int32_t sisso_l0_autotune(sisso_l0 *h, int32_t D, int32_t k, const char *cache_path, int32_t *chosen);

/* Synchronise the stream and copy the result of the last search to HOST
 * buffers: idx (k*D int32, row-major, ascending indices within a row), sse
 * (k doubles, SSE summed over tasks) and, unless NULL, coef (k*T*(D+1)
 * doubles: for result r and task t, coef[(r*T + t)*(D+1)] is the intercept
 * and the next D entries the coefficients of the tuple's features, in the
 * units of F and y).  Rows beyond the number of full-rank tuples are filled
 * with idx -1, sse +inf, coef NaN.  Errors: ESTATE before a search or for k
 * above the searched k; EINVAL for null idx/sse or non-finite input data;
 * EDEVICE for a HIP error, or if the several-task D = 3 search's step queue
 * overflowed (sized for every sweep step, so it is not expected; the result
 * would be incomplete and is not returned). */
int32_t sisso_l0_topk(sisso_l0 *h, int32_t k, int32_t *idx, double *sse, double *coef);

/* Synchronise the stream and copy task t's precomputed statistics to HOST
 * buffers (any may be NULL): G (S*S doubles, row-major) the correlation
 * matrix of the task's centred columns, G[i][j] = x_ic.x_jc / (|x_ic||x_jc|)
 * with a unit diagonal (0 on the diagonal, and 0 in the row and column, of a
 * column constant on the task as defined at sisso_l0_search); b (S
 * doubles) b_j = x_jc.y_c / |x_jc|; c (1 double) |y_c|^2, where x_c, y_c are
 * the task's columns minus their means.  ESTATE before sisso_gram, EINVAL for
 * t out of range. */
int32_t sisso_gram_read(sisso_l0 *h, int32_t t, double *G, double *b, double *c);

/* Number of tuples the last search scored (C(S, D), or r1 - r0 for a range
 * search), for throughput accounting.  Host-only. */
uint64_t sisso_l0_scored(const sisso_l0 *h);

/* Accuracy report of the precision form, also valid for FP64 (synchronises
 * the stream).  out[0]: largest |G_used - G_fp64| over nsample sampled
 * entries per task (the FP64 value is the centred dot product straight from
 * F, computed here); out[1]: entries compared; out[2]: largest relative
 * difference between the SSE the search ranked by (from G_used) and the
 * exact re-scored SSE over the k results of the last search (0 before a
 * search); out[3]: slices per value (0 for FP64).  ESTATE before
 * sisso_gram; EINVAL for nsample < 1 or a null out. */
int32_t sisso_l0_precision_report(sisso_l0 *h, int32_t nsample, double *out);

/* Gram error of the handle's precision mode (section "l0-regularization"
 * names precision as the method's main accuracy/speed trade-off): the
 * largest |G_used - G_fp64| over 4096 sampled entries per task of the
 * correlation matrices, whose entries lie in [-1, 1], so the absolute error
 * is also the error relative to the unit diagonal.  G_fp64 is the centred
 * dot product recomputed in FP64 straight from F.  Equals out[0] of
 * sisso_l0_precision_report(h, 4096, out).  Synchronises the stream; ESTATE
 * before sisso_gram, EINVAL for null arguments. */
int32_t sisso_gram_error(sisso_l0 *h, double *max_abs_rel);

/* Per-phase timing with HIP events recorded on the handle's stream.
 * sisso_l0_profile(h, 1) turns it on (0 off; off by default).  After a
 * sisso_gram / sisso_l0_search, sisso_l0_phase_ms fills ms[SISSO_NPHASE]
 * (milliseconds of the last run of each phase; 0 if it has not run) and
 * synchronises the stream.  Phases: statistics, Gram, threshold pre-pass,
 * search kernel, merge, exact re-score, final ordering. */
#define SISSO_NPHASE 7
enum {
    SISSO_PHASE_STATS = 0,
    SISSO_PHASE_GRAM = 1,
    SISSO_PHASE_PREPASS = 2,
    SISSO_PHASE_SEARCH = 3,
    SISSO_PHASE_MERGE = 4,
    SISSO_PHASE_RESCORE = 5,
    SISSO_PHASE_FINAL = 6
};
int32_t sisso_l0_profile(sisso_l0 *h, int32_t enable);
int32_t sisso_l0_phase_ms(sisso_l0 *h, double *ms);

/* Diagnostics of the last search (synchronises the stream): out[0] tuples
 * that passed the filter and were offered to a top-k list, out[1] work
 * items, out[2] the bit pattern of the pre-pass SSE bound (+inf if none),
 * out[3] the bit pattern of the final device-wide SSE bound.  ESTATE before
 * a search. */
int32_t sisso_l0_search_stats(sisso_l0 *h, uint64_t *out);

/* Wait for the work enqueued on the handle's stream, then release the
 * handle (NULL-safe).  Does not free caller memory; the workspace may be
 * released once this returns. */
void sisso_l0_destroy(sisso_l0 *h);

/* Message for the last error on h ("" if none); valid until the next call on
 * h.  With h == NULL, the message of the last failed sisso_l0_create. */
const char *sisso_l0_last_error(const sisso_l0 *h);

/* Lexicographic rank <-> tuple (combinatorial number system), host side.
 * rank_of returns UINT64_MAX for an invalid tuple; unrank returns EINVAL for
 * r >= C(S, D). */
uint64_t sisso_l0_rank_of(int64_t S, int32_t D, const int32_t *tuple);
int32_t sisso_l0_unrank(int64_t S, int32_t D, uint64_t r, int32_t *tuple);

#ifdef __cplusplus
}
#endif
#endif /* SISSO_L0_H */
