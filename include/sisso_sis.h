/*
 * sisso_sis.h -- C ABI of the steps around the l0 search on MI355X
 * (gfx950): sure-independence screening (SIS), feature creation, model
 * residuals, exact top-m selection and the SISSO dimension loop.
 *
 * Paper, section "SISSO": descriptor identification alternates SIS, which
 * picks the features most correlated with the target (first dimension) or
 * with the residuals of the best models of the previous dimension, with an
 * l0 search over every tuple of the selected subspace.  Section "Feature
 * generation and SIS": candidate features are operators applied to child
 * features, kept when their values pass value rules, and screened by the
 * Pearson correlation of eq. (1); the last rung can be generated on the fly
 * during screening instead of being stored.
 *
 * Conventions (as in sisso_l0.h): every function returns SISSO_OK (0) or a
 * negative SISSO_E* code; device pointers are caller-owned HIP device
 * memory; the library allocates no device memory (callers pass workspaces);
 * all device work is enqueued on the given stream (a hipStream_t) and is
 * asynchronous unless stated otherwise; results do not depend on launch
 * configuration or scheduling.  Feature matrices are column-major
 * ("feature-major"): sample i of feature j is X[j * n_total + i].  Rows of a
 * task are contiguous, task t owning rows [task_offsets[t],
 * task_offsets[t+1]).
 */
#ifndef SISSO_SIS_H
#define SISSO_SIS_H

#include <stddef.h>
#include <stdint.h>

#include "sisso_l0.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Operators of feature creation (section "Feature generation and SIS" and
 * the operator list of section "Test Cases").  Binary codes < 16 take two
 * children (a, b); unary codes >= 16 take one (a). */
enum {
    SISSO_OP_ADD = 0,      /* a + b */
    SISSO_OP_SUB = 1,      /* a - b */
    SISSO_OP_MUL = 2,      /* a * b */
    SISSO_OP_DIV = 3,      /* a / b */
    SISSO_OP_ABS_DIFF = 4, /* |a - b| */
    SISSO_OP_EXP = 16,     /* exp(a) */
    SISSO_OP_NEG_EXP = 17, /* exp(-a) */
    SISSO_OP_LOG = 18,     /* ln(a) */
    SISSO_OP_ABS = 19,     /* |a| */
    SISSO_OP_SQRT = 20,    /* sqrt(a) */
    SISSO_OP_CBRT = 21,    /* cube root of a */
    SISSO_OP_SQ = 22,      /* a * a */
    SISSO_OP_CB = 23,      /* (a * a) * a */
    SISSO_OP_INV = 24,     /* 1 / a */
    SISSO_OP_SIN = 25,     /* sin(a) */
    SISSO_OP_COS = 26,     /* cos(a) */
    SISSO_OP_SIX_POW = 27  /* ((a * a) * a) * ((a * a) * a) */
};

#define SISSO_SIS_MAX_RES 16      /* largest number of residuals screened against */
#define SISSO_TOPM_MAX (1 << 20)  /* largest m of sisso_topm */

/* ------------------------------------------------------------------ SIS
 * A screening handle holds the targets a feature is scored against: nres
 * residual vectors (or the target itself, nres = 1), centred per task, and
 * their per-task sums of squares.  Score of a feature x (eq. (1), summed over
 * tasks): for each residual rho,
 *     s_rho(x) = sum_t c_t(rho) r_t(x, rho)^2 / sum_t c_t(rho),
 * r_t the Pearson correlation over task t's rows and c_t(rho) =
 * |rho_t - mean|^2 (a task where rho is identically zero adds nothing); the
 * score is max over rho of s_rho.  For one task and one residual it is r^2,
 * so the order is the order of |r|; in general it is the share of the total
 * variation explained by a one-feature fit with an intercept per task.  A
 * feature that is constant on some task (|x_t - mean|^2 <= 1e-10 |x_t|^2,
 * the l0 search's rule) or has a non-finite value scores NaN and is never
 * selected. */
typedef struct sisso_sis sisso_sis;

typedef struct {
    const double *R;              /* device, n_total x nres, column-major; copied (centred) at create */
    const int64_t *task_offsets;  /* host, T+1 entries; copied at create */
    int64_t n_total;
    int32_t T;                    /* 1..SISSO_MAX_T */
    int32_t nres;                 /* 1..SISSO_SIS_MAX_RES */
    void *workspace;              /* device, >= sisso_sis_workspace_bytes(desc), 256-B aligned */
    size_t workspace_bytes;
    void *stream;
} sisso_sis_desc;

/* Device bytes of a screening handle's workspace (pure); 0 for a bad shape. */
size_t sisso_sis_workspace_bytes(const sisso_sis_desc *desc);
/* Validate, create the handle and enqueue the centring of the residuals.
 * EINVAL for null pointers, offsets not covering [0, n_total) with at least
 * 2 rows per task, T or nres out of range; ENOMEM for a small workspace. */
int32_t sisso_sis_create(const sisso_sis_desc *desc, sisso_sis **out);
void sisso_sis_destroy(sisso_sis *h); /* NULL-safe; frees no caller memory */
const char *sisso_sis_last_error(const sisso_sis *h); /* h == NULL: last failed create */

/* Scores of M stored features X (device, n_total x M) into scores (device
 * double [M]).  HBM-bound: each feature's samples are read from HBM once. */
int32_t sisso_sis_score(sisso_sis *h, const double *X, int64_t M, double *scores);

/* Feature creation fused with screening (the paper's on-the-fly last rung):
 * for candidate p, the new feature v = op(X[:, pairs[2p]], X[:, pairs[2p+1]])
 * (unary ops ignore the second index) is evaluated sample by sample, checked
 * by the value rules of sisso_fc_eval, and scored; its values are never
 * stored.  X: device n_total x Mc children; pairs: device int32 [P][2],
 * indices in [0, Mc); scores: device double [P] (NaN when a value rule
 * fails); valid: device uint8 [P] or NULL.  EINVAL for a bad op, P < 0 or
 * lower > upper; an index out of range gives valid 0 and score NaN. */
int32_t sisso_sis_score_op(sisso_sis *h, int32_t op, const double *X, int64_t Mc, const int32_t *pairs,
                           int64_t P, double lower, double upper, double *scores, uint8_t *valid);

/* --------------------------------------------------------- feature creation
 * Values and validity of op over P candidate child pairs (operators in the
 * outer loop, one call per operator, as the paper's GPU algorithm orders
 * them).  Value rules: every value finite, the largest absolute value within
 * [lower, upper], and the values not all identical.  (The paper's rules on
 * the children, such as no zero in a divisor, only avoid evaluating features
 * that a value rule would reject anyway.)  X: device n_total x Mc; pairs:
 * device int32 [P][2]; out: device n_total x P values, or NULL to keep only
 * the validity; valid: device uint8 [P] (1 = passes).  Asynchronous on
 * stream.  EINVAL for null pointers, a bad op, n_total < 1, P < 0 or
 * lower > upper; an index out of range gives valid 0 (values unspecified). */
int32_t sisso_fc_eval(int32_t op, const double *X, int64_t n_total, int64_t Mc, const int32_t *pairs, int64_t P,
                      double lower, double upper, double *out, uint8_t *valid, void *stream);

/* ------------------------------------------------------------ exact top-m
 * Indices of the m largest finite scores, ordered by (score descending,
 * index ascending); non-finite scores are never selected.  *count (HOST)
 * gets min(m, number of finite scores); out_idx (device int64 [m]) and
 * out_score (device double [m], may be NULL) are filled up to *count.
 * Exact: a radix selection on the 96-bit key (score, complemented index)
 * followed by a rank count, so ties are broken by index and the result is
 * independent of scheduling.  Synchronises the stream (to return *count).
 * EINVAL for null pointers, M < 1, M >= 2^31, m < 1 or m > SISSO_TOPM_MAX;
 * ENOMEM for a small workspace. */
size_t sisso_topm_workspace_bytes(int64_t M, int32_t m);
int32_t sisso_topm(const double *scores, int64_t M, int32_t m, int64_t *out_idx, double *out_score, int32_t *count,
                   void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- residuals
 * Residuals of r models: R[:, q] = y - (alpha_{q,t} + sum_d beta_{q,t,d}
 * F[:, idx[q][d]]) on the rows of each task t.  F: device n_total x S;
 * y: device [n_total]; task_offsets: DEVICE int64 [T+1]; idx: device int32
 * [r][D]; coef: device double [r][T][D+1] ([alpha, beta_1..beta_D] as
 * sisso_l0_topk returns them); R: device n_total x r.  Asynchronous.
 * EINVAL for null pointers or sizes < 1. */
int32_t sisso_residuals(const double *F, const double *y, int64_t n_total, int64_t S, const int64_t *task_offsets,
                        int32_t T, const int32_t *idx, const double *coef, int32_t r, int32_t D, double *R,
                        void *stream);

/* ----------------------------------------------------------- dimension loop
 * SISSO's descriptor identification (section "SISSO"): for D = 1..D_max,
 * screen every candidate feature not yet in the subspace against the target
 * (D = 1) or the residuals of the n_res best models of dimension D - 1, add
 * the m_sis best to the subspace (which lists features in the order they
 * were selected), and search every D-tuple of the subspace (the l0 search of
 * sisso_l0.h, FP64).  Synchronous (returns when done).
 * Outputs (HOST):
 *   subspace [D_max * m_sis]   global feature indices in selection order;
 *   models   [D_max][k][D_max] global indices of dimension D's k best
 *                              models in the first D entries of a row
 *                              (ascending), -1 for unused entries;
 *   sse      [D_max][k]        their SSE (summed over tasks), +inf if unused;
 *   coef     [D_max][k][T][D_max+1] or NULL: intercept and coefficients
 *                              (the first D+1 entries; NaN beyond).
 * Models are ordered by (SSE, lexicographic tuple of subspace positions).
 * Errors: EINVAL for null pointers, D_max outside 1..SISSO_MAX_D, m_sis < 1,
 * M < D_max * m_sis, n_res outside 1..min(k, SISSO_SIS_MAX_RES), k outside
 * 1..SISSO_MAX_K or k > C(m_sis, 1), a task with fewer than D_max + 2 rows;
 * ENOMEM for a small workspace; errors of the l0 calls are passed on.
 * Message: sisso_fit_last_error(). */
typedef struct {
    const double *X;              /* device, n_total x M candidate features */
    const double *y;              /* device, n_total */
    const int64_t *task_offsets;  /* host, T+1 */
    int64_t n_total, M;
    int32_t T, D_max, m_sis, n_res, k;
    void *workspace;              /* device, >= sisso_fit_workspace_bytes(desc), 256-B aligned */
    size_t workspace_bytes;
    void *stream;
} sisso_fit_desc;

size_t sisso_fit_workspace_bytes(const sisso_fit_desc *desc);
int32_t sisso_fit(const sisso_fit_desc *desc, int32_t *subspace, int32_t *models, double *sse, double *coef);
const char *sisso_fit_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SISSO_SIS_H */
