/*
 * sisso_mlp.h -- C ABI of the small network behind the learned proposal of
 * the l0 step (gfx950).  The paper's exhaustive l0 step is the reference;
 * the proposal ranks (D-1)-prefixes by a learned score so that a D-search
 * can evaluate only the extensions of the best-ranked prefixes exactly
 * (sisso_l0_search_list), with exhaustive search as the reference for recall.
 *
 * Network: x (SISSO_MLP_IN features, from sisso_l0_prefix_features) ->
 * h1 = relu(x W1 + b1) -> h2 = relu(h1 W2 + b2) -> y = h2 W3 + b3, hidden
 * width SISSO_MLP_HIDDEN.  Parameters are one float array of
 * SISSO_MLP_NPARAM entries: W1 [IN][H] row-major (input-major), b1 [H],
 * W2 [H][H] (input-major), b2 [H], W3 [H], b3 [1].
 *
 * Conventions: every pointer is DEVICE memory owned by the caller; all work
 * is enqueued on the given hipStream_t (NULL = default stream) and is
 * asynchronous.  Returns SISSO_OK (0) or SISSO_EINVAL (-1) for bad sizes
 * or null pointers, SISSO_EDEVICE (-4) if a launch fails.
 */
#ifndef SISSO_MLP_H
#define SISSO_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SISSO_MLP_IN 8
#define SISSO_MLP_HIDDEN 128
#define SISSO_MLP_NPARAM (SISSO_MLP_IN * SISSO_MLP_HIDDEN + SISSO_MLP_HIDDEN + SISSO_MLP_HIDDEN * SISSO_MLP_HIDDEN + \
                          SISSO_MLP_HIDDEN + SISSO_MLP_HIDDEN + 1)

/* Device bytes of the training workspace for batches of up to n samples
 * (activations, their gradients and per-block partial sums). */
size_t sisso_mlp_workspace_bytes(int64_t n);

/* FP32 forward pass of n samples: out[n].  Keeps the activations in the
 * workspace for a following sisso_mlp_backward on the same x. */
int32_t sisso_mlp_forward(const float *params, const float *x, int64_t n, float *out, void *workspace,
                          size_t workspace_bytes, void *stream);

/* FP32 gradient of the mean squared error L = (1/n) sum (out - target)^2
 * with respect to the parameters, into grad[SISSO_MLP_NPARAM], and L into
 * loss[0].  Needs the activations of a sisso_mlp_forward of the same x, n
 * and parameters in the workspace.  Sums over samples run in a fixed order
 * (per-block partials, then an ordered reduction): deterministic. */
int32_t sisso_mlp_backward(const float *params, const float *x, const float *target, int64_t n, float *grad,
                           float *loss, void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * 1-based step count) on params with first/second moments m, v. */
int32_t sisso_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, void *stream);

/* Inference of n samples with both hidden layers on BF16 MFMA (inputs,
 * W1, W2 and the first layer's activations rounded to BF16, FP32
 * accumulation, output layer in FP32): out[n]. */
int32_t sisso_mlp_infer_bf16(const float *params, const float *x, int64_t n, float *out, void *stream);

/* Top-K selection over n scores (larger is better): writes to out[] the
 * indices of every score at or above the lower edge of the histogram bin
 * (4096 bins over the float ordering) that holds the K-th largest score,
 * so *count >= K; NaN scores are never selected; index order is
 * unspecified, the selected set is not.  workspace: DEVICE, at least
 * sisso_select_workspace_bytes().  Synchronises the stream to return
 * *count (HOST); EINVAL if it exceeds cap (out then holds cap of them). */
size_t sisso_select_workspace_bytes(void);
int32_t sisso_select_top(const float *scores, int64_t n, int64_t K, uint64_t *out, int64_t cap, int64_t *count,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Message of the last failed sisso_select_top / sisso_select_top_noalloc
 * call on this host thread ("" after a successful call). */
const char *sisso_select_last_error(void);

/* sisso_select_top without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same selection, results and errors as
 * sisso_select_top; its scratch (the two level histograms and the cut
 * state, sisso_select_noalloc_scratch_bytes() = 16,640 bytes, independent
 * of n) is a fixed device array of the library that each GPU holds from the
 * first call on it until the process ends.  The call allocates nothing,
 * host or device.  The stream must belong to the current device (EINVAL
 * otherwise).  Every call on one GPU uses that GPU's one array: calls that
 * overlap in time on the same GPU (several host threads, or several streams
 * in flight) race and must be serialised by the caller.  The array keeps
 * the last call's contents; each call clears what it needs before use. */
size_t sisso_select_noalloc_scratch_bytes(void);
int32_t sisso_select_top_noalloc(const float *scores, int64_t n, int64_t K, uint64_t *out, int64_t cap,
                                 int64_t *count, void *stream);

/* Colexicographic unranking of n ranks (DEVICE uint64) into prefix rows
 * (DEVICE int32 [n][m], ascending), 1 <= m <= 3: rank r maps to the r-th
 * m-subset of the non-negative integers ordered by largest element, then
 * recursively (the order of sisso_l0_prefix_features_range). */
int32_t sisso_colex_unrank(int32_t m, const uint64_t *ranks, int64_t n, int32_t *prefixes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SISSO_MLP_H */
