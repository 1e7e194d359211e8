// Launchers of the screening, feature-creation, residual and top-m kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sis {

struct ScoreArgs {
    const double *X;       // stored features (n x P) or children (n x Mc)
    int64_t n, Mc;
    const int32_t *pairs;  // [P][2] child indices (created features), else null
    int64_t P;             // features or candidates to score
    const int64_t *off;    // device task offsets [T+1]
    int T;
    const double *Rc;      // centred residuals, residual_width(nres) rows of stride ldr (zero-padded)
    int64_t ldr;
    const double *Rsum;    // [T][residual_width(nres)] task sums of the centred residuals (zero-padded)
    const double *Ctot;    // [nres] total sum of squares of each residual
    int nres;
    double lower, upper;   // value rules (created features)
    double *scores;
    uint8_t *valid;        // may be null
};

struct FcArgs {
    const double *X;
    int64_t n, Mc;
    const int32_t *pairs;
    int64_t P;
    double lower, upper;
    double *out;  // may be null
    uint8_t *valid;
};

constexpr int OP_STORED_FEATURES = -1;

bool op_known(int op);
int launch_score(int op, const ScoreArgs &a, hipStream_t st);  // op = OP_STORED_FEATURES for stored columns
int launch_fc(int op, const FcArgs &a, hipStream_t st);
// Residuals nres x n are centred per task into Rc (residual_width(nres) rows
// of stride residual_stride(n), padding zero); ctask[r * T + t] gets their
// per-task sums of squares, ctot[r] the totals, rsum[t * width + r] the task
// sums of Rc (zero for r >= nres).
int launch_centre(const double *R, int64_t n, const int64_t *off, int T, int nres, double *Rc, double *ctask,
                  double *ctot, double *rsum, hipStream_t st);
int residual_width(int nres);        // nres rounded up to 1, 2, 4, 8, 10 or 16
int64_t residual_stride(int64_t n);  // row stride of the centred residuals
int launch_residuals(const double *F, const double *y, int64_t n, const int64_t *off, int T, const int32_t *idx,
                     const double *coef, int r, int D, double *R, hipStream_t st);
size_t topm_ws_bytes(int64_t M, int m);
// count_dev receives the device address of the number selected
int launch_topm(const double *sc, int64_t M, int m, int64_t *out_idx, double *out_sc, void *ws, hipStream_t st,
                uint32_t **count_dev);
int launch_mask(const int32_t *sel, int64_t ns, double *scores, hipStream_t st);
int launch_gather(const double *X, int64_t n, const int32_t *sel, int64_t first, int64_t count, double *Fs,
                  hipStream_t st);
int launch_narrow(const int64_t *in, int64_t m, int32_t *out, hipStream_t st);

}  // namespace sis
