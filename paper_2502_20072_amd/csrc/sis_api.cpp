// C ABI of screening, feature creation, residuals, top-m and the dimension
// loop: argument checks, workspace carving and the order of launches.  All
// arithmetic happens in the kernels (sis.hip) and the l0 library calls.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/sisso_l0.h"
#include "../../include/sisso_sis.h"
#include "sis.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool offsets_ok(const int64_t *o, int T, int64_t n, int64_t min_rows) {
    if (!o || T < 1 || T > SISSO_MAX_T || o[0] != 0 || o[T] != n) return false;
    for (int t = 0; t < T; ++t)
        if (o[t + 1] - o[t] < min_rows) return false;
    return true;
}

struct SisLayout {
    size_t off, Rc, ctask, ctot, rsum, total;
};

SisLayout sis_layout(int64_t n, int T, int nres) {
    SisLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align256(o + b);
        return at;
    };
    L.off = take((size_t)(T + 1) * sizeof(int64_t));
    L.Rc = take((size_t)sis::residual_stride(n) * sis::residual_width(nres) * sizeof(double));
    L.ctask = take((size_t)nres * T * sizeof(double));
    L.ctot = take((size_t)nres * sizeof(double));
    const int w = sis::residual_width(nres);
    L.rsum = take((size_t)T * w * sizeof(double));
    L.total = o;
    return L;
}

thread_local std::string g_sis_create_err;
thread_local std::string g_fit_err;

}  // namespace

struct sisso_sis {
    int64_t n;
    int T, nres;
    hipStream_t stream;
    int64_t *off;
    double *Rc, *ctask, *ctot, *rsum;
    std::string err;
};

static int32_t sis_fail(sisso_sis *h, int32_t code, const char *msg) {
    if (h) h->err = msg;
    else g_sis_create_err = msg;
    return code;
}

static bool sis_shape_ok(const sisso_sis_desc *d) {
    return d && d->n_total >= 2 && d->T >= 1 && d->T <= SISSO_MAX_T && d->nres >= 1 &&
           d->nres <= SISSO_SIS_MAX_RES;
}

extern "C" size_t sisso_sis_workspace_bytes(const sisso_sis_desc *d) {
    if (!sis_shape_ok(d)) return 0;
    return sis_layout(d->n_total, d->T, d->nres).total;
}

extern "C" int32_t sisso_sis_create(const sisso_sis_desc *d, sisso_sis **out) {
    if (!d || !out) return sis_fail(nullptr, SISSO_EINVAL, "null descriptor or output");
    if (!d->R || !d->task_offsets || !d->workspace) return sis_fail(nullptr, SISSO_EINVAL, "null R, offsets or workspace");
    if (!sis_shape_ok(d)) return sis_fail(nullptr, SISSO_EINVAL, "n_total, T or nres out of range");
    if (!offsets_ok(d->task_offsets, d->T, d->n_total, 2))
        return sis_fail(nullptr, SISSO_EINVAL, "task offsets must span [0, n_total) with >= 2 rows per task");
    if (((uintptr_t)d->workspace & 255) != 0) return sis_fail(nullptr, SISSO_EINVAL, "workspace must be 256-byte aligned");
    const SisLayout L = sis_layout(d->n_total, d->T, d->nres);
    if (d->workspace_bytes < L.total) return sis_fail(nullptr, SISSO_ENOMEM, "workspace smaller than sisso_sis_workspace_bytes");
    sisso_sis *h = new (std::nothrow) sisso_sis();
    if (!h) return sis_fail(nullptr, SISSO_ENOMEM, "host allocation failed");
    char *b = (char *)d->workspace;
    h->n = d->n_total;
    h->T = d->T;
    h->nres = d->nres;
    h->stream = (hipStream_t)d->stream;
    h->off = (int64_t *)(b + L.off);
    h->Rc = (double *)(b + L.Rc);
    h->ctask = (double *)(b + L.ctask);
    h->ctot = (double *)(b + L.ctot);
    h->rsum = (double *)(b + L.rsum);
    if (hipMemcpyAsync(h->off, d->task_offsets, (size_t)(d->T + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        sis::launch_centre(d->R, h->n, h->off, h->T, h->nres, h->Rc, h->ctask, h->ctot, h->rsum,
                           h->stream) != 0 ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        delete h;
        return sis_fail(nullptr, SISSO_EDEVICE, "could not prepare the residuals on the device");
    }
    *out = h;
    return SISSO_OK;
}

extern "C" void sisso_sis_destroy(sisso_sis *h) { delete h; }

extern "C" const char *sisso_sis_last_error(const sisso_sis *h) { return h ? h->err.c_str() : g_sis_create_err.c_str(); }

static sis::ScoreArgs score_args(sisso_sis *h, const double *X, int64_t Mc, const int32_t *pairs, int64_t P,
                                 double lower, double upper, double *scores, uint8_t *valid) {
    sis::ScoreArgs a{};
    a.X = X;
    a.n = h->n;
    a.Mc = Mc;
    a.pairs = pairs;
    a.P = P;
    a.off = h->off;
    a.T = h->T;
    a.Rc = h->Rc;
    a.ldr = sis::residual_stride(h->n);
    a.Rsum = h->rsum;
    a.Ctot = h->ctot;
    a.nres = h->nres;
    a.lower = lower;
    a.upper = upper;
    a.scores = scores;
    a.valid = valid;
    return a;
}

extern "C" int32_t sisso_sis_score(sisso_sis *h, const double *X, int64_t M, double *scores) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (M < 0 || (M > 0 && (!X || !scores))) return sis_fail(h, SISSO_EINVAL, "null pointer or M < 0");
    if (M == 0) return SISSO_OK;
    const sis::ScoreArgs a = score_args(h, X, M, nullptr, M, 0.0, 0.0, scores, nullptr);
    if (sis::launch_score(sis::OP_STORED_FEATURES, a, h->stream))
        return sis_fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_sis_score_op(sisso_sis *h, int32_t op, const double *X, int64_t Mc, const int32_t *pairs,
                                      int64_t P, double lower, double upper, double *scores, uint8_t *valid) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (!sis::op_known(op)) return sis_fail(h, SISSO_EINVAL, "unknown operator");
    if (P < 0 || Mc < 1 || !(lower <= upper)) return sis_fail(h, SISSO_EINVAL, "P < 0, Mc < 1 or lower > upper");
    if (P > 0 && (!X || !pairs || !scores)) return sis_fail(h, SISSO_EINVAL, "null pointer");
    if (P == 0) return SISSO_OK;
    const sis::ScoreArgs a = score_args(h, X, Mc, pairs, P, lower, upper, scores, valid);
    if (sis::launch_score(op, a, h->stream)) return sis_fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_fc_eval(int32_t op, const double *X, int64_t n_total, int64_t Mc, const int32_t *pairs,
                                 int64_t P, double lower, double upper, double *out, uint8_t *valid, void *stream) {
    if (!sis::op_known(op) || n_total < 1 || Mc < 1 || P < 0 || !(lower <= upper)) return SISSO_EINVAL;
    if (P == 0) return SISSO_OK;
    if (!X || !pairs || !valid) return SISSO_EINVAL;
    sis::FcArgs a{X, n_total, Mc, pairs, P, lower, upper, out, valid};
    return sis::launch_fc(op, a, (hipStream_t)stream) ? SISSO_EDEVICE : SISSO_OK;
}

extern "C" size_t sisso_topm_workspace_bytes(int64_t M, int32_t m) {
    if (M < 1 || M >= (1ll << 31) || m < 1 || m > SISSO_TOPM_MAX) return 0;
    return sis::topm_ws_bytes(M, m);
}

extern "C" int32_t sisso_topm(const double *scores, int64_t M, int32_t m, int64_t *out_idx, double *out_score,
                              int32_t *count, void *workspace, size_t workspace_bytes, void *stream) {
    if (!scores || !out_idx || !count || !workspace || M < 1 || M >= (1ll << 31) || m < 1 || m > SISSO_TOPM_MAX)
        return SISSO_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return SISSO_EINVAL;
    if (workspace_bytes < sis::topm_ws_bytes(M, m)) return SISSO_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    uint32_t *cnt_dev = nullptr;
    if (sis::launch_topm(scores, M, m, out_idx, out_score, workspace, st, &cnt_dev)) return SISSO_EDEVICE;
    uint32_t c = 0;
    if (hipMemcpyAsync(&c, cnt_dev, sizeof c, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SISSO_EDEVICE;
    *count = (int32_t)(c < (uint32_t)m ? c : (uint32_t)m);
    return SISSO_OK;
}

extern "C" int32_t sisso_residuals(const double *F, const double *y, int64_t n_total, int64_t S,
                                   const int64_t *task_offsets, int32_t T, const int32_t *idx, const double *coef,
                                   int32_t r, int32_t D, double *R, void *stream) {
    if (!F || !y || !task_offsets || !idx || !coef || !R || n_total < 1 || S < 1 || T < 1 || T > SISSO_MAX_T ||
        r < 1 || r > 65535 || D < 1)
        return SISSO_EINVAL;
    return sis::launch_residuals(F, y, n_total, task_offsets, T, idx, coef, r, D, R, (hipStream_t)stream)
               ? SISSO_EDEVICE
               : SISSO_OK;
}

// ------------------------------------------------------------ dimension loop
namespace {

struct FitLayout {
    size_t off, R, sis, scores, topm, topm_idx, sel, Fs, l0, midx, mcoef, total;
    size_t sis_bytes, topm_bytes, l0_bytes;
};

sisso_l0_desc l0_desc_for(const sisso_fit_desc *d, const double *Fs, int64_t S, int D, void *ws, size_t wsb) {
    sisso_l0_desc q{};
    q.F = Fs;
    q.y = d->y;
    q.task_offsets = d->task_offsets;
    q.n_total = d->n_total;
    q.S = S;
    q.T = d->T;
    q.D_max = D;
    q.k_max = d->k;
    q.precision = SISSO_PREC_FP64;
    q.workspace = ws;
    q.workspace_bytes = wsb;
    q.stream = d->stream;
    return q;
}

bool fit_shape_ok(const sisso_fit_desc *d) {
    if (!d || d->T < 1 || d->T > SISSO_MAX_T || d->D_max < 1 || d->D_max > SISSO_MAX_D || d->m_sis < 1 ||
        d->k < 1 || d->k > SISSO_MAX_K || d->n_res < 1 || d->n_res > SISSO_SIS_MAX_RES || d->n_res > d->k ||
        d->n_total < 2 || d->M < 1 || d->M >= (1ll << 31))
        return false;
    if ((int64_t)d->D_max * d->m_sis > d->M || d->k > d->m_sis) return false;
    return true;
}

FitLayout fit_layout(const sisso_fit_desc *d) {
    FitLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align256(o + b);
        return at;
    };
    const int64_t Smax = (int64_t)d->D_max * d->m_sis;
    const size_t dd = sizeof(double);
    L.off = take((size_t)(d->T + 1) * sizeof(int64_t));
    L.R = take((size_t)d->n_total * d->n_res * dd);
    L.sis_bytes = sis_layout(d->n_total, d->T, d->n_res).total;
    L.sis = take(L.sis_bytes);
    L.scores = take((size_t)d->M * dd);
    L.topm_bytes = sis::topm_ws_bytes(d->M, d->m_sis);
    L.topm = take(L.topm_bytes);
    L.topm_idx = take((size_t)d->m_sis * sizeof(int64_t));
    L.sel = take((size_t)Smax * sizeof(int32_t));
    L.Fs = take((size_t)Smax * d->n_total * dd);
    // dimension D searches a subspace of D * m_sis features with D_max = D
    L.l0_bytes = 0;
    for (int D = 1; D <= d->D_max; ++D) {
        const sisso_l0_desc q = l0_desc_for(d, nullptr, (int64_t)D * d->m_sis, D, nullptr, 0);
        const size_t need = sisso_l0_workspace_bytes(&q);
        if (need == 0) {
            L.l0_bytes = 0;
            break;
        }
        L.l0_bytes = std::max(L.l0_bytes, need);
    }
    L.l0 = take(L.l0_bytes);
    L.midx = take((size_t)d->n_res * d->D_max * sizeof(int32_t));
    L.mcoef = take((size_t)d->n_res * d->T * (d->D_max + 1) * dd);
    L.total = o;
    return L;
}

int32_t fit_fail(int32_t code, const std::string &msg) {
    g_fit_err = msg;
    return code;
}

}  // namespace

extern "C" size_t sisso_fit_workspace_bytes(const sisso_fit_desc *d) {
    if (!fit_shape_ok(d)) return 0;
    const FitLayout L = fit_layout(d);
    return L.l0_bytes ? L.total : 0;
}

extern "C" const char *sisso_fit_last_error(void) { return g_fit_err.c_str(); }

extern "C" int32_t sisso_fit(const sisso_fit_desc *d, int32_t *subspace, int32_t *models, double *sse, double *coef) {
    g_fit_err.clear();
    if (!d || !subspace || !models || !sse) return fit_fail(SISSO_EINVAL, "null descriptor or output");
    if (!d->X || !d->y || !d->task_offsets || !d->workspace) return fit_fail(SISSO_EINVAL, "null X, y, offsets or workspace");
    if (!fit_shape_ok(d)) return fit_fail(SISSO_EINVAL, "sizes out of range (T, D_max, m_sis, n_res, k, M)");
    if (!offsets_ok(d->task_offsets, d->T, d->n_total, d->D_max + 2))
        return fit_fail(SISSO_EINVAL, "task offsets must span [0, n_total) with >= D_max + 2 rows per task");
    if (((uintptr_t)d->workspace & 255) != 0) return fit_fail(SISSO_EINVAL, "workspace must be 256-byte aligned");
    const FitLayout L = fit_layout(d);
    if (!L.l0_bytes) return fit_fail(SISSO_EINVAL, "subspace shape rejected by the l0 search");
    if (d->workspace_bytes < L.total) return fit_fail(SISSO_ENOMEM, "workspace smaller than sisso_fit_workspace_bytes");
    char *b = (char *)d->workspace;
    hipStream_t st = (hipStream_t)d->stream;
    const int64_t n = d->n_total;
    const int T = d->T, Dm = d->D_max, k = d->k, ms = d->m_sis;
    int64_t *off = (int64_t *)(b + L.off);
    double *R = (double *)(b + L.R);
    double *scores = (double *)(b + L.scores);
    int64_t *tidx = (int64_t *)(b + L.topm_idx);
    int32_t *sel = (int32_t *)(b + L.sel);
    double *Fs = (double *)(b + L.Fs);
    int32_t *midx = (int32_t *)(b + L.midx);
    double *mcoef = (double *)(b + L.mcoef);
    for (int D = 0; D < Dm; ++D)
        for (int q = 0; q < k; ++q) {
            sse[(size_t)D * k + q] = INFINITY;
            for (int j = 0; j < Dm; ++j) models[((size_t)D * k + q) * Dm + j] = -1;
            if (coef)
                for (int t = 0; t < T; ++t)
                    for (int j = 0; j <= Dm; ++j) coef[(((size_t)D * k + q) * T + t) * (Dm + 1) + j] = NAN;
        }
    if (hipMemcpyAsync(off, d->task_offsets, (size_t)(T + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return fit_fail(SISSO_EDEVICE, "copying the task offsets failed");
    std::vector<int32_t> sub;  // host copy of the subspace, selection order
    std::vector<int32_t> pidx((size_t)k * Dm);
    std::vector<double> psse(k), pcoef((size_t)k * T * (Dm + 1));
    // the target itself is the first "residual"
    if (hipMemcpyAsync(R, d->y, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fit_fail(SISSO_EDEVICE, "copying y failed");
    int nres = 1;
    for (int D = 1; D <= Dm; ++D) {
        // screening of every candidate against the residuals
        sisso_sis_desc sd{};
        sd.R = R;
        sd.task_offsets = d->task_offsets;
        sd.n_total = n;
        sd.T = T;
        sd.nres = nres;
        sd.workspace = b + L.sis;
        sd.workspace_bytes = L.sis_bytes;
        sd.stream = d->stream;
        sisso_sis *sh = nullptr;
        int32_t rc = sisso_sis_create(&sd, &sh);
        if (rc != SISSO_OK) return fit_fail(rc, std::string("screening: ") + sisso_sis_last_error(nullptr));
        rc = sisso_sis_score(sh, d->X, d->M, scores);
        sisso_sis_destroy(sh);
        if (rc != SISSO_OK) return fit_fail(rc, "screening launch failed");
        if (sis::launch_mask(sel, (int64_t)sub.size(), scores, st)) return fit_fail(SISSO_EDEVICE, "mask launch failed");
        int32_t got = 0;
        rc = sisso_topm(scores, d->M, ms, tidx, nullptr, &got, b + L.topm, L.topm_bytes, d->stream);
        if (rc != SISSO_OK) return fit_fail(rc, "top-m selection failed");
        if (got < ms) return fit_fail(SISSO_EINVAL, "fewer screenable features than m_sis");
        const int64_t first = (int64_t)sub.size();
        if (sis::launch_narrow(tidx, ms, sel + first, st) ||
            sis::launch_gather(d->X, n, sel, first, ms, Fs, st))
            return fit_fail(SISSO_EDEVICE, "subspace gather failed");
        sub.resize(first + ms);
        if (hipMemcpyAsync(sub.data() + first, sel + first, (size_t)ms * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fit_fail(SISSO_EDEVICE, "reading the selection failed");
        // l0 search of every D-tuple of the subspace
        const int64_t S = (int64_t)sub.size();
        const sisso_l0_desc q = l0_desc_for(d, Fs, S, D, b + L.l0, L.l0_bytes);
        sisso_l0 *lh = nullptr;
        rc = sisso_l0_create(&q, &lh);
        if (rc != SISSO_OK) return fit_fail(rc, std::string("l0 create: ") + sisso_l0_last_error(nullptr));
        const uint64_t ntup = [&] {
            uint64_t c = 1;
            for (int j = 0; j < D; ++j) c = c * (uint64_t)(S - j) / (uint64_t)(j + 1);
            return c;
        }();
        const int kk = (uint64_t)k < ntup ? k : (int)ntup;
        rc = sisso_gram(lh);
        if (rc == SISSO_OK) rc = sisso_l0_search(lh, D, kk);
        if (rc == SISSO_OK) rc = sisso_l0_topk(lh, kk, pidx.data(), psse.data(), pcoef.data());
        if (rc != SISSO_OK) {
            const std::string m = std::string("l0: ") + sisso_l0_last_error(lh);
            sisso_l0_destroy(lh);
            return fit_fail(rc, m);
        }
        sisso_l0_destroy(lh);
        int live = 0;
        for (int qq = 0; qq < kk; ++qq) {
            if (!(psse[qq] < INFINITY)) continue;
            ++live;
            sse[(size_t)(D - 1) * k + qq] = psse[qq];
            std::vector<int32_t> g(D);
            for (int j = 0; j < D; ++j) g[j] = sub[pidx[(size_t)qq * D + j]];
            std::sort(g.begin(), g.end());
            for (int j = 0; j < D; ++j) models[((size_t)(D - 1) * k + qq) * Dm + j] = g[j];
            if (coef)
                for (int t = 0; t < T; ++t) {
                    // the fit's coefficients follow the subspace positions in
                    // ascending order; report them for the ascending global indices
                    std::vector<std::pair<int32_t, double>> cj(D);
                    for (int j = 0; j < D; ++j)
                        cj[j] = {sub[pidx[(size_t)qq * D + j]], pcoef[((size_t)qq * T + t) * (D + 1) + 1 + j]};
                    std::sort(cj.begin(), cj.end());
                    double *o = coef + (((size_t)(D - 1) * k + qq) * T + t) * (Dm + 1);
                    o[0] = pcoef[((size_t)qq * T + t) * (D + 1)];
                    for (int j = 0; j < D; ++j) o[1 + j] = cj[j].second;
                }
        }
        if (D == Dm) break;
        // residuals of the n_res best models for the next dimension
        nres = live < d->n_res ? live : d->n_res;
        if (nres < 1) return fit_fail(SISSO_EINVAL, "no full-rank model to take residuals from");
        if (hipMemcpyAsync(midx, pidx.data(), (size_t)nres * D * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(mcoef, pcoef.data(), (size_t)nres * T * (D + 1) * sizeof(double), hipMemcpyHostToDevice,
                           st) != hipSuccess)
            return fit_fail(SISSO_EDEVICE, "copying the models failed");
        if (sis::launch_residuals(Fs, d->y, n, off, T, midx, mcoef, nres, D, R, st))
            return fit_fail(SISSO_EDEVICE, "residual launch failed");
    }
    for (size_t i = 0; i < sub.size(); ++i) subspace[i] = sub[i];
    if (hipStreamSynchronize(st) != hipSuccess) return fit_fail(SISSO_EDEVICE, "stream synchronisation failed");
    return SISSO_OK;
}
