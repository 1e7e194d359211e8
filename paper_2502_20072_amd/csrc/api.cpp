// C ABI of the gfx950 l0 library: argument checks, workspace carving and the
// order of launches.  All arithmetic happens in the kernels.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace sl0;

struct sisso_l0 {
    sisso_l0_desc desc;
    std::vector<int64_t> offsets;
    Layout lay;
    Ctx ctx;
    hipStream_t stream;
    bool gram_done = false;
    bool search_done = false;
    int last_D = 0, last_k = 0;
    uint64_t scored = 0;
    std::string err;
    hipEvent_t ev[2 * SISSO_NPHASE] = {};
    bool ran[SISSO_NPHASE] = {};
    bool prof = false;
    char *stage = nullptr;  // pinned host copy of the result block (one transfer per readout)
    const void *btab_owner = nullptr;  // the batch whose search table this handle's workspace holds
    ~sisso_l0() {
        // the caller may release the workspace once destroy returns: let the
        // handle's enqueued work finish first
        (void)hipStreamSynchronize(stream);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (stage) (void)hipHostFree(stage);
    }
};

static thread_local std::string g_create_err;

static int32_t fail(sisso_l0 *h, int32_t code, const char *msg) {
    if (h) h->err = msg;
    else g_create_err = msg;
    return code;
}

// slices per value of a precision mode (0: FP64 Gram; -1: unknown mode)
static int precision_slices(int32_t precision) {
    switch (precision) {
        case SISSO_PREC_FP64: return 0;
        case SISSO_PREC_BF16_COMP: return 3;
        case SISSO_PREC_FP16_COMP: return 2;
        case SISSO_PREC_FP32_SOLVE: return 0;
        default: return -1;
    }
}

static Layout compute_layout(int64_t n_total, int64_t S, int T, int D_max, int k_max, int lp_ns, bool fp32) {
    Layout L{};
    L.lp_ns = lp_ns > 0 ? lp_ns : 0;
    L.fp32 = fp32 ? 1 : 0;
    // chunks of LP_XC samples per task; bounded without reading the offsets
    L.lp_nchunk = L.lp_ns ? (int)((n_total + LP_XC - 1) / LP_XC + T) : 0;
    L.TP = next_pow2(T);
    const int64_t ntile = (S + GRAM_TILE - 1) / GRAM_TILE;
    const int64_t blocks = ntile * (ntile + 1) / 2 * T;
    // Split the rows of every tile pair into ns parts (>= 256 rows each, at
    // most 8) so that the Gram's workgroups, about equal in cost and one per
    // CU at a time, fill whole rounds of the 256 CUs: the launch takes
    // ceil(blocks ns / 256) rounds of 1/ns of a tile pair's work; a split is
    // taken while it cuts that time by more than 2 % (the finish kernel reads
    // every split's partial matrices).
    // With several tasks the workgroups' costs follow the tasks' row counts
    // (and are launched largest first), so only a small launch is split, to
    // about 512 workgroups.
    const int64_t byrows = n_total / 256 > 1 ? n_total / 256 : 1;
    int64_t ns = 1;
    if (T == 1) {
        const int64_t nsmax = byrows < 8 ? byrows : 8;
        double best = (double)((blocks + 255) / 256);
        for (int64_t q = 2; q <= nsmax; ++q) {
            const double f = (double)((blocks * q + 255) / 256) / (double)q;
            if (f < 0.98 * best) {
                best = f;
                ns = q;
            }
        }
    } else {
        ns = (512 + blocks - 1) / blocks;
        if (ns > byrows) ns = byrows;
        if (ns > 16) ns = 16;
        if (ns < 1) ns = 1;
    }
    L.nsplit = (int)ns;
    // candidates re-scored exactly: k + 16 leaves a margin for FP64
    // normal-equation rounding at the k-th position; the precision forms rank
    // by SSEs from an approximate Gram (relative error ~1e-6..1e-5) or from
    // FP32 solves, so they keep twice as many candidates for the exact re-score
    L.KP = next_pow2((L.lp_ns > 0 || fp32) ? 2 * (k_max + 16) : k_max + 16);
    if (L.KP > KP_MAX) L.KP = KP_MAX;
    if (L.KP < 64) L.KP = 64;
    L.search_wgs = SEARCH_WGS_DEFAULT;
    L.nwaves = SEARCH_WGS_MAX * SEARCH_WAVES;
    const int64_t nlists = L.nwaves;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t d = sizeof(double);
    L.self = take(sizeof(Ctx));
    L.btab = take(S3B_TABLE_BYTES);
    L.off_dev = take((T + 1) * sizeof(int64_t));
    L.torder = take(T * sizeof(int32_t));
    L.ybar = take(T * d);
    L.cyy = take(T * d);
    L.mu = take((size_t)T * S * d);
    L.inv_s = take((size_t)T * S * d);
    L.bhat = take((size_t)S * L.TP * d);
    const size_t Sp = (size_t)((S + GT - 1) / GT) * GT;
    L.G = take(Sp * Sp * L.TP * d);
    L.part = take((size_t)L.nsplit * T * S * S * d);
    L.flags = take(64 * sizeof(uint32_t));
    L.lp_cbase = take((size_t)(T + 1) * sizeof(int32_t));
    L.lp_exp = take((size_t)S * L.lp_nchunk * sizeof(int32_t));
    L.lp_slices = take((size_t)L.lp_ns * S * L.lp_nchunk * LP_XC * 2);
    L.stat_bits = take(4 * sizeof(uint64_t));
    // pre-pass + counters: theta, work counter, cand counter, cum table, prefixes, scores
    L.pre = take(64 + (size_t)(S / 4 + 8) * sizeof(uint64_t) + PRE_Q * SISSO_MAX_D * sizeof(int32_t) +
                 64 + (size_t)PRE_Q * S * d + PRE_Q * d + 1024 +
                 (size_t)(SISSO_MAX_D + 1) * (S + 1) * sizeof(uint64_t) + 64 + 256);
    // one row of four (i1, j) records per j > i1 group: sum over groups of (S - 2 - 4 g)
    {
        const int64_t ng3 = S >= 3 ? (S - 3) / 4 + 1 : 0;
        const int64_t rows3 = ng3 * (S - 2) - 4 * (ng3 * (ng3 - 1) / 2);
        L.rec3_bytes = (D_max >= 3 && S >= 3 && !fp32) ? (size_t)rows3 * 16 * d : 0;
    }
    L.rec3 = take(L.rec3_bytes);
    // D = 4, one task: a record row per (pair group, j); kept only while the
    // table stays within S4_TABLE_MAX (else the general kernel runs)
    {
        const int64_t rows4 = S >= 4 ? s4_rows_below(S, S - 2) : 0;
        const size_t b4 = (size_t)rows4 * S4_ROW * d;
        L.rec4_bytes = (D_max >= 4 && T == 1 && S >= 4 && !fp32 && b4 <= S4_TABLE_MAX && s4_tiles_host(S) < (1ull << 31)) ? b4 : 0;
    }
    L.rec4 = take(L.rec4_bytes);
    L.r4off = take(L.rec4_bytes ? (size_t)(S + 1) * sizeof(int64_t) : 0);
    L.G1_bytes = (D_max >= 3 && S >= 3 && T > 1) ? Sp * Sp * d : 0;
    L.G1 = take(L.G1_bytes);
    // several tasks, D = 3: a pool with a record for every step of the sweep
    // plus one partly filled chunk per wave, so that it cannot run out (the
    // pool grows as S^3: 2 GB at S = 5000); above MTQ_POOL_MAX bytes of
    // records the several-task search keeps its general kernel
    L.mtq_chunks = 0;
    if (L.G1_bytes) {
        const uint64_t steps = s3_tiles_host(S) * (uint64_t)s3_rows_per_tile();
        const uint64_t chunks = (steps + MTQ_CHUNK - 1) / MTQ_CHUNK + (uint64_t)nlists;
        if (chunks * MTQ_CHUNK * 3 * sizeof(uint64_t) <= MTQ_POOL_MAX) L.mtq_chunks = (int)chunks;
    }
    const size_t nch = (size_t)L.mtq_chunks;
    L.mtq = take(nch * MTQ_CHUNK * 3 * sizeof(uint64_t));
    L.mtq_n = take(nch * sizeof(uint32_t));
    L.mtq_pre = take(nch ? (nch + 1) * sizeof(uint64_t) : 0);
    L.lists = take((size_t)nlists * L.KP * 2 * d + (size_t)nlists * L.KP * 2 * d);
    L.merged = take((size_t)L.KP * 2 * d);
    L.rescored = take((size_t)L.KP * d);
    L.coef = take((size_t)L.KP * T * (D_max + 1) * d);
    {
        const size_t idx_bytes = ((size_t)k_max * D_max * sizeof(int32_t) + 7) & ~(size_t)7;
        const size_t coef_bytes = (size_t)k_max * T * (D_max + 1) * d;
        L.res_bytes = 16 + (size_t)k_max * d + idx_bytes + coef_bytes;
        L.res = take(L.res_bytes);
        L.res_sse = L.res + 16;
        L.res_idx = L.res_sse + (size_t)k_max * d;
        L.res_coef = L.res_idx + idx_bytes;
    }
    L.total = o;
    return L;
}

static bool shape_ok(const sisso_l0_desc *d) {
    return d && d->n_total >= 1 && d->S >= 1 && d->T >= 1 && d->T <= SISSO_MAX_T && d->D_max >= 1 &&
           d->D_max <= SISSO_MAX_D && d->k_max >= 1 && d->k_max <= SISSO_MAX_K && d->S < (1 << 30);
}

extern "C" size_t sisso_l0_workspace_bytes(const sisso_l0_desc *d) {
    if (!shape_ok(d)) return 0;
    const int ns = precision_slices(d->precision);
    if (ns < 0) return 0;
    return compute_layout(d->n_total, d->S, d->T, d->D_max, d->k_max, ns, d->precision == SISSO_PREC_FP32_SOLVE).total +
           256;
}

static void carve(sisso_l0 *h) {
    const Layout &L = h->lay;
    char *base = (char *)h->desc.workspace;
    Ctx &c = h->ctx;
    c = Ctx{};
    c.F = h->desc.F;
    c.y = h->desc.y;
    c.n_total = h->desc.n_total;
    c.S = h->desc.S;
    c.T = h->desc.T;
    c.TP = L.TP;
    c.Gnt = (c.S + GT - 1) / GT;
    c.rows_max = 0;
    for (int t = 0; t < c.T; ++t)
        c.rows_max = std::max(c.rows_max, h->offsets[t + 1] - h->offsets[t]);
    c.off_dev = (int64_t *)(base + L.off_dev);
    c.torder = (int32_t *)(base + L.torder);
    c.ybar = (double *)(base + L.ybar);
    c.cyy = (double *)(base + L.cyy);
    c.mu = (double *)(base + L.mu);
    c.inv_s = (double *)(base + L.inv_s);
    c.bhat = (double *)(base + L.bhat);
    c.G = (double *)(base + L.G);
    c.part = (double *)(base + L.part);
    c.flags = (uint32_t *)(base + L.flags);
    c.lp_cbase = (int32_t *)(base + L.lp_cbase);
    c.lp_exp = (int32_t *)(base + L.lp_exp);
    c.lp_slices = (__bf16 *)(base + L.lp_slices);
    c.err_bits = (unsigned long long *)(base + L.stat_bits);
    c.lp_ns = L.lp_ns;
    c.fp32 = L.fp32;
    char *p = base + L.pre;
    c.theta_bits = (unsigned long long *)p;
    c.work_counter = (unsigned int *)(p + 8);
    c.cand_counter = (unsigned int *)(p + 12);
    c.pre_count = (int32_t *)(p + 16);
    c.pre_done = (unsigned int *)(p + 20);
    c.mtq_taken = (unsigned int *)(p + 60);
    c.stats = (uint64_t *)(p + 24);
    c.merge_count = (unsigned int *)(p + 56);
    p += 64;
    c.cum = (uint64_t *)p;
    p += (size_t)(c.S / 4 + 8) * sizeof(uint64_t);
    c.pre_prefix = (int32_t *)p;
    p += align256(PRE_Q * SISSO_MAX_D * sizeof(int32_t));
    c.pre_bound = (double *)p;
    p += align256(PRE_Q * sizeof(double));
    c.pre_sse = (double *)p;
    p += align256((size_t)PRE_Q * c.S * sizeof(double));
    c.btab = (uint64_t *)p;
    p += (size_t)(SISSO_MAX_D + 1) * (c.S + 1) * sizeof(uint64_t);
    c.tstar = (int32_t *)p;
    c.rec3 = L.rec3_bytes ? (double *)(base + L.rec3) : nullptr;
    c.G1 = L.G1_bytes ? (double *)(base + L.G1) : c.G;
    c.rec4 = L.rec4_bytes ? (double *)(base + L.rec4) : nullptr;
    c.r4off = L.rec4_bytes ? (int64_t *)(base + L.r4off) : nullptr;
    c.mtq_chunks = L.mtq_chunks;
    c.mtq = L.mtq_chunks ? (uint64_t *)(base + L.mtq) : nullptr;
    c.mtq_n = L.mtq_chunks ? (uint32_t *)(base + L.mtq_n) : nullptr;
    c.mtq_pre = L.mtq_chunks ? (uint64_t *)(base + L.mtq_pre) : nullptr;
    const int64_t nl = L.nwaves;
    char *q = base + L.lists;
    c.list_sse = (double *)q;
    q += (size_t)nl * L.KP * sizeof(double);
    c.list_rank = (uint64_t *)q;
    q += (size_t)nl * L.KP * sizeof(uint64_t);  // KP >= 64: every region stays 256-byte aligned
    c.cand_sse = (double *)q;
    q += (size_t)nl * L.KP * sizeof(double);
    c.cand_rank = (uint64_t *)q;
    c.merged_sse = (double *)(base + L.merged);
    c.merged_rank = (uint64_t *)(base + L.merged + (size_t)L.KP * sizeof(double));
    c.resc_sse = (double *)(base + L.rescored);
    c.resc_coef = (double *)(base + L.coef);
    c.res_flags = (uint32_t *)(base + L.res);
    c.res_idx = (int32_t *)(base + L.res_idx);
    c.res_sse = (double *)(base + L.res_sse);
    c.res_coef = (double *)(base + L.res_coef);
    c.nsplit = L.nsplit;
    c.KP = L.KP;
    c.nwaves = L.nwaves;
    c.search_wgs = L.search_wgs;
    c.D_max = h->desc.D_max;
    c.k_max = h->desc.k_max;
    c.ev = h->prof ? h->ev : nullptr;
}

extern "C" int32_t sisso_l0_create(const sisso_l0_desc *d, sisso_l0 **out) {
    if (!d || !out) return fail(nullptr, SISSO_EINVAL, "null descriptor or output pointer");
    if (!d->F || !d->y || !d->task_offsets || !d->workspace)
        return fail(nullptr, SISSO_EINVAL, "null F, y, task_offsets or workspace");
    if (!shape_ok(d)) return fail(nullptr, SISSO_EINVAL, "shape out of range (n_total, S, T, D_max, k_max)");
    if (precision_slices(d->precision) < 0) return fail(nullptr, SISSO_ENOTSUP, "unknown precision mode");
    const int64_t *o = d->task_offsets;
    if (o[0] != 0 || o[d->T] != d->n_total) return fail(nullptr, SISSO_EINVAL, "task offsets must span [0, n_total)");
    for (int t = 0; t < d->T; ++t)
        if (o[t + 1] <= o[t]) return fail(nullptr, SISSO_EINVAL, "every task needs at least one row");
    if (((uintptr_t)d->workspace & 255) != 0) return fail(nullptr, SISSO_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = sisso_l0_workspace_bytes(d);
    if (d->workspace_bytes < need) return fail(nullptr, SISSO_ENOMEM, "workspace smaller than sisso_l0_workspace_bytes");
    sisso_l0 *h = new (std::nothrow) sisso_l0();
    if (!h) return fail(nullptr, SISSO_ENOMEM, "host allocation failed");
    h->desc = *d;
    h->offsets.assign(o, o + d->T + 1);
    h->desc.task_offsets = h->offsets.data();
    h->lay = compute_layout(d->n_total, d->S, d->T, d->D_max, d->k_max, precision_slices(d->precision),
                            d->precision == SISSO_PREC_FP32_SOLVE);
    h->stream = (hipStream_t)d->stream;
    carve(h);
    if (hipHostMalloc((void **)&h->stage, h->lay.res_bytes, hipHostMallocDefault) != hipSuccess) {
        h->stage = nullptr;
        delete h;
        return fail(nullptr, SISSO_EDEVICE, "could not allocate the pinned result stage");
    }
    // precision form: chunks of LP_XC samples per task (the count never
    // exceeds the bound the layout was sized with)
    std::vector<int32_t> cbase(d->T + 1, 0);
    for (int t = 0; t < d->T; ++t) cbase[t + 1] = cbase[t] + (int32_t)((o[t + 1] - o[t] + LP_XC - 1) / LP_XC);
    h->ctx.lp_nchunk = h->lay.lp_ns ? cbase[d->T] : 0;
    // the Gram's workgroups of the largest tasks go first (a task's
    // workgroups take time in proportion to its rows)
    std::vector<int32_t> order(d->T);
    for (int t = 0; t < d->T; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return o[a + 1] - o[a] > o[b + 1] - o[b]; });
    if (hipMemcpyAsync((char *)d->workspace + h->lay.self, &h->ctx, sizeof(Ctx), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ctx.off_dev, h->offsets.data(), (d->T + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ctx.torder, order.data(), d->T * sizeof(int32_t), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ctx.lp_cbase, cbase.data(), (d->T + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        delete h;
        return fail(nullptr, SISSO_EDEVICE, "could not initialise the workspace on the device");
    }
    *out = h;
    return SISSO_OK;
}

extern "C" int32_t sisso_gram(sisso_l0 *h) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (launch_stats(h->ctx, h->stream) || launch_gram(h->ctx, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    h->ran[SISSO_PHASE_STATS] = h->ran[SISSO_PHASE_GRAM] = h->prof;
    h->gram_done = true;
    h->search_done = false;
    return SISSO_OK;
}

// Argument and state checks of a search; fills the launch description.
static int32_t check_search(sisso_l0 *h, int32_t D, int32_t k, bool ranged, uint64_t r0, uint64_t r1,
                            bool need_gram, SearchCall *sc, uint64_t *scored) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (need_gram && !h->gram_done) return fail(h, SISSO_ESTATE, "sisso_gram must run before a search");
    if (D > h->desc.D_max || D > SISSO_MAX_D) return fail(h, SISSO_ENOTSUP, "D exceeds D_max");
    if (D < 1 || D > h->desc.S) return fail(h, SISSO_EINVAL, "need 1 <= D <= S");
    if (k < 1 || k > h->desc.k_max) return fail(h, SISSO_EINVAL, "need 1 <= k <= k_max");
    if (D > 1 && (uint64_t)h->desc.S > (1ull << (64 / D)))
        return fail(h, SISSO_ENOTSUP, "S exceeds 2^(64/D), the range of the packed top-k key");
    const uint64_t total = binom(h->desc.S, D);
    if (total >= (1ull << 63)) return fail(h, SISSO_ENOTSUP, "C(S, D) does not fit the 63-bit rank space");
    if (ranged) {
        if (r0 >= r1 || r1 > total) return fail(h, SISSO_EINVAL, "need r0 < r1 <= C(S, D)");
        if ((uint64_t)k > r1 - r0) return fail(h, SISSO_EINVAL, "k exceeds the number of tuples in the range");
    } else if ((uint64_t)k > total) {
        return fail(h, SISSO_EINVAL, "k exceeds C(S, D)");
    }
    for (int t = 0; t < h->desc.T; ++t)
        if (h->offsets[t + 1] - h->offsets[t] < D + 2) return fail(h, SISSO_EINVAL, "a task has fewer than D + 2 rows");
    *sc = SearchCall{D, k, ranged ? 1 : 0, ranged ? r0 : 0, ranged ? r1 : total};
    *scored = ranged ? r1 - r0 : total;
    return SISSO_OK;
}

static int32_t do_search(sisso_l0 *h, int32_t D, int32_t k, bool ranged, uint64_t r0, uint64_t r1) {
    SearchCall sc;
    uint64_t scored = 0;
    const int32_t rc = check_search(h, D, k, ranged, r0, r1, true, &sc, &scored);
    if (rc != SISSO_OK) return rc;
    if (launch_search(h->ctx, sc, h->stream)) return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    for (int ph = SISSO_PHASE_PREPASS; ph <= SISSO_PHASE_FINAL; ++ph) h->ran[ph] = h->prof;
    h->search_done = true;
    h->last_D = D;
    h->last_k = k;
    h->scored = scored;
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_search(sisso_l0 *h, int32_t D, int32_t k) { return do_search(h, D, k, false, 0, 0); }

extern "C" int32_t sisso_l0_search_range(sisso_l0 *h, int32_t D, int32_t k, uint64_t r0, uint64_t r1) {
    return do_search(h, D, k, true, r0, r1);
}

// ------------------------------------------------------ prefix-list calls
static int32_t check_prefixes(sisso_l0 *h, int32_t m, const void *pre, int64_t n) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (!h->gram_done) return fail(h, SISSO_ESTATE, "sisso_gram must run first");
    if (n < 0 || (n > 0 && !pre)) return fail(h, SISSO_EINVAL, "null prefix list or negative count");
    if (m < 1 || m > h->desc.S) return fail(h, SISSO_EINVAL, "need 1 <= prefix length <= S");
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_prefix_best(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, double *best) {
    int32_t rc = check_prefixes(h, m, prefixes, n);
    if (rc != SISSO_OK) return rc;
    if (m + 1 > SISSO_MAX_D) return fail(h, SISSO_ENOTSUP, "prefix length + 1 exceeds SISSO_MAX_D");
    if (n > 0 && !best) return fail(h, SISSO_EINVAL, "null output");
    for (int t = 0; t < h->desc.T; ++t)
        if (h->offsets[t + 1] - h->offsets[t] < m + 3) return fail(h, SISSO_EINVAL, "a task has too few rows");
    if (n == 0) return SISSO_OK;
    if (launch_prefix_best(h->ctx, m, prefixes, n, best, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_prefix_target(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, double *best,
                                          float *target) {
    int32_t rc = sisso_l0_prefix_best(h, m, prefixes, n, best);
    if (rc != SISSO_OK) return rc;
    if (n > 0 && !target) return fail(h, SISSO_EINVAL, "null output");
    if (n == 0) return SISSO_OK;
    if (launch_prefix_target(h->ctx, best, n, target, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_prefix_features(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, float *feat) {
    int32_t rc = check_prefixes(h, m, prefixes, n);
    if (rc != SISSO_OK) return rc;
    if (m > SISSO_MAX_D) return fail(h, SISSO_ENOTSUP, "prefix length exceeds SISSO_MAX_D");
    if (n > 0 && !feat) return fail(h, SISSO_EINVAL, "null output");
    if (n == 0) return SISSO_OK;
    if (launch_prefix_features(h->ctx, m, prefixes, n, feat, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_prefix_extend(sisso_l0 *h, int32_t m, const int32_t *prefixes, int64_t n, int32_t *out) {
    int32_t rc = check_prefixes(h, m, prefixes, n);
    if (rc != SISSO_OK) return rc;
    if (m + 1 > SISSO_MAX_D) return fail(h, SISSO_ENOTSUP, "prefix length + 1 exceeds SISSO_MAX_D");
    if (m >= h->desc.S) return fail(h, SISSO_EINVAL, "a prefix of length S has no extension");
    if (n > 0 && !out) return fail(h, SISSO_EINVAL, "null output");
    if (n > (int64_t(1) << 40) / (h->desc.S - m)) return fail(h, SISSO_EINVAL, "too many extensions");
    if (n == 0) return SISSO_OK;
    if (launch_prefix_extend(h->ctx, m, prefixes, n, out, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_prefix_features_range(sisso_l0 *h, int32_t m, uint64_t r0, int64_t n, float *feat) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (!h->gram_done) return fail(h, SISSO_ESTATE, "sisso_gram must run first");
    if (m < 1 || m > 3 || m > h->desc.S) return fail(h, SISSO_EINVAL, "need 1 <= m <= 3 and m <= S");
    if (n < 0 || (n > 0 && !feat)) return fail(h, SISSO_EINVAL, "null output or negative count");
    const uint64_t total = binom(h->desc.S, m);
    if (r0 > total || (uint64_t)n > total - r0) return fail(h, SISSO_EINVAL, "rank range exceeds C(S, m)");
    if (n == 0) return SISSO_OK;
    if (launch_prefix_features_range(h->ctx, m, r0, n, feat, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_search_list(sisso_l0 *h, int32_t D, int32_t k, const int32_t *prefixes, int64_t n) {
    int32_t rc = check_prefixes(h, D - 1, prefixes, n);
    if (rc != SISSO_OK) return rc;
    SearchCall sc;
    uint64_t scored = 0;
    rc = check_search(h, D, k, false, 0, 0, true, &sc, &scored);
    if (rc != SISSO_OK) return rc;
    if (D < 2) return fail(h, SISSO_EINVAL, "a prefix list needs D >= 2");
    if (launch_list_search(h->ctx, D, k, prefixes, n, h->stream))
        return fail(h, SISSO_EDEVICE, hipGetErrorString(hipGetLastError()));
    for (int ph = SISSO_PHASE_PREPASS; ph <= SISSO_PHASE_FINAL; ++ph) h->ran[ph] = h->prof;
    h->search_done = true;
    h->last_D = D;
    h->last_k = k;
    h->scored = (uint64_t)n * (uint64_t)(h->desc.S - D + 1);
    return SISSO_OK;
}

// ---------------------------------------------------------------- autotuner
// The persistent search grid is the one launch parameter whose best value
// depends on the problem (items per workgroup vs. latency hiding) and that
// changes no arithmetic: every grid size gives bit-identical results.

extern "C" int32_t sisso_l0_set_search_grid(sisso_l0 *h, int32_t workgroups) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (workgroups < 1 || workgroups > SEARCH_WGS_MAX) return fail(h, SISSO_EINVAL, "grid size out of range");
    h->ctx.search_wgs = workgroups;
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_search_grid(const sisso_l0 *h) { return h ? h->ctx.search_wgs : 0; }

// Cache file: a JSON object with one entry per line,
//   "<arch>|D=<D>|S=<S rounded up to a power of two>|T=<T>|P=<precision>": {"search_wgs": W, "ms": t},
static std::map<std::string, std::pair<int, double>> read_cache(const char *path) {
    std::map<std::string, std::pair<int, double>> m;
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return m;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        const char *q0 = strchr(line, '"');
        const char *q1 = q0 ? strchr(q0 + 1, '"') : nullptr;
        const char *w = q1 ? strstr(q1, "\"search_wgs\":") : nullptr;
        const char *t = q1 ? strstr(q1, "\"ms\":") : nullptr;
        if (!w || !t) continue;
        m[std::string(q0 + 1, q1)] = {atoi(w + 13), atof(t + 5)};
    }
    fclose(f);
    return m;
}

static bool write_cache(const char *path, const std::map<std::string, std::pair<int, double>> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fputs("{\n", f);
    size_t i = 0;
    for (const auto &e : m)
        fprintf(f, "\"%s\": {\"search_wgs\": %d, \"ms\": %.6f}%s\n", e.first.c_str(), e.second.first, e.second.second,
                ++i < m.size() ? "," : "");
    fputs("}\n", f);
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

extern "C" int32_t sisso_l0_autotune(sisso_l0 *h, int32_t D, int32_t k, const char *cache_path, int32_t *chosen) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    SearchCall sc;
    uint64_t scored = 0;
    int32_t rc = check_search(h, D, k, false, 0, 0, true, &sc, &scored);
    if (rc != SISSO_OK) return rc;
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(h, SISSO_EDEVICE, "cannot query the device");
    char key[256];
    snprintf(key, sizeof key, "%s|D=%d|S=%d|T=%d|P=%d", prop.gcnArchName, D, next_pow2((int)h->desc.S), h->desc.T,
             h->desc.precision);
    auto cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end() && it->second.first >= 1 && it->second.first <= SEARCH_WGS_MAX) {
        h->ctx.search_wgs = it->second.first;
        if (chosen) *chosen = h->ctx.search_wgs;
        return SISSO_OK;
    }
    static const int cand[] = {256, 512, 768, 1024, 1280, 1536, 2048};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(h, SISSO_EDEVICE, "hipEventCreate failed");
    hipEvent_t *saved_ev = h->ctx.ev;
    h->ctx.ev = nullptr;  // no phase events inside the timed launches
    int best = h->ctx.search_wgs;
    double best_ms = 1e300;
    bool ok = true;
    for (int w : cand) {
        h->ctx.search_wgs = w;
        if (launch_search(h->ctx, sc, h->stream)) { ok = false; break; }  // warm-up
        float ms = 0.f;
        if (hipEventRecord(e0, h->stream) != hipSuccess) { ok = false; break; }
        for (int r = 0; r < 3; ++r)
            if (launch_search(h->ctx, sc, h->stream)) { ok = false; break; }
        if (!ok || hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { ok = false; break; }
        if (ms / 3.0 < best_ms) {
            best_ms = ms / 3.0;
            best = w;
        }
    }
    h->ctx.ev = saved_ev;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->ctx.search_wgs = best;
    // the timed launches left a complete search of (D, k) behind
    h->search_done = ok;
    h->last_D = D;
    h->last_k = k;
    h->scored = scored;
    if (!ok) return fail(h, SISSO_EDEVICE, "a timed search launch failed");
    if (chosen) *chosen = best;
    if (cache_path) {
        cache[key] = {best, best_ms};
        if (!write_cache(cache_path, cache)) return fail(h, SISSO_EINVAL, "cannot write the autotune cache");
    }
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_topk(sisso_l0 *h, int32_t k, int32_t *idx, double *sse, double *coef) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (!h->search_done) return fail(h, SISSO_ESTATE, "no search has run");
    if (k < 1 || k > h->last_k) return fail(h, SISSO_ESTATE, "k exceeds the searched k");
    if (!idx || !sse) return fail(h, SISSO_EINVAL, "null idx or sse");
    const int D = h->last_D, T = h->desc.T;
    const Layout &L = h->lay;
    // the final kernel leaves status words, SSEs, indices and coefficients in
    // one block: a single transfer into the pinned stage, then host copies
    const size_t bytes = coef ? L.res_bytes : L.res_coef - L.res;
    hipError_t e = hipMemcpyAsync(h->stage, h->ctx.res_flags, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, SISSO_EDEVICE, hipGetErrorString(e));
    uint32_t flags[4];
    memcpy(flags, h->stage, sizeof(flags));
    if (flags[FLAG_NONFINITE]) return fail(h, SISSO_EINVAL, "F or y holds a non-finite value");
    if (flags[FLAG_CAPACITY]) return fail(h, SISSO_EDEVICE, "internal step queue overflow (results incomplete)");
    memcpy(sse, h->stage + (L.res_sse - L.res), (size_t)k * sizeof(double));
    memcpy(idx, h->stage + (L.res_idx - L.res), (size_t)k * D * sizeof(int32_t));
    if (coef) memcpy(coef, h->stage + (L.res_coef - L.res), (size_t)k * T * (D + 1) * sizeof(double));
    return SISSO_OK;
}

extern "C" int32_t sisso_gram_read(sisso_l0 *h, int32_t t, double *G, double *b, double *c) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (!h->gram_done) return fail(h, SISSO_ESTATE, "sisso_gram has not run");
    if (t < 0 || t >= h->desc.T) return fail(h, SISSO_EINVAL, "task index out of range");
    const size_t S = (size_t)h->desc.S, TP = (size_t)h->ctx.TP, d = sizeof(double);
    hipError_t e = hipSuccess;
    // the tiled, task-fastest matrix is unpacked into the Gram partial buffer
    // (free after sisso_gram) and copied from there
    if (G) {
        if (launch_untile(h->ctx, t, h->ctx.part, h->stream)) return fail(h, SISSO_EDEVICE, "untile launch failed");
        e = hipMemcpyAsync(G, h->ctx.part, S * S * d, hipMemcpyDeviceToHost, h->stream);
    }
    if (e == hipSuccess && b) e = hipMemcpy2DAsync(b, d, h->ctx.bhat + t, TP * d, d, S, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && c) e = hipMemcpyAsync(c, h->ctx.cyy + t, d, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, SISSO_EDEVICE, hipGetErrorString(e));
    return SISSO_OK;
}

extern "C" uint64_t sisso_l0_scored(const sisso_l0 *h) { return h ? h->scored : 0; }

extern "C" int32_t sisso_l0_profile(sisso_l0 *h, int32_t enable) {
    if (!h) return SISSO_EINVAL;
    h->err.clear();
    if (enable && !h->ev[0]) {
        for (auto &e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(h, SISSO_EDEVICE, "hipEventCreate failed");
    }
    h->prof = enable != 0;
    h->ctx.ev = h->prof ? h->ev : nullptr;
    for (auto &r : h->ran) r = false;
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_search_stats(sisso_l0 *h, uint64_t *out) {
    if (!h || !out) return SISSO_EINVAL;
    h->err.clear();
    if (!h->search_done) return fail(h, SISSO_ESTATE, "no search has run");
    hipError_t e = hipMemcpyAsync(out, h->ctx.stats, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, SISSO_EDEVICE, hipGetErrorString(e));
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_precision_report(sisso_l0 *h, int32_t nsample, double *out) {
    if (!h || !out || nsample < 1) return SISSO_EINVAL;
    h->err.clear();
    if (!h->gram_done) return fail(h, SISSO_ESTATE, "sisso_gram has not run");
    uint64_t bits[2] = {0, 0};
    hipError_t e = hipMemsetAsync(h->ctx.err_bits, 0, sizeof(uint64_t), h->stream);
    if (e == hipSuccess && launch_gram_check(h->ctx, nsample, h->ctx.err_bits, h->stream)) e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(bits, h->ctx.err_bits, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, SISSO_EDEVICE, hipGetErrorString(e));
    double g, s;
    memcpy(&g, &bits[0], sizeof g);
    memcpy(&s, &bits[1], sizeof s);
    out[0] = g;
    out[1] = (double)nsample * h->desc.T;
    out[2] = h->search_done ? s : 0.0;
    out[3] = h->lay.lp_ns;
    return SISSO_OK;
}

extern "C" int32_t sisso_gram_error(sisso_l0 *h, double *max_abs_rel) {
    if (!h || !max_abs_rel) return SISSO_EINVAL;
    double rep[4];
    const int32_t rc = sisso_l0_precision_report(h, 4096, rep);
    if (rc != SISSO_OK) return rc;
    *max_abs_rel = rep[0];
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_phase_ms(sisso_l0 *h, double *ms) {
    if (!h || !ms) return SISSO_EINVAL;
    h->err.clear();
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, SISSO_EDEVICE, "stream synchronisation failed");
    for (int ph = 0; ph < SISSO_NPHASE; ++ph) {
        ms[ph] = 0.0;
        if (!h->ran[ph]) continue;
        float f = 0.f;
        if (hipEventElapsedTime(&f, h->ev[2 * ph], h->ev[2 * ph + 1]) != hipSuccess)
            return fail(h, SISSO_EDEVICE, "hipEventElapsedTime failed");
        ms[ph] = f;
    }
    return SISSO_OK;
}

extern "C" void sisso_l0_destroy(sisso_l0 *h) { delete h; }

extern "C" const char *sisso_l0_last_error(const sisso_l0 *h) {
    return h ? h->err.c_str() : g_create_err.c_str();
}

extern "C" uint64_t sisso_l0_rank_of(int64_t S, int32_t D, const int32_t *t) {
    if (!t || D < 1 || D > 8 || S < D) return UINT64_MAX;
    for (int m = 0; m < D; ++m) {
        if (t[m] < 0 || t[m] >= S) return UINT64_MAX;
        if (m > 0 && t[m] <= t[m - 1]) return UINT64_MAX;
    }
    return lex_rank(BinomCalc{}, S, D, t);
}

extern "C" int32_t sisso_l0_unrank(int64_t S, int32_t D, uint64_t r, int32_t *t) {
    if (!t || D < 1 || D > 8 || S < D || r >= binom(S, D)) return SISSO_EINVAL;
    lex_unrank(BinomCalc{}, S, D, r, t);
    return SISSO_OK;
}

// ------------------------------------------------------------------ batching
// A batch is one HIP graph holding, for every problem, the statistics, Gram
// and search launches as a chain on its own branch (branches run
// concurrently); the graph is captured once and then launched as one unit,
// as often as needed.  Each problem's results are then read with
// sisso_l0_topk on its handle, exactly as after an unbatched search.
struct sisso_l0_batch {
    std::vector<sisso_l0 *> hs;
    std::vector<sisso_l0 *> leads;             // handles whose workspace holds a shared-search table
    std::vector<BatchSearchArgs> tables;       // the shared search launches
    std::vector<SearchCall> calls;
    std::vector<uint64_t> scored;
    int D = 0, k = 0;
    hipStream_t user = nullptr, cap = nullptr;
    std::vector<hipStream_t> br;
    std::vector<hipEvent_t> evs;
    hipEvent_t in = nullptr, out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~sisso_l0_batch() {
        for (auto h : leads)
            if (h->btab_owner == this) h->btab_owner = nullptr;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : evs) (void)hipEventDestroy(e);
        if (in) (void)hipEventDestroy(in);
        if (out) (void)hipEventDestroy(out);
        for (auto s : br) (void)hipStreamDestroy(s);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

static thread_local std::string g_batch_err;

static int32_t batch_fail(sisso_l0_batch *b, int32_t code, const char *msg) {
    g_batch_err = msg;
    delete b;
    return code;
}

extern "C" int32_t sisso_l0_batch_create(sisso_l0 *const *hs, int32_t P, int32_t D, int32_t k, sisso_l0_batch **out) {
    if (!hs || !out || P < 1) {
        g_batch_err = "null handles or output, or P < 1";
        return SISSO_EINVAL;
    }
    sisso_l0_batch *b = new (std::nothrow) sisso_l0_batch();
    if (!b) return SISSO_ENOMEM;
    b->D = D;
    b->k = k;
    b->user = hs[0] ? hs[0]->stream : nullptr;
    for (int p = 0; p < P; ++p) {
        sisso_l0 *h = hs[p];
        if (!h) return batch_fail(b, SISSO_EINVAL, "null handle in batch");
        if (h->stream != b->user) return batch_fail(b, SISSO_EINVAL, "all handles of a batch must share one stream");
        for (int q = 0; q < p; ++q)
            if (hs[q] == h) return batch_fail(b, SISSO_EINVAL, "a handle appears twice in the batch");
        SearchCall sc;
        uint64_t sc_n = 0;
        const int32_t rc = check_search(h, D, k, false, 0, 0, false, &sc, &sc_n);
        if (rc != SISSO_OK) return batch_fail(b, rc, h->err.c_str());
        b->hs.push_back(h);
        b->calls.push_back(sc);
        b->scored.push_back(sc_n);
    }
    const int NB = P < 16 ? P : 16;  // concurrent branches
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return batch_fail(b, SISSO_EDEVICE, "stream creation failed");
    b->br.resize(NB, nullptr);
    for (auto &st : b->br)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return batch_fail(b, SISSO_EDEVICE, "stream creation failed");
    b->evs.resize(3 * (NB + 1), nullptr);
    for (auto &e : b->evs)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return batch_fail(b, SISSO_EDEVICE, "event creation failed");
    if (hipEventCreateWithFlags(&b->in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->out, hipEventDisableTiming) != hipSuccess)
        return batch_fail(b, SISSO_EDEVICE, "event creation failed");
    // one-task D = 3 problems share one search launch (a device queue of tile
    // runs, largest problems first); the others keep their own search
    std::vector<int> shared;
    for (int p = 0; p < P; ++p)
        if (s3_batchable(b->hs[p]->ctx, D)) shared.push_back(p);
    std::stable_sort(shared.begin(), shared.end(), [&](int x, int y) {
        return s3_tiles_host(b->hs[x]->desc.S) > s3_tiles_host(b->hs[y]->desc.S);
    });
    std::vector<char> in_shared(P, 0);
    for (int p : shared) in_shared[p] = 1;
    // the shared launches' tables (item prefix, context pointers) live in the
    // workspace of each launch's first problem, which a batch holds until it is
    // destroyed
    for (size_t g0 = 0; g0 < shared.size(); g0 += S3B_MAXP) {
        BatchSearchArgs a{};
        a.P = (int)std::min(shared.size() - g0, (size_t)S3B_MAXP);
        sisso_l0 *lead = b->hs[shared[g0]];
        if (lead->btab_owner) return batch_fail(b, SISSO_EINVAL, "a handle already leads another live batch");
        std::vector<uint32_t> ends(a.P);
        std::vector<const Ctx *> ptrs(a.P);
        uint32_t acc = 0;
        for (int q = 0; q < a.P; ++q) {
            sisso_l0 *h = b->hs[shared[g0 + q]];
            acc += (uint32_t)((s3_tiles_host(h->desc.S) + S3B_RUN - 1) / S3B_RUN);
            ends[q] = acc;
            ptrs[q] = (const Ctx *)((const char *)h->desc.workspace + h->lay.self);
            a.KPmax = std::max(a.KPmax, h->ctx.KP);
        }
        char *tab = (char *)lead->desc.workspace + lead->lay.btab;
        a.item_end = (const uint32_t *)tab;
        a.ctx = (const Ctx *const *)(tab + S3B_MAXP * sizeof(uint32_t));
        if (hipMemcpyAsync(tab, ends.data(), a.P * sizeof(uint32_t), hipMemcpyHostToDevice, b->user) != hipSuccess ||
            hipMemcpyAsync(tab + S3B_MAXP * sizeof(uint32_t), ptrs.data(), a.P * sizeof(void *), hipMemcpyHostToDevice,
                           b->user) != hipSuccess ||
            hipStreamSynchronize(b->user) != hipSuccess)
            return batch_fail(b, SISSO_EDEVICE, "could not write the batch search table");
        lead->btab_owner = b;
        b->leads.push_back(lead);
        b->tables.push_back(a);
    }
    // capture: fork to every branch (problems sharing a branch run one after
    // another); phase 1 = statistics, Gram and the searches' set-up (the whole
    // search for the others); join; the shared search launches; fork; phase 2 =
    // merge, re-score and final ordering of the shared problems; join
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return batch_fail(b, SISSO_EDEVICE, "hipStreamBeginCapture failed");
    auto fork = [&](int stage) {
        bool ok = hipEventRecord(b->evs[stage * (NB + 1) + NB], b->cap) == hipSuccess;
        for (int i = 0; i < NB && ok; ++i) ok = hipStreamWaitEvent(b->br[i], b->evs[stage * (NB + 1) + NB], 0) == hipSuccess;
        return ok;
    };
    auto join = [&](int stage) {
        bool ok = true;
        for (int i = 0; i < NB && ok; ++i)
            ok = hipEventRecord(b->evs[stage * (NB + 1) + i], b->br[i]) == hipSuccess &&
                 hipStreamWaitEvent(b->cap, b->evs[stage * (NB + 1) + i], 0) == hipSuccess;
        return ok;
    };
    bool ok = fork(0);
    for (int p = 0; p < P && ok; ++p) {
        sisso_l0 *h = b->hs[p];
        Ctx c = h->ctx;
        c.ev = nullptr;  // no timing events inside a graph
        hipStream_t st = b->br[p % NB];
        ok = launch_stats(c, st) == 0 && launch_gram(c, st) == 0 &&
             (in_shared[p] ? launch_batch_prologue(c, b->calls[p], st) == 0 : launch_search(c, b->calls[p], st) == 0);
    }
    ok = ok && join(0);
    for (size_t q = 0; q < b->tables.size() && ok; ++q) ok = launch_batch_search3(b->tables[q], 0, b->cap) == 0;
    ok = ok && fork(1);
    for (size_t q = 0; q < shared.size() && ok; ++q) {
        const int p = shared[q];
        Ctx c = b->hs[p]->ctx;
        c.ev = nullptr;
        ok = launch_batch_epilogue(c, b->calls[p], b->br[q % NB]) == 0;
    }
    ok = ok && join(1);
    const hipError_t ec = hipStreamEndCapture(b->cap, &b->graph);
    if (!ok || ec != hipSuccess || !b->graph) return batch_fail(b, SISSO_EDEVICE, "graph capture failed");
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return batch_fail(b, SISSO_EDEVICE, "graph instantiation failed");
    *out = b;
    return SISSO_OK;
}

extern "C" int32_t sisso_l0_batch_launch(sisso_l0_batch *b) {
    if (!b) return SISSO_EINVAL;
    hipError_t e = hipEventRecord(b->in, b->user);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->cap);
    if (e == hipSuccess) e = hipEventRecord(b->out, b->cap);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->out, 0);
    if (e != hipSuccess) {
        g_batch_err = hipGetErrorString(e);
        return SISSO_EDEVICE;
    }
    for (size_t p = 0; p < b->hs.size(); ++p) {
        sisso_l0 *h = b->hs[p];
        h->gram_done = true;
        h->search_done = true;
        h->last_D = b->D;
        h->last_k = b->k;
        h->scored = b->scored[p];
        for (auto &r : h->ran) r = false;
    }
    return SISSO_OK;
}

extern "C" void sisso_l0_batch_destroy(sisso_l0_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->cap);
    delete b;
}

extern "C" const char *sisso_l0_batch_last_error(void) { return g_batch_err.c_str(); }

extern "C" int32_t sisso_l0_search_batch(sisso_l0 *const *hs, int32_t P, int32_t D, int32_t k) {
    sisso_l0_batch *b = nullptr;
    int32_t rc = sisso_l0_batch_create(hs, P, D, k, &b);
    if (rc != SISSO_OK) return rc;
    rc = sisso_l0_batch_launch(b);
    sisso_l0_batch_destroy(b);
    return rc;
}
