// Sure-independence screening, feature creation, residuals and exact top-m
// selection on gfx950.
//
// All kernels here stream feature columns from HBM: one wave owns one
// feature (or one candidate child pair) at a time and walks its samples
// lane-strided (64 consecutive doubles = one 512-byte coalesced load per
// step).  Reductions are wave butterflies in a fixed order, so every result
// is independent of the launch configuration.
#include <hip/hip_runtime.h>
#include <math.h>

#include <stdint.h>

#include "../../include/sisso_l0.h"
#include "../../include/sisso_sis.h"
#include "sis.h"

namespace sis {

constexpr int WAVE = 64;
constexpr double RANK_EPS = 1e-10;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
    return v;
}

// The operator, sample by sample (compile-time OP; OP_STORED reads a column).
constexpr int OP_STORED = -1;
template <int OP>
__device__ inline double apply(double a, double b) {
    if constexpr (OP == SISSO_OP_ADD) return a + b;
    else if constexpr (OP == SISSO_OP_SUB) return a - b;
    else if constexpr (OP == SISSO_OP_MUL) return a * b;
    else if constexpr (OP == SISSO_OP_DIV) return a / b;
    else if constexpr (OP == SISSO_OP_ABS_DIFF) return fabs(a - b);
    else if constexpr (OP == SISSO_OP_EXP) return exp(a);
    else if constexpr (OP == SISSO_OP_NEG_EXP) return exp(-a);
    else if constexpr (OP == SISSO_OP_LOG) return log(a);
    else if constexpr (OP == SISSO_OP_ABS) return fabs(a);
    else if constexpr (OP == SISSO_OP_SQRT) return sqrt(a);
    else if constexpr (OP == SISSO_OP_CBRT) return cbrt(a);
    else if constexpr (OP == SISSO_OP_SQ) return a * a;
    else if constexpr (OP == SISSO_OP_CB) return (a * a) * a;
    else if constexpr (OP == SISSO_OP_INV) return 1.0 / a;
    else if constexpr (OP == SISSO_OP_SIN) return sin(a);
    else if constexpr (OP == SISSO_OP_COS) return cos(a);
    else if constexpr (OP == SISSO_OP_SIX_POW) {
        const double c = (a * a) * a;
        return c * c;
    } else return a;
}

constexpr bool is_binary(int op) { return op >= 0 && op < 16; }

// Where a wave's samples come from: a stored column, or op over one or two
// child columns.
template <int OP>
struct Src {
    const double *a;
    const double *b;
    __device__ inline double at(int64_t i) const {
        if constexpr (OP == OP_STORED) return a[i];
        else if constexpr (is_binary(OP)) return apply<OP>(a[i], b[i]);
        else return apply<OP>(a[i], 0.0);
    }
};

// Resolve the source of item f; false if a child index is out of range.
template <int OP>
__device__ inline bool source(const double *X, int64_t n, int64_t Mc, const int32_t *pairs, int64_t f, Src<OP> &s) {
    if constexpr (OP == OP_STORED) {
        s.a = X + f * n;
        s.b = nullptr;
        return true;
    } else {
        const int32_t ia = pairs[2 * f], ib = pairs[2 * f + 1];
        if (ia < 0 || ia >= Mc) return false;
        if (is_binary(OP) && (ib < 0 || ib >= Mc)) return false;
        s.a = X + (int64_t)ia * n;
        s.b = is_binary(OP) ? X + (int64_t)ib * n : nullptr;
        return true;
    }
}

// ----------------------------------------------------------- value rules
// One wave per candidate: every value finite, max |v| in [lower, upper],
// not all values identical; optionally the values are written out.
template <int OP>
__global__ void __launch_bounds__(256) fc_eval_kernel(const double *__restrict__ X, int64_t n, int64_t Mc,
                                                      const int32_t *__restrict__ pairs, int64_t P, double lower,
                                                      double upper, double *__restrict__ out,
                                                      uint8_t *__restrict__ valid) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t f = wid; f < P; f += nw) {
        Src<OP> s;
        if (!source<OP>(X, n, Mc, pairs, f, s)) {
            if (lane == 0) valid[f] = 0;
            continue;
        }
        double amax = 0.0, vmin = INFINITY, vmax = -INFINITY;
        bool fin = true;
        double *o = out ? out + f * n : nullptr;
        for (int64_t i = lane; i < n; i += WAVE) {
            const double v = s.at(i);
            fin = fin && isfinite(v);
            amax = fmax(amax, fabs(v));
            vmin = fmin(vmin, v);
            vmax = fmax(vmax, v);
            if (o) o[i] = v;
        }
        const bool all_fin = __all(fin);
        amax = wave_max(amax);
        vmin = wave_min(vmin);
        vmax = wave_max(vmax);
        if (lane == 0) valid[f] = (all_fin && amax >= lower && amax <= upper && vmin != vmax) ? 1 : 0;
    }
}

// ------------------------------------------------------------- screening
// One lane per candidate feature, 64 candidates (a group) per wave.  The
// wave walks the samples of each task in tiles of SC_TS: its lanes load the
// group's 64 columns cooperatively (16 consecutive lanes read 16 consecutive
// samples of one column, a 128-byte segment; a group whose candidates share
// their first child reads that child's segment once), create the values
// (the operator, for created features) and write them transposed into a
// wave-private LDS tile; each lane then reads its own feature's 16 values
// back into registers.  The residuals are then taken residual by residual,
// 16 consecutive samples at a time, from addresses uniform across the wave:
// scalar operands, never waited for together with LDS reads.  No cross-lane
// reduction is needed: every sum is one lane's own.
//
// Per task, a feature's sums are shifted by its first sample K (u = v - K):
// su = sum u, suu = sum u^2, sur_r = sum u rho_r over the task's rows.  Then
// mean = K + su / n_t, the centred sum of squares is xss = suu - su^2 / n_t,
// and since every residual is centred over the task, the centred cross
// product is sur_r - (su / n_t) sum rho_r (the last sum is zero up to
// rounding).  The shift keeps the cancellation in xss to the ratio suu / xss
// = 1 + n_t (mean - K)^2 / xss <= 1 + n_t; where that ratio exceeds SC_REDO
// for some lane, the wave takes the task's sums again with those lanes
// shifted by their mean (the other lanes repeat the same arithmetic and get
// the same sums).
constexpr int SC_TS = 16;     // samples per tile
constexpr int SC_LD = 66;     // LDS row stride of a tile (doubles): conflict-free writes and reads
constexpr int SC_WPB = 4;     // waves per workgroup
constexpr double SC_REDO = 1024.0;

// The residual count of a kernel instantiation: nres rounded up to 1, 2, 4,
// 8, 10 or 16 (the padding residuals are zero).
__host__ __device__ constexpr int nr_pad(int nres) {
    return nres <= 1 ? 1 : nres <= 2 ? 2 : nres <= 4 ? 4 : nres <= 8 ? 8 : nres <= 10 ? 10 : 16;
}

// Load one tile: samples [s0, s0 + cnt) of the group's 64 columns.  Lane l
// fills sample s0 + (l & 15) of slot (l >> 4) + 4 q, q = 0..15.  ua >= 0:
// every slot's first child is column ua (read once per lane).
template <int OP>
__device__ inline void screen_load(const double *__restrict__ X, const int64_t *__restrict__ ca,
                                   const int64_t *__restrict__ cb, int64_t ua, int64_t s0, int cnt, double *tile,
                                   int lane) {
    const int s = lane & (SC_TS - 1);
    if (s >= cnt) return;
    if constexpr (is_binary(OP)) {
        if (ua >= 0) {
            const double a = X[ua + s0 + s];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int slot = (lane >> 4) + 4 * q;
                tile[s * SC_LD + slot] = apply<OP>(a, X[cb[slot] + s0 + s]);
            }
            return;
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int slot = (lane >> 4) + 4 * q;
        const double a = X[ca[slot] + s0 + s];
        double v;
        if constexpr (OP == OP_STORED) v = a;
        else if constexpr (is_binary(OP)) v = apply<OP>(a, X[cb[slot] + s0 + s]);
        else v = apply<OP>(a, 0.0);
        tile[s * SC_LD + slot] = v;
    }
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NR>
struct ScreenSums {
    double su, suu;
    double sur[NR];
};

// The sums over the tile samples [0, cnt) (all SC_TS when FULL).  rc:
// residual 0 at the tile's first sample, residual r at rc + r ldr; 16
// samples from there are always readable (rows are padded), and u = 0 past
// cnt adds nothing.  RULES: track the value rules.
template <int NR, bool RULES, bool FULL>
__device__ inline void screen_tile(const double *tile, int lane, const double *__restrict__ rc, int64_t ldr,
                                   int cnt, double K, ScreenSums<NR> &A, bool &fin, double &vmin, double &vmax) {
    double u[SC_TS];
#pragma unroll
    for (int j = 0; j < SC_TS; ++j) {
        u[j] = 0.0;
        if (FULL || j < cnt) {
            const double v = tile[j * SC_LD + lane];
            u[j] = v - K;
            A.su += u[j];
            A.suu = fma(u[j], u[j], A.suu);
            if constexpr (RULES) {
                fin = fin && isfinite(v);
                vmin = fmin(vmin, v);
                vmax = fmax(vmax, v);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const double *rr = rc + (int64_t)r * ldr;
#pragma unroll
        for (int j = 0; j < SC_TS; ++j) A.sur[r] = fma(u[j], rr[j], A.sur[r]);
    }
}

// One pass over the rows [r0, r1) of a task.  FIRST: K is set to the
// lane's first value and the value rules are tracked.
template <int OP, int NR, bool FIRST>
__device__ inline void screen_pass(const double *__restrict__ X, const int64_t *__restrict__ ca,
                                   const int64_t *__restrict__ cb, int64_t ua, int64_t r0, int64_t r1,
                                   const double *__restrict__ Rc, int64_t ldr, double *tile, int lane, double &K,
                                   ScreenSums<NR> &A, bool &fin, double &vmin, double &vmax) {
    constexpr bool RULES = FIRST && OP != OP_STORED;
    A.su = A.suu = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) A.sur[r] = 0.0;
    for (int64_t s0 = r0; s0 < r1; s0 += SC_TS) {
        const int cnt = (int)(r1 - s0 < SC_TS ? r1 - s0 : SC_TS);
        screen_load<OP>(X, ca, cb, ua, s0, cnt, tile, lane);
        wave_lds_sync();
        if (FIRST && s0 == r0) K = tile[lane];
        if (cnt == SC_TS)
            screen_tile<NR, RULES, true>(tile, lane, Rc + s0, ldr, cnt, K, A, fin, vmin, vmax);
        else
            screen_tile<NR, RULES, false>(tile, lane, Rc + s0, ldr, cnt, K, A, fin, vmin, vmax);
        wave_lds_sync();
    }
}

template <int OP, int NR>
__global__ void __launch_bounds__(256) screen_kernel(const double *__restrict__ X, int64_t n, int64_t Mc,
                                                     const int32_t *__restrict__ pairs, int64_t P,
                                                     const int64_t *__restrict__ off, int T,
                                                     const double *__restrict__ Rc, int64_t ldr,
                                                     const double *__restrict__ Rsum,
                                                     const double *__restrict__ Ctot, int nres, double lower,
                                                     double upper, double *__restrict__ scores,
                                                     uint8_t *__restrict__ valid) {
    __shared__ double tiles[SC_WPB][SC_TS * SC_LD];
    __shared__ int64_t cols[SC_WPB][2][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    double *tile = tiles[wv];
    int64_t *ca = cols[wv][0], *cb = cols[wv][1];
    const int64_t groups = (P + WAVE - 1) / WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * SC_WPB;
    for (int64_t g = (int64_t)blockIdx.x * SC_WPB + wv; g < groups; g += nwaves) {
        const int64_t f = g * WAVE + lane;
        // the lane's columns; a lane past P or with an index out of range
        // loads column 0 (Mc >= 1) and is not scored
        bool live = f < P, good = live;
        int64_t oa = 0, ob = 0;
        if (live) {
            if constexpr (OP == OP_STORED) {
                oa = f * n;
            } else {
                const int32_t ia = pairs[2 * f], ib = pairs[2 * f + 1];
                good = ia >= 0 && ia < Mc && (!is_binary(OP) || (ib >= 0 && ib < Mc));
                if (good) {
                    oa = (int64_t)ia * n;
                    ob = is_binary(OP) ? (int64_t)ib * n : 0;
                }
            }
        }
        ca[lane] = oa;
        cb[lane] = ob;
        // one first child for the whole group (the usual case of pair lists
        // in lexicographic order)
        const int64_t oa0 = __shfl(oa, 0, WAVE);
        const int64_t ua = (is_binary(OP) && __all(good && oa == oa0)) ? oa0 : -1;
        wave_lds_sync();
        double num[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) num[r] = 0.0;
        bool fin = true, flat = false, nonfinite = false;
        double vmin = INFINITY, vmax = -INFINITY;
        for (int t = 0; t < T; ++t) {
            const int64_t r0 = off[t], r1 = off[t + 1];
            const double nt = (double)(r1 - r0);
            ScreenSums<NR> A;
            double K = 0.0;
            screen_pass<OP, NR, true>(X, ca, cb, ua, r0, r1, Rc, ldr, tile, lane, K, A, fin, vmin, vmax);
            double mu = A.su / nt, xss = A.suu - A.su * mu;
            // heavy cancellation: the task again, around the mean
            const bool redo = good && isfinite(xss) && A.suu > SC_REDO * xss;
            if (__any(redo)) {
                if (redo) K += mu;
                screen_pass<OP, NR, false>(X, ca, cb, ua, r0, r1, Rc, ldr, tile, lane, K, A, fin, vmin, vmax);
                mu = A.su / nt;
                xss = A.suu - A.su * mu;
            }
            const double raw = A.suu + K * (2.0 * A.su + nt * K);  // sum of v^2
            if (!(isfinite(A.su) && isfinite(A.suu) && isfinite(K))) nonfinite = true;
            if (xss <= RANK_EPS * raw) flat = true;  // constant on this task
            const double inv = xss > 0.0 ? 1.0 / xss : 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double c = A.sur[r] - mu * Rsum[t * NR + r];
                num[r] = fma(c * c, inv, num[r]);
            }
        }
        if (live) {
            bool ok = fin && good;
            if constexpr (OP != OP_STORED) {
                const double amax = fmax(fabs(vmin), fabs(vmax));  // the largest |v|
                ok = ok && amax >= lower && amax <= upper && vmin != vmax;
            }
            double best = -INFINITY;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r < nres) {
                    const double c = Ctot[r];
                    best = fmax(best, c > 0.0 ? num[r] / c : 0.0);
                }
            }
            scores[f] = (ok && !flat && !nonfinite) ? best + 0.0 : __builtin_nan("");
            if (valid) valid[f] = ok ? 1 : 0;
        }
    }
}

// -------------------------------------------------- residual preparation
// One wave per (residual, task): rho_c = rho - mean over the task's rows,
// c = |rho_c|^2 into ctask[r * T + t] and the sum of rho_c (zero up to
// rounding) into rsum[t * NR + r].
__global__ void __launch_bounds__(256) centre_kernel(const double *__restrict__ R, int64_t n,
                                                     const int64_t *__restrict__ off, int T, int nres, int NR,
                                                     double *__restrict__ Rc, int64_t ldr,
                                                     double *__restrict__ ctask, double *__restrict__ rsum) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (w >= (int64_t)nres * T) return;
    const int r = (int)(w / T), t = (int)(w % T);
    const int64_t r0 = off[t], r1 = off[t + 1];
    const double *x = R + (int64_t)r * n;
    double *y = Rc + (int64_t)r * ldr;
    double sum = 0.0;
    for (int64_t i = r0 + lane; i < r1; i += WAVE) sum += x[i];
    const double mean = wave_sum(sum) / (double)(r1 - r0);
    double ss = 0.0, sc = 0.0;
    for (int64_t i = r0 + lane; i < r1; i += WAVE) {
        const double d = x[i] - mean;
        y[i] = d;
        ss += d * d;
        sc += d;
    }
    ss = wave_sum(ss);
    sc = wave_sum(sc);
    if (lane == 0) {
        ctask[w] = ss;
        rsum[t * NR + r] = sc;
    }
}

// The padding of the centred residuals: rows nres..NR-1, the SC_TS columns
// past n of every row, and the task sums of the padding rows, all zero.
__global__ void __launch_bounds__(256) pad_kernel(int64_t n, int64_t ldr, int T, int nres, int NR,
                                                  double *__restrict__ Rc, double *__restrict__ rsum) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < NR * ldr && (e / ldr >= nres || e % ldr >= n)) Rc[e] = 0.0;
    if (e < (int64_t)T * NR && (int)(e % NR) >= nres) rsum[e] = 0.0;
}

// Totals over tasks, in task order.
__global__ void ctot_kernel(const double *__restrict__ ctask, int T, int nres, double *__restrict__ ctot) {
    const int r = threadIdx.x;
    if (r >= nres) return;
    double c = 0.0;
    for (int t = 0; t < T; ++t) c += ctask[r * T + t];
    ctot[r] = c;
}

// -------------------------------------------------------------- residuals
// One thread per (sample, model): R[:, q] = y - (alpha + sum_d beta_d F[:, idx_d])
// of the sample's task, the sum in the order d = 0..D-1.
__global__ void __launch_bounds__(256) residual_kernel(const double *__restrict__ F, const double *__restrict__ y,
                                                       int64_t n, const int64_t *__restrict__ off, int T,
                                                       const int32_t *__restrict__ idx,
                                                       const double *__restrict__ coef, int D,
                                                       double *__restrict__ R) {
    const int q = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int t = 0;
        while (t + 1 < T && i >= off[t + 1]) ++t;
        const double *c = coef + ((int64_t)q * T + t) * (D + 1);
        double fit = c[0];
        for (int d = 0; d < D; ++d) fit += c[1 + d] * F[(int64_t)idx[q * D + d] * n + i];
        R[(int64_t)q * n + i] = y[i] - fit;
    }
}

// ---------------------------------------------------------- exact top-m
// Key of score s at index i: 96 bits, the order-preserving image of s in
// the top 64 bits and the complement of i in the low 32 (so among equal
// scores the lower index is larger).  Eight levels of 12-bit digits find
// the exact key of the m-th largest; every key at or above it is selected.
constexpr int TM_BITS = 12, TM_BINS = 1 << TM_BITS, TM_LEVELS = 8;

struct TopmState {
    uint32_t digit[TM_LEVELS];
    int64_t need;    // selections still to place among keys matching the digits so far
    int64_t finite;  // finite scores (level 0 total)
    uint32_t count;  // compaction counter
    uint32_t pad;
};

__device__ inline uint64_t order_key(double s) {
    const uint64_t u = (uint64_t)__double_as_longlong(s + 0.0);  // -0 -> +0
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline uint32_t digit_of(uint64_t hi, uint32_t lo, int L) {
    const int sh = 84 - TM_BITS * L;  // bit position of the digit's least significant bit
    if (sh >= 32) return (uint32_t)(hi >> (sh - 32)) & (TM_BINS - 1);
    if (sh == 24) return (uint32_t)(((hi & 0xfull) << 8) | (lo >> 24));
    return (lo >> sh) & (TM_BINS - 1);
}

__global__ void __launch_bounds__(1024) topm_hist_kernel(const double *__restrict__ sc, int64_t M, int L,
                                                         const TopmState *__restrict__ st,
                                                         unsigned int *__restrict__ hist) {
    __shared__ unsigned int h[TM_BINS];
    __shared__ uint32_t pre[TM_LEVELS];
    for (int b = threadIdx.x; b < TM_BINS; b += blockDim.x) h[b] = 0u;
    if (threadIdx.x < TM_LEVELS) pre[threadIdx.x] = st->digit[threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
        const double s = sc[i];
        if (!isfinite(s)) continue;
        const uint64_t hi = order_key(s);
        const uint32_t lo = ~(uint32_t)i;
        bool match = true;
        for (int l = 0; l < L; ++l) match = match && digit_of(hi, lo, l) == pre[l];
        if (match) atomicAdd(&h[digit_of(hi, lo, L)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < TM_BINS; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// One workgroup of TM_THREADS: the level's digit is the bin b with
// I[b] >= need > I[b + 1], I[b] = sum of hist[b'] over b' >= b (inclusive
// suffix count; I[TM_BINS] = 0): the bin that holds the need-th largest
// matching key.  Level 0 first sets need = min(m, number of finite scores).
// Each thread sums 4 consecutive bins; the suffix sums of those partial
// sums are a Hillis-Steele scan in LDS.
constexpr int TM_THREADS = TM_BINS / 4;
__global__ void __launch_bounds__(TM_THREADS) topm_digit_kernel(const unsigned int *__restrict__ hist, int L,
                                                                int64_t m, TopmState *__restrict__ st) {
    __shared__ int64_t part[2][TM_THREADS];
    const int t = threadIdx.x;
    int64_t h[4], own = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = hist[4 * t + q];
        own += h[q];
    }
    // suffix scan: part[.][t] = sum of own over threads >= t
    int cur = 0;
    part[0][t] = own;
    __syncthreads();
    for (int d = 1; d < TM_THREADS; d <<= 1) {
        const int64_t v = part[cur][t] + (t + d < TM_THREADS ? part[cur][t + d] : 0);
        part[cur ^ 1][t] = v;
        cur ^= 1;
        __syncthreads();
    }
    const int64_t total = part[cur][0];
    const int64_t above = part[cur][t] - own;  // I[4 t + 4]
    const int64_t need = L == 0 ? (m < total ? m : total) : st->need;
    __syncthreads();
    int64_t I = above;
#pragma unroll
    for (int q = 3; q >= 0; --q) {
        const int64_t below = I;  // I[4 t + q + 1]
        I += h[q];                // I[4 t + q]
        const int b = 4 * t + q;
        // need <= 0 (nothing left to place) keeps the top bin, as in a
        // serial scan from the top that stops at once
        const bool pick = need > 0 ? (I >= need && below < need) || (b == 0 && I < need) : b == TM_BINS - 1;
        if (pick) {
            st->digit[L] = (uint32_t)b;
            st->need = need - (need > 0 ? below : 0);
            if (L == 0) st->finite = total;
        }
    }
}

__global__ void topm_init_kernel(TopmState *__restrict__ st, unsigned int *__restrict__ hist) {
    if (threadIdx.x < TM_LEVELS) st->digit[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        st->need = 0;
        st->finite = 0;
        st->count = 0u;
    }
    for (int b = threadIdx.x; b < TM_BINS; b += blockDim.x) hist[b] = 0u;
}

__global__ void topm_clear_kernel(unsigned int *__restrict__ hist) {
    for (int b = threadIdx.x; b < TM_BINS; b += blockDim.x) hist[b] = 0u;
}

// Every finite key >= the selected key (compared digit by digit from the
// top) is appended to the candidate list.
__global__ void __launch_bounds__(1024) topm_compact_kernel(const double *__restrict__ sc, int64_t M,
                                                            TopmState *__restrict__ st, double *__restrict__ csc,
                                                            int64_t *__restrict__ cidx, int64_t cap) {
    __shared__ uint32_t pre[TM_LEVELS];
    if (threadIdx.x < TM_LEVELS) pre[threadIdx.x] = st->digit[threadIdx.x];
    __syncthreads();
    if (st->finite == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
        const double s = sc[i];
        if (!isfinite(s)) continue;
        const uint64_t hi = order_key(s);
        const uint32_t lo = ~(uint32_t)i;
        int cmp = 0;
        for (int l = 0; l < TM_LEVELS && cmp == 0; ++l) {
            const uint32_t d = digit_of(hi, lo, l);
            cmp = d > pre[l] ? 1 : (d < pre[l] ? -1 : 0);
        }
        if (cmp >= 0) {
            const uint32_t at = atomicAdd(&st->count, 1u);
            if ((int64_t)at < cap) {
                csc[at] = s + 0.0;
                cidx[at] = i;
            }
        }
    }
}

// Rank of each candidate = candidates with a larger (score, -index) key;
// one wave per candidate, its lanes striding over the others.
__global__ void __launch_bounds__(256) topm_rank_kernel(const double *__restrict__ csc,
                                                        const int64_t *__restrict__ cidx,
                                                        const TopmState *__restrict__ st, int64_t cap,
                                                        int64_t *__restrict__ out_idx, double *__restrict__ out_sc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t cnt = (int64_t)st->count < cap ? (int64_t)st->count : cap;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (e >= cnt) return;
    const double s = csc[e];
    const int64_t ix = cidx[e];
    int64_t rank = 0;
    for (int64_t j = lane; j < cnt; j += WAVE) {
        const double sj = csc[j];
        rank += (sj > s || (sj == s && cidx[j] < ix)) ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rank += __shfl_xor(rank, o, WAVE);
    if (lane == 0) {
        out_idx[rank] = ix;
        if (out_sc) out_sc[rank] = s;
    }
}

// ----------------------------------------------------- dimension-loop glue
__global__ void mask_kernel(const int32_t *__restrict__ sel, int64_t ns, double *__restrict__ scores) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) scores[sel[i]] = __builtin_nan("");
}

__global__ void __launch_bounds__(256) gather_kernel(const double *__restrict__ X, int64_t n,
                                                     const int32_t *__restrict__ sel, int64_t first, int64_t count,
                                                     double *__restrict__ Fs) {
    for (int64_t c = blockIdx.y; c < count; c += gridDim.y) {
        const double *src = X + (int64_t)sel[first + c] * n;
        double *dst = Fs + (first + c) * n;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            dst[i] = src[i];
    }
}

__global__ void narrow_kernel(const int64_t *__restrict__ in, int64_t m, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = (int32_t)in[i];
}

// ------------------------------------------------------------- launchers
static unsigned grid_for(int64_t items, int per_block) {
    const int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <int OP, int NR>
static void launch_screen_nr(const ScoreArgs &a, hipStream_t st) {
    const int64_t groups = (a.P + WAVE - 1) / WAVE;
    hipLaunchKernelGGL((screen_kernel<OP, NR>), dim3(grid_for(groups, SC_WPB)), dim3(SC_WPB * WAVE), 0, st, a.X, a.n,
                       a.Mc, a.pairs, a.P, a.off, a.T, a.Rc, a.ldr, a.Rsum, a.Ctot, a.nres, a.lower, a.upper,
                       a.scores, a.valid);
}

template <int OP>
static void launch_score_op(const ScoreArgs &a, hipStream_t st) {
    switch (nr_pad(a.nres)) {
        case 1: launch_screen_nr<OP, 1>(a, st); break;
        case 2: launch_screen_nr<OP, 2>(a, st); break;
        case 4: launch_screen_nr<OP, 4>(a, st); break;
        case 8: launch_screen_nr<OP, 8>(a, st); break;
        case 10: launch_screen_nr<OP, 10>(a, st); break;
        default: launch_screen_nr<OP, 16>(a, st); break;
    }
}

template <int OP>
static void launch_fc_op(const FcArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((fc_eval_kernel<OP>), dim3(grid_for(a.P, 4)), dim3(256), 0, st, a.X, a.n, a.Mc, a.pairs, a.P,
                       a.lower, a.upper, a.out, a.valid);
}

#define SIS_OP_CASES(M)                                                                                   \
    M(SISSO_OP_ADD) M(SISSO_OP_SUB) M(SISSO_OP_MUL) M(SISSO_OP_DIV) M(SISSO_OP_ABS_DIFF) M(SISSO_OP_EXP) \
    M(SISSO_OP_NEG_EXP) M(SISSO_OP_LOG) M(SISSO_OP_ABS) M(SISSO_OP_SQRT) M(SISSO_OP_CBRT) M(SISSO_OP_SQ) \
    M(SISSO_OP_CB) M(SISSO_OP_INV) M(SISSO_OP_SIN) M(SISSO_OP_COS) M(SISSO_OP_SIX_POW)

bool op_known(int op) {
    switch (op) {
#define SIS_CASE(O) case O:
        SIS_OP_CASES(SIS_CASE) return true;
#undef SIS_CASE
        default: return false;
    }
}

int launch_score(int op, const ScoreArgs &a, hipStream_t st) {
    switch (op) {
        case OP_STORED: launch_score_op<OP_STORED>(a, st); break;
#define SIS_CASE(O) \
    case O: launch_score_op<O>(a, st); break;
        SIS_OP_CASES(SIS_CASE)
#undef SIS_CASE
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fc(int op, const FcArgs &a, hipStream_t st) {
    switch (op) {
#define SIS_CASE(O) \
    case O: launch_fc_op<O>(a, st); break;
        SIS_OP_CASES(SIS_CASE)
#undef SIS_CASE
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_centre(const double *R, int64_t n, const int64_t *off, int T, int nres, double *Rc, double *ctask,
                  double *ctot, double *rsum, hipStream_t st) {
    const int NR = nr_pad(nres);
    const int64_t ldr = residual_stride(n);
    const int64_t waves = (int64_t)nres * T;
    hipLaunchKernelGGL(centre_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, R, n, off, T, nres, NR, Rc,
                       ldr, ctask, rsum);
    hipLaunchKernelGGL(ctot_kernel, dim3(1), dim3(64), 0, st, ctask, T, nres, ctot);
    const int64_t e = NR * ldr > (int64_t)T * NR ? NR * ldr : (int64_t)T * NR;
    hipLaunchKernelGGL(pad_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, n, ldr, T, nres, NR, Rc, rsum);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int64_t residual_stride(int64_t n) { return n + SC_TS; }

int residual_width(int nres) { return nr_pad(nres); }

int launch_residuals(const double *F, const double *y, int64_t n, const int64_t *off, int T, const int32_t *idx,
                     const double *coef, int r, int D, double *R, hipStream_t st) {
    const unsigned gx = grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024;
    hipLaunchKernelGGL(residual_kernel, dim3(gx, (unsigned)r), dim3(256), 0, st, F, y, n, off, T, idx, coef, D, R);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t topm_ws_bytes(int64_t M, int m) {
    (void)M;
    const size_t a = 256 + TM_BINS * sizeof(unsigned int);
    return a + (size_t)m * (sizeof(double) + sizeof(int64_t)) + 256;
}

int launch_topm(const double *sc, int64_t M, int m, int64_t *out_idx, double *out_sc, void *ws, hipStream_t st,
                uint32_t **count_dev) {
    char *base = (char *)ws;
    TopmState *state = (TopmState *)base;
    unsigned int *hist = (unsigned int *)(base + 256);
    double *csc = (double *)(base + 256 + TM_BINS * sizeof(unsigned int));
    int64_t *cidx = (int64_t *)(csc + m);
    static_assert(sizeof(TopmState) <= 256, "state slot");
    const unsigned grid = grid_for(M, 1024) < 2048 ? grid_for(M, 1024) : 2048;
    hipLaunchKernelGGL(topm_init_kernel, dim3(1), dim3(1024), 0, st, state, hist);
    for (int L = 0; L < TM_LEVELS; ++L) {
        if (L > 0) hipLaunchKernelGGL(topm_clear_kernel, dim3(1), dim3(1024), 0, st, hist);
        hipLaunchKernelGGL(topm_hist_kernel, dim3(grid), dim3(1024), 0, st, sc, M, L, state, hist);
        hipLaunchKernelGGL(topm_digit_kernel, dim3(1), dim3(TM_THREADS), 0, st, hist, L, (int64_t)m, state);
    }
    hipLaunchKernelGGL(topm_compact_kernel, dim3(grid), dim3(1024), 0, st, sc, M, state, csc, cidx, (int64_t)m);
    hipLaunchKernelGGL(topm_rank_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, csc, cidx, state,
                       (int64_t)m, out_idx, out_sc);
    *count_dev = &state->count;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mask(const int32_t *sel, int64_t ns, double *scores, hipStream_t st) {
    if (ns < 1) return 0;
    hipLaunchKernelGGL(mask_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, sel, ns, scores);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gather(const double *X, int64_t n, const int32_t *sel, int64_t first, int64_t count, double *Fs,
                  hipStream_t st) {
    if (count < 1) return 0;
    const unsigned gx = grid_for(n, 256) < 64 ? grid_for(n, 256) : 64;
    const unsigned gy = (unsigned)(count < 4096 ? count : 4096);
    hipLaunchKernelGGL(gather_kernel, dim3(gx, gy), dim3(256), 0, st, X, n, sel, first, count, Fs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_narrow(const int64_t *in, int64_t m, int32_t *out, hipStream_t st) {
    if (m < 1) return 0;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, in, m, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sis
