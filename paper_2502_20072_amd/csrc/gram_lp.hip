// Precision forms of the Gram step: BF16 or FP16 slices on MFMA with FP32
// chunk sums and FP64 accumulation.
//
// Each centred column x of a task is cut, per chunk of LP_XC consecutive
// samples, into NS slices of small integers that the element type holds
// exactly (SB significant bits: 8 for BF16, 11 for FP16):
//     x = 2^(e - (SB-1)) (a_0 + a_1 2^-SB + a_2 2^-2SB + ...),  |a_s| <= 2^(SB-1),
// with 2^e > max |x| over the chunk (a_0 = rint(x 2^(SB-1-e)), each further
// slice the rounded, 2^SB-scaled remainder).  The cross products
//     sum_k x_i[k] x_j[k] = 2^(e_i + e_j - 2(SB-1)) sum_m 2^(-SB m) P_m,
//     P_m = sum_k sum_{s+u=m} a_s(i,k) a_u(j,k),
// keep the slice pairs with s + u < NS, accumulated in the FP32 accumulators
// of the MFMA over a chunk; only the chunk totals are scaled and summed in
// FP64 (the compensating FP64 sum).
//  * BF16, NS = 3 (six products per K-step): every term of P_m is an integer
//    of magnitude <= 2^14, a chunk holds at most 256 samples and at most 3
//    pairs per m, so P_m (< 2^24) is exact in FP32.  The result differs from
//    the FP64 Gram only by the dropped slice pairs and the truncation of x to
//    three slices (~2^-20 M_i M_j per sample, M the chunk maxima).
//  * FP16, NS = 2 (three products per K-step, half the BF16 work): 22 bits of
//    each value; terms up to 2^20, so the FP32 chunk sums round (a few ulps
//    of sums below 2^29 per chunk), and the truncation and the dropped
//    product leave ~2^-18 M_i M_j per sample.
// F^T y and |y|^2 stay exact FP64 (statistics kernel); the search and the
// re-score are unchanged.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sl0 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int LP_BK = 32;        // MFMA K (samples per K-step)
constexpr int LP_TILE = 128;     // output tile per workgroup
constexpr int LP_ROW = LP_BK + 8;  // LDS row stride in BF16 elements (80 B: conflict-free 16-B reads)
constexpr int LP_WG = 512;       // threads per Gram workgroup (8 waves)
constexpr int LP_WN = 2;         // 16-column blocks per wave (64 x 32 per wave)

// ------------------------------------------------------------------ slices
// One wavefront per (feature j, chunk g).  Chunks tile every task's rows in
// LP_XC-sample pieces (a task's last chunk is zero-padded).  Writes the
// chunk exponent and the NS slices of the centred samples.
template <typename E, int SB>
__global__ __launch_bounds__(256) void slice_kernel(Ctx c, int NS) {
    const int lane = threadIdx.x & 63;
    const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= c.S * c.lp_nchunk) return;
    const int64_t j = job / c.lp_nchunk;
    const int g = (int)(job % c.lp_nchunk);
    int t = 0;
    while (t + 1 < c.T && c.lp_cbase[t + 1] <= g) ++t;
    const int64_t r0 = c.off_dev[t], r1 = c.off_dev[t + 1];
    const int64_t row0 = r0 + (int64_t)(g - c.lp_cbase[t]) * LP_XC;
    const double m = c.mu[(int64_t)t * c.S + j];
    const double *col = c.F + j * c.n_total;
    constexpr int PER = LP_XC / 64;
    double x[PER];
    double mx = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int64_t i = row0 + lane + 64 * q;
        x[q] = i < r1 ? col[i] - m : 0.0;
        mx = fmax(mx, fabs(x[q]));
    }
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    const int e = mx > 0.0 ? ilogb(mx) + 1 : 0;  // 2^e > max |x|
    if (lane == 0) c.lp_exp[j * c.lp_nchunk + g] = e;
    const int64_t np = (int64_t)c.lp_nchunk * LP_XC;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        double r = ldexp(x[q], SB - 1 - e);
        E *sl = reinterpret_cast<E *>(c.lp_slices);
        for (int s = 0; s < NS; ++s) {
            const double a = rint(r);
            sl[((int64_t)s * c.S + j) * np + (int64_t)g * LP_XC + lane + 64 * q] = (E)(float)a;
            r = (r - a) * (double)(1 << SB);
        }
    }
}

// ------------------------------------------------------------ Gram tiles
// One workgroup (8 waves) per (split, task, 128x128 tile pair bi <= bj); each
// wave owns a 64x32 piece as 4x2 blocks of 16x16, with the FP32 sums of every
// slice order m and the FP64 accumulators in registers.  K-steps of 32 samples
// are staged through LDS (all NS slices of both operands; a diagonal tile
// loads one operand); every LP_XC samples the FP32 sums P_m are scaled by the
// chunk exponents and added to FP64 accumulators.  Writes raw centred sums
// to part[split][t][S][S], like the FP64 path.
//
// v_mfma_f32_16x16x32_bf16 operands: A[i][k] in lane i + 16 (k / 8), element
// k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; result D[i][j] in lane
// j + 16 (i / 4), register i % 4.
template <typename E, int NS, int SB>
__global__ __launch_bounds__(LP_WG) void gram_lp_kernel(Ctx c, int ntile, int nsplit) {
    typedef E ex8 __attribute__((ext_vector_type(8)));
    __shared__ __attribute__((aligned(16))) E As[NS][LP_TILE][LP_ROW];
    __shared__ __attribute__((aligned(16))) E Bs[NS][LP_TILE][LP_ROW];
    __shared__ int es[2 * LP_TILE];

    int64_t b = blockIdx.x;
    const int npair = ntile * (ntile + 1) / 2;
    const int split = (int)(b / ((int64_t)c.T * npair));
    b -= (int64_t)split * c.T * npair;
    const int t = (int)(b / npair);
    int pr = (int)(b - (int64_t)t * npair);
    int bi = 0;
    while (pr >= ntile - bi) {
        pr -= ntile - bi;
        ++bi;
    }
    const int bj = bi + pr;
    const bool diag = bi == bj;

    const int g0t = c.lp_cbase[t], g1t = c.lp_cbase[t + 1];
    const int per = (g1t - g0t + nsplit - 1) / nsplit;
    const int g0 = g0t + split * per;
    const int g1 = g0 + per < g1t ? g0 + per : g1t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
    const int64_t np = (int64_t)c.lp_nchunk * LP_XC;

    // loader: 16-byte pieces (8 samples); thread tid loads pieces tid and
    // tid + LP_WG of every slice of both operands (piece p: feature p / 4,
    // samples 8 (p % 4) of the K-step).  Rows past S load row S - 1 (their
    // outputs are not stored).  Loads are unconditional so none is waited on
    // before the MFMAs; a diagonal tile loads its panel twice (the second
    // read hits the cache).
    constexpr int PPT = LP_TILE * 4 / LP_WG;
    const E *pa[PPT], *pb[PPT];  // slice 0 of each piece; slice s is s * sstride further
    const E *slices = reinterpret_cast<const E *>(c.lp_slices);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int p = tid + LP_WG * q;
        int64_t fa = (int64_t)bi * LP_TILE + (p >> 2), fb = (int64_t)bj * LP_TILE + (p >> 2);
        fa = fa < c.S ? fa : c.S - 1;
        fb = fb < c.S ? fb : c.S - 1;
        pa[q] = slices + fa * np + 8 * (p & 3);
        pb[q] = slices + fb * np + 8 * (p & 3);
    }
    const int64_t sstride = c.S * np;
    ex8 ra[NS][PPT], rb[NS][PPT];
    auto load_step = [&](int64_t k0) {  // k0: first sample of the K-step (multiple of 32)
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                ra[s][q] = *reinterpret_cast<const ex8 *>(pa[q] + s * sstride + k0);
                rb[s][q] = *reinterpret_cast<const ex8 *>(pb[q] + s * sstride + k0);
            }
    };
    auto store_step = [&]() {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int p = tid + LP_WG * q;
                *reinterpret_cast<ex8 *>(&As[s][p >> 2][8 * (p & 3)]) = ra[s][q];
                *reinterpret_cast<ex8 *>(&Bs[s][p >> 2][8 * (p & 3)]) = rb[s][q];
            }
    };
    (void)diag;
    E (*Bsrc)[LP_TILE][LP_ROW] = Bs;

    double4_t acc[4][LP_WN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < LP_WN; ++n) acc[m][n] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const int ksteps = LP_XC / LP_BK;
    const int64_t nsteps = (int64_t)(g1 - g0) * ksteps;
    if (nsteps > 0) {
        load_step((int64_t)g0 * LP_XC);
        store_step();
    }
    for (int g = g0; g < g1; ++g) {
        // chunk exponents of the tile's rows (A) and columns (B); the barrier
        // keeps them from overwriting those the last promotion still reads
        __syncthreads();
        if (tid < 2 * LP_TILE) {
            const int blk = tid < LP_TILE ? bi : bj;
            int64_t f = (int64_t)blk * LP_TILE + (tid & (LP_TILE - 1));
            es[tid] = f < c.S ? c.lp_exp[f * c.lp_nchunk + g] : 0;
        }
        f32x4 p32[NS][4][LP_WN];
#pragma unroll
        for (int mm = 0; mm < NS; ++mm)
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < LP_WN; ++n) p32[mm][m][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < ksteps; ++ks) {
            __syncthreads();
            const int64_t step = (int64_t)(g - g0) * ksteps + ks;
            const bool more = step + 1 < nsteps;
            if (more) load_step((int64_t)g0 * LP_XC + (step + 1) * LP_BK);
            const int kr = 8 * (lane >> 4);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                ex8 av[4];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    av[m] = *reinterpret_cast<const ex8 *>(&As[s][wr + 16 * m + (lane & 15)][kr]);
#pragma unroll
                for (int u = 0; u + s < NS; ++u) {
                    ex8 bv[LP_WN];
#pragma unroll
                    for (int n = 0; n < LP_WN; ++n)
                        bv[n] = *reinterpret_cast<const ex8 *>(&Bsrc[u][wc + 16 * n + (lane & 15)][kr]);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int n = 0; n < LP_WN; ++n) {
                            if constexpr (std::is_same<E, _Float16>::value)
                                p32[s + u][m][n] =
                                    __builtin_amdgcn_mfma_f32_16x16x32_f16(av[m], bv[n], p32[s + u][m][n], 0, 0, 0);
                            else
                                p32[s + u][m][n] =
                                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[n], p32[s + u][m][n], 0, 0, 0);
                        }
                }
            }
            __syncthreads();
            if (more) store_step();
        }
        // promote the chunk sums: acc += 2^(e_i + e_j - 2(SB-1)) sum_m 2^(-SB m) P_m
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < LP_WN; ++n) {
                const int ej = es[LP_TILE + wc + 16 * n + (lane & 15)];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ei = es[wr + 16 * m + 4 * (lane >> 4) + r];
                    double v = (double)p32[NS - 1][m][n][r];
#pragma unroll
                    for (int mm = NS - 2; mm >= 0; --mm) v = fma(v, 1.0 / (double)(1 << SB), (double)p32[mm][m][n][r]);
                    acc[m][n][r] += ldexp(v, ei + ej - 2 * (SB - 1));
                }
            }
    }

    double *P = c.part + ((int64_t)split * c.T + t) * c.S * c.S;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < LP_WN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = (int64_t)bi * LP_TILE + wr + 16 * m + 4 * (lane >> 4) + r;
                const int64_t gj = (int64_t)bj * LP_TILE + wc + 16 * n + (lane & 15);
                if (gi < c.S && gj < c.S) P[gi * c.S + gj] = acc[m][n][r];
            }
}

// ------------------------------------------------------ sampled error check
// Max |G_lp - G_fp64| over sampled entries of every task: entry e picks
// (i, j) by a fixed multiplicative hash; the FP64 value is the centred dot
// product straight from F, scaled like the stored matrix.  One wavefront per
// (entry, task).
__global__ __launch_bounds__(256) void gram_check_kernel(Ctx c, int nsample, unsigned long long *out_bits) {
    const int lane = threadIdx.x & 63;
    const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= (int64_t)nsample * c.T) return;
    const int e = (int)(job / c.T);
    const int t = (int)(job % c.T);
    const uint64_t h = (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
    const int64_t i = (int64_t)((h >> 20) % (uint64_t)c.S);
    const int64_t j = (int64_t)((h >> 40) % (uint64_t)c.S);
    const int64_t r0 = c.off_dev[t], r1 = c.off_dev[t + 1];
    const double mi = c.mu[(int64_t)t * c.S + i], mj = c.mu[(int64_t)t * c.S + j];
    double s = 0.0;
    for (int64_t r = r0 + lane; r < r1; r += 64) s += (c.F[i * c.n_total + r] - mi) * (c.F[j * c.n_total + r] - mj);
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
        const double is = c.inv_s[(int64_t)t * c.S + i], js = c.inv_s[(int64_t)t * c.S + j];
        const double ref = i == j ? (is > 0.0 ? 1.0 : 0.0) : s * is * js;
        const double got = c.G[gidx(i, j, c.Gnt, c.TP, t)];
        const double d = fabs(got - ref);
        atomicMax(out_bits, (unsigned long long)__double_as_longlong(d));
    }
}

int launch_gram_lp(const Ctx &c, int NS, hipStream_t st) {
    const int64_t jobs = c.S * c.lp_nchunk;
    const int ntile = (int)((c.S + LP_TILE - 1) / LP_TILE);
    const int64_t blocks = (int64_t)c.nsplit * c.T * ntile * (ntile + 1) / 2;
    const dim3 sgrid((unsigned)((jobs + 3) / 4));
    // the slice count names the form: three BF16 slices or two FP16 slices
    switch (NS) {
        case 3:
            hipLaunchKernelGGL((slice_kernel<__bf16, 8>), sgrid, dim3(256), 0, st, c, NS);
            hipLaunchKernelGGL((gram_lp_kernel<__bf16, 3, 8>), dim3((unsigned)blocks), dim3(LP_WG), 0, st, c, ntile,
                               c.nsplit);
            break;
        case 2:
            hipLaunchKernelGGL((slice_kernel<_Float16, 11>), sgrid, dim3(256), 0, st, c, NS);
            hipLaunchKernelGGL((gram_lp_kernel<_Float16, 2, 11>), dim3((unsigned)blocks), dim3(LP_WG), 0, st, c,
                               ntile, c.nsplit);
            break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gram_check(const Ctx &c, int nsample, unsigned long long *out_bits, hipStream_t st) {
    const int64_t jobs = (int64_t)nsample * c.T;
    hipLaunchKernelGGL(gram_check_kernel, dim3((unsigned)((jobs + 3) / 4)), dim3(256), 0, st, c, nsample, out_bits);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sl0
