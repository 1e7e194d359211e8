// Per-task column statistics and the centred Gram precompute (FP64 MFMA).
//
// Every least-squares system the l0 step solves is the normal-equation
// system of [1, x_i1, ..., x_iD] against y on the rows of one task.
// Eliminating the intercept first leaves the centred cross-products, so all
// systems are sub-matrices of G_t = X_tc^T X_tc, b_t = X_tc^T y_tc and
// c_t = |y_tc|^2 (X_tc: columns of task t minus their means).  These are
// computed once here; the search never touches F again.  G_t is stored as a
// correlation matrix (scaled by 1/|x_i - mean| on both sides, unit diagonal),
// which leaves every SSE unchanged and makes pivot ratios plain pivots.
#include "common.h"
#include "kernels.h"

namespace sl0 {

// ---------------------------------------------------------------- a0: stats
// One wavefront per (feature j or the target, task t).  Sums run over the
// task's rows with a fixed lane-strided order (lane l adds rows r0 + l + 64 u
// in increasing u) and a fixed butterfly, so the result does not depend on
// scheduling.  Both sums are two-pass: the mean first, then the centred
// moments.  With VPT > 0 (every task at most 64 VPT rows; VPT is the
// smallest power of two from 2 to SX_VPT that covers the largest task) a
// lane loads its rows, and the target's, once into registers with all loads
// in flight together, and both passes run on the registers: one memory round
// trip per column instead of one per few rows.  With VPT = 0 both passes
// stream the column.  The order of the additions is the same in every form,
// so their results agree bit for bit.
__device__ inline double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

constexpr int SX_VPT = 32;  // most rows per lane held in registers (tasks of up to 2048 rows)

// One workgroup: clears the status words, then wave w handles tasks w,
// w + 4, ... (so no other workgroup can set a status bit before the clear).
// Last, it names the filter tasks: the tasks of largest and second largest
// c_t (the first such; -1 for the second when T = 1), whose SSEs bound any
// tuple's SSE summed over tasks from below.
template <int VPT>
__global__ __launch_bounds__(256) void stats_y_kernel(const double *__restrict__ y,
                                                      const int64_t *__restrict__ off, int T,
                                                      double *__restrict__ ybar,
                                                      double *__restrict__ cyy,
                                                      uint32_t *__restrict__ flags,
                                                      int32_t *__restrict__ tstar) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) flags[threadIdx.x] = 0u;
    __syncthreads();
    for (int t = threadIdx.x >> 6; t < T; t += 4) {
        const int64_t r0 = off[t], r1 = off[t + 1];
        double s = 0.0, ss = 0.0, m;
        bool bad = false;
        if constexpr (VPT > 0) {
            double v[VPT];
#pragma unroll
            for (int u = 0; u < VPT; ++u) {
                const int64_t i = r0 + lane + 64 * u;
                v[u] = i < r1 ? y[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < VPT; ++u) {
                if (r0 + lane + 64 * u < r1) {
                    bad |= !isfinite(v[u]);
                    s += v[u];
                }
            }
            s = wave_sum(s);
            m = s / (double)(r1 - r0);
#pragma unroll
            for (int u = 0; u < VPT; ++u) {
                if (r0 + lane + 64 * u < r1) {
                    const double d = v[u] - m;
                    ss += d * d;
                }
            }
        } else {
#pragma unroll 8
            for (int64_t i = r0 + lane; i < r1; i += 64) {
                const double v = y[i];
                bad |= !isfinite(v);
                s += v;
            }
            s = wave_sum(s);
            m = s / (double)(r1 - r0);
#pragma unroll 8
            for (int64_t i = r0 + lane; i < r1; i += 64) {
                const double d = y[i] - m;
                ss += d * d;
            }
        }
        ss = wave_sum(ss);
        if (__any(bad) && lane == 0) atomicOr(&flags[FLAG_NONFINITE], 1u);
        if (lane == 0) {
            ybar[t] = m;
            cyy[t] = ss;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = 0, second = -1;
        for (int t = 1; t < T; ++t) {
            if (cyy[t] > cyy[best]) {
                second = best;
                best = t;
            } else if (second < 0 || cyy[t] > cyy[second]) {
                second = t;
            }
        }
        tstar[0] = best;
        tstar[1] = second;
    }
}

template <int VPT>
__global__ __launch_bounds__(256) void stats_x_kernel(const double *__restrict__ F,
                                                      const double *__restrict__ y,
                                                      const int64_t *__restrict__ off,
                                                      int64_t n_total, int64_t S, int T, int TP,
                                                      const double *__restrict__ ybar,
                                                      double *__restrict__ mu,
                                                      double *__restrict__ inv_s,
                                                      double *__restrict__ bhat,
                                                      uint32_t *__restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= S * T) return;
    const int64_t j = job / T;
    const int t = (int)(job % T);
    const int64_t r0 = off[t], r1 = off[t + 1];
    const double *col = F + j * n_total;
    const double ym = ybar[t];
    double s = 0.0, ss = 0.0, sy = 0.0, sr = 0.0, m;
    bool bad = false;
    if constexpr (VPT > 0) {
        double v[VPT], w[VPT];
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int64_t i = r0 + lane + 64 * u;
            v[u] = i < r1 ? col[i] : 0.0;
            w[u] = i < r1 ? y[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            if (r0 + lane + 64 * u < r1) {
                bad |= !isfinite(v[u]);
                s += v[u];
            }
        }
        s = wave_sum(s);
        m = s / (double)(r1 - r0);
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            if (r0 + lane + 64 * u < r1) {
                const double d = v[u] - m;
                ss += d * d;
                sy += d * (w[u] - ym);
                sr += v[u] * v[u];
            }
        }
    } else {
#pragma unroll 8
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            const double v = col[i];
            bad |= !isfinite(v);
            s += v;
        }
        s = wave_sum(s);
        m = s / (double)(r1 - r0);
#pragma unroll 8
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            const double v = col[i];
            const double d = v - m;
            ss += d * d;
            sy += d * (y[i] - ym);
            sr += v * v;
        }
    }
    ss = wave_sum(ss);
    sy = wave_sum(sy);
    sr = wave_sum(sr);
    if (__any(bad) && lane == 0) atomicOr(&flags[FLAG_NONFINITE], 1u);
    if (lane == 0) {
        // a column constant on the task up to RANK_EPS (1 - uncentred R^2 on
        // the intercept: |x - mean|^2 <= RANK_EPS |x|^2) is treated as
        // constant: its centred values would be rounding noise
        const bool live = ss > RANK_EPS * sr && isfinite(ss);
        const double is = live ? 1.0 / sqrt(ss) : 0.0;
        mu[(int64_t)t * S + j] = m;
        inv_s[(int64_t)t * S + j] = is;
        bhat[j * TP + t] = sy * is;
    }
}

// ------------------------------------------------------- a1: Gram on MFMA
// One workgroup (4 waves) computes a GRAM_TILE x GRAM_TILE block (bi <= bj)
// of the centred Gram of one task over one split of its rows; each wave owns
// a 64x64 quarter as 4x4 MFMA 16x16 accumulators.  Samples are staged through
// LDS in chunks of GRAM_KC, centred on load (x - mean).
//
// v_mfma_f64_16x16x4f64 operand layout: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, result D[i][j] in lane j + 16*(i%4), register i/4.
typedef double double4_t __attribute__((ext_vector_type(4)));

// LDS holds the chunk feature-major, [feature][sample] with a row of KC + 1
// doubles: the loader's stores (16 consecutive samples of a feature) are
// contiguous, and the MFMA operand reads (16 features at one sample) fall on
// distinct banks (row stride 34 dwords).
constexpr int LDS_STRIDE = GRAM_KC + 1;

// One wave per SIMD is all this launch needs (about one workgroup per CU), so
// the register budget is the whole file: no spills around the prefetch.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void gram_kernel(const double *__restrict__ F, int64_t n_total,
                                                   int64_t S, const int64_t *__restrict__ off,
                                                   const int32_t *__restrict__ torder,
                                                   int T, const double *__restrict__ mu,
                                                   int ntile, int nsplit,
                                                   double *__restrict__ part) {
    __shared__ double As[GRAM_TILE][LDS_STRIDE];
    __shared__ double Bs[GRAM_TILE][LDS_STRIDE];

    // blockIdx.x -> (split, task rank, tile pair); tile pairs enumerate
    // bi <= bj row by row; task ranks follow decreasing row counts
    int64_t b = blockIdx.x;
    const int npair = ntile * (ntile + 1) / 2;
    const int split = (int)(b / ((int64_t)T * npair));
    b -= (int64_t)split * T * npair;
    const int tr = (int)(b / npair);
    const int t = torder[tr];
    int pr = (int)(b - (int64_t)tr * npair);
    int bi = 0;
    while (pr >= ntile - bi) {
        pr -= ntile - bi;
        ++bi;
    }
    const int bj = bi + pr;

    const int64_t r0 = off[t], r1 = off[t + 1];
    const int64_t nchunk = (r1 - r0 + GRAM_KC - 1) / GRAM_KC;
    const int64_t per = (nchunk + nsplit - 1) / nsplit;
    const int64_t c0 = (int64_t)split * per;
    const int64_t c1 = c0 + per < nchunk ? c0 + per : nchunk;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (wave >> 1) * 64;  // wave's row offset inside the tile
    const int wc = (wave & 1) * 64;   // wave's column offset
    const double *mut = mu + (int64_t)t * S;

    double4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = (double4_t){0.0, 0.0, 0.0, 0.0};

    // loader mapping: kk = tid % KC (consecutive samples), feature = tid / KC + FPP r
    constexpr int FPP = 256 / GRAM_KC;          // features per loader pass
    constexpr int NP = GRAM_TILE / FPP;         // loader passes per operand
    const int kk = tid % GRAM_KC;
    const int f0 = tid / GRAM_KC;
    double muA[NP], muB[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
        const int64_t ga = (int64_t)bi * GRAM_TILE + f0 + FPP * r;
        const int64_t gb = (int64_t)bj * GRAM_TILE + f0 + FPP * r;
        muA[r] = ga < S ? mut[ga] : 0.0;
        muB[r] = gb < S ? mut[gb] : 0.0;
    }

    // register-staged double buffering: the global loads of chunk c+1 are in
    // flight while the MFMAs of chunk c run out of LDS.  Loads are
    // unconditional (row and feature clamped into range); masking and centring
    // happen at the LDS store, so no load is waited on before the MFMAs.
    int64_t fa[NP], fb[NP];
    bool ina[NP], inb[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
        const int64_t ga = (int64_t)bi * GRAM_TILE + f0 + FPP * r;
        const int64_t gb = (int64_t)bj * GRAM_TILE + f0 + FPP * r;
        ina[r] = ga < S;
        inb[r] = gb < S;
        fa[r] = (ina[r] ? ga : S - 1) * n_total;
        fb[r] = (inb[r] ? gb : S - 1) * n_total;
    }
    double sa[NP], sb[NP];
    int64_t row = r0 + c0 * GRAM_KC + kk;
    if (c0 < c1) {
        const int64_t rowc = row < r1 ? row : r1 - 1;
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            sa[r] = F[fa[r] + rowc];
            sb[r] = F[fb[r] + rowc];
        }
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            As[f0 + FPP * r][kk] = (row < r1 && ina[r]) ? sa[r] - muA[r] : 0.0;
            Bs[f0 + FPP * r][kk] = (row < r1 && inb[r]) ? sb[r] - muB[r] : 0.0;
        }
    }
    __syncthreads();
    for (int64_t c = c0; c < c1; ++c) {
        const bool more = c + 1 < c1;
        row += GRAM_KC;
        if (more) {
            const int64_t rowc = row < r1 ? row : r1 - 1;
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                sa[r] = F[fa[r] + rowc];
                sb[r] = F[fb[r] + rowc];
            }
        }
#pragma unroll
        for (int ks = 0; ks < GRAM_KC / 4; ++ks) {
            const int krow = ks * 4 + (lane >> 4);
            double a[4], bv[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) a[m] = As[wr + m * 16 + (lane & 15)][krow];
#pragma unroll
            for (int m = 0; m < 4; ++m) bv[m] = Bs[wc + m * 16 + (lane & 15)][krow];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], bv[n], acc[m][n], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                As[f0 + FPP * r][kk] = (row < r1 && ina[r]) ? sa[r] - muA[r] : 0.0;
                Bs[f0 + FPP * r][kk] = (row < r1 && inb[r]) ? sb[r] - muB[r] : 0.0;
            }
        }
        __syncthreads();
    }

    // store the raw block into part[split][t][i][j]
    double *P = part + ((int64_t)split * T + t) * S * S;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = (int64_t)bi * GRAM_TILE + wr + m * 16 + (lane >> 4) + 4 * r;
                const int64_t gj = (int64_t)bj * GRAM_TILE + wc + n * 16 + (lane & 15);
                if (gi < S && gj < S) P[gi * S + gj] = acc[m][n][r];
            }

}

// Sum the split partials, scale to a correlation matrix and write the tiled
// layout.  One workgroup per (task, 64x64 output tile pair ti <= tk): it reads
// every partial of the canonical upper block once (coalesced rows), writes
// tile (ti, tk) row by row and tile (tk, ti) through an LDS transpose, so the
// mirrored elements are bitwise equal and both writes are coalesced.  The
// diagonal is 1 for a non-constant column and 0 for a constant one; padding
// rows/columns and padded tasks are written as zeros.
constexpr int FIN_ROWS = 16;  // tile rows per finishing workgroup (divides 64)
//
// With several tasks the filter task's tiles are also written, in the
// one-task layout, to G1 (bitwise the values written to G).
__global__ __launch_bounds__(256) void gram_finish_kernel(const double *__restrict__ part, int64_t S, int T,
                                                          int TP, int nsplit, const double *__restrict__ inv_s,
                                                          double *__restrict__ G, int64_t nt,
                                                          double *__restrict__ G1,
                                                          const int32_t *__restrict__ tstar) {
    __shared__ double tr[GT][FIN_ROWS + 1];
    const int64_t npair = nt * (nt + 1) / 2;
    const int qr = (int)(blockIdx.x % (GT / FIN_ROWS));  // row band of the tile pair
    const int64_t pb = blockIdx.x / (GT / FIN_ROWS);
    const int t = (int)(pb / npair);
    int64_t pr = pb % npair;
    int64_t ti = 0, tk = 0;
    // tile pairs in groups of 8 tile rows, column by column: consecutive
    // workgroups write tile (ti, tk) in 8 streams and its mirror (tk, ti)
    // in one, instead of a mirror nt tiles further for every pair (at
    // S = 50,000 the finishing pass took 28.7 ms in row-by-row order, 13 ms
    // in this one)
    {
        int64_t r0 = 0;
        for (;;) {
            const int64_t g = nt - r0 < 8 ? nt - r0 : 8;
            const int64_t cnt = g * (g + 1) / 2 + g * (nt - r0 - g);
            if (pr < cnt) {
                const int64_t tri = g * (g + 1) / 2;
                if (pr < tri) {
                    int64_t k = 0;
                    while ((k + 1) * (k + 2) / 2 <= pr) ++k;
                    tk = r0 + k;
                    ti = r0 + (pr - k * (k + 1) / 2);
                } else {
                    const int64_t q = pr - tri;
                    tk = r0 + g + q / g;
                    ti = r0 + q % g;
                }
                break;
            }
            pr -= cnt;
            r0 += g;
        }
    }

    const double *ist = inv_s + (int64_t)t * S;
    const bool one = G1 != nullptr && t == *tstar;  // also write the one-task copy
    // each thread owns PER elements of rows [FIN_ROWS qr, FIN_ROWS (qr + 1));
    // the split partials are summed split by split, eight splits of loads in
    // flight (indices clamped in range, out-of-range elements masked after)
    constexpr int PER = GT * FIN_ROWS / 256;
    int64_t src[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + 256 * m;
        const int li = FIN_ROWS * qr + (e >> 6), lk = e & 63;
        int64_t i = ti * GT + li, k = tk * GT + lk;
        i = i < S ? i : S - 1;
        k = k < S ? k : S - 1;
        const int64_t a = (ti == tk && i > k) ? k : i, cc = (ti == tk && i > k) ? i : k;  // canonical (upper)
        src[m] = a * S + cc;
    }
    double acc[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) acc[m] = 0.0;
#pragma unroll 8
    for (int sp = 0; sp < nsplit; ++sp) {
        const double *P = part + ((int64_t)sp * T + t) * S * S;
#pragma unroll
        for (int m = 0; m < PER; ++m) acc[m] += P[src[m]];
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + 256 * m;
        const int li = FIN_ROWS * qr + (e >> 6), lk = e & 63;
        const int64_t i = ti * GT + li, k = tk * GT + lk;
        double v = 0.0;
        if (i < S && k < S) {
            const int64_t a = src[m] / S, cc = src[m] % S;
            v = i == k ? (ist[i] > 0.0 ? 1.0 : 0.0) : acc[m] * (ist[a] * ist[cc]);
        }
        G[((((ti * nt + tk) << 12) + (li << 6) + lk)) * TP + t] = v;
        if (one) G1[((ti * nt + tk) << 12) + (li << 6) + lk] = v;
        tr[lk][li - FIN_ROWS * qr] = v;
        if (t == T - 1)
            for (int tp = T; tp < TP; ++tp) G[((((ti * nt + tk) << 12) + (li << 6) + lk)) * TP + tp] = 0.0;
    }
    if (ti == tk) return;
    __syncthreads();
    for (int e = threadIdx.x; e < GT * FIN_ROWS; e += 256) {
        // row li of tile (tk, ti) = column li of tile (ti, tk): this band
        // holds columns [FIN_ROWS qr, FIN_ROWS (qr + 1)) of every such row
        const int li = e / FIN_ROWS, lk = FIN_ROWS * qr + e % FIN_ROWS;
        G[((((tk * nt + ti) << 12) + (li << 6) + lk)) * TP + t] = tr[li][lk - FIN_ROWS * qr];
        if (one) G1[((tk * nt + ti) << 12) + (li << 6) + lk] = tr[li][lk - FIN_ROWS * qr];
        if (t == T - 1)
            for (int tp = T; tp < TP; ++tp) G[((((tk * nt + ti) << 12) + (li << 6) + lk)) * TP + tp] = 0.0;
    }
}

// Several tasks (TP <= 16): one workgroup per (tile pair ti <= tk, band of
// FR_T rows) takes every task, so that each element's TP task values (task
// fastest in G) are written together.  Per task the split partials of the
// band are summed in the same order as the one-task kernel and scaled; the
// band is held in LDS for all tasks ([task][row][col], one padding double per
// task against bank conflicts), then written row by row to tile (ti, tk) and
// column by column to tile (tk, ti), both as contiguous runs of whole task
// groups.  The filter task's values also go to G1.
constexpr int FR_T = 4;  // tile rows per workgroup of the several-task finish
__global__ __launch_bounds__(256) void gram_finish_tasks_kernel(const double *__restrict__ part, int64_t S, int T,
                                                                int TP, int nsplit, const double *__restrict__ inv_s,
                                                                double *__restrict__ G, int64_t nt,
                                                                double *__restrict__ G1,
                                                                const int32_t *__restrict__ tstar) {
    extern __shared__ double val[];  // [TP][FR_T * 64 + 1]
    constexpr int NB = GT / FR_T;
    constexpr int VS = FR_T * GT + 1;
    const int qr = (int)(blockIdx.x % NB);
    int64_t pr = blockIdx.x / NB;
    int64_t ti = 0;
    while (pr >= nt - ti) {
        pr -= nt - ti;
        ++ti;
    }
    const int64_t tk = ti + pr;
    const int ts = G1 != nullptr ? *tstar : -1;
    const int tid = threadIdx.x;
    for (int t = 0; t < TP; ++t) {
        const double *ist = inv_s + (int64_t)t * S;
        for (int e = tid; e < FR_T * GT; e += 256) {
            const int li = FR_T * qr + e / GT, lk = e % GT;
            const int64_t i = ti * GT + li, k = tk * GT + lk;
            double v = 0.0;
            if (t < T && i < S && k < S) {
                const int64_t a = (ti == tk && i > k) ? k : i, cc = (ti == tk && i > k) ? i : k;  // canonical (upper)
                double acc = 0.0;
                for (int sp = 0; sp < nsplit; ++sp) acc += part[((int64_t)sp * T + t) * S * S + a * S + cc];
                v = i == k ? (ist[i] > 0.0 ? 1.0 : 0.0) : acc * (ist[a] * ist[cc]);
            }
            val[t * VS + e] = v;
            if (t == ts) G1[((ti * nt + tk) << 12) + (li << 6) + lk] = v;
        }
    }
    __syncthreads();
    for (int x = tid; x < FR_T * GT * TP; x += 256) {
        const int t = x % TP, e = x / TP;
        const int li = FR_T * qr + e / GT, lk = e % GT;
        G[(((ti * nt + tk) << 12) + (li << 6) + lk) * TP + t] = val[t * VS + e];
    }
    if (ti == tk) return;
    for (int x = tid; x < GT * FR_T * TP; x += 256) {
        const int t = x % TP, y = x / TP;
        const int r = y % FR_T, lk = y / FR_T;
        const double v = val[t * VS + r * GT + lk];
        G[(((tk * nt + ti) << 12) + (lk << 6) + FR_T * qr + r) * TP + t] = v;
        if (t == ts) G1[((tk * nt + ti) << 12) + (lk << 6) + FR_T * qr + r] = v;
    }
}

// Unpack task t of the tiled matrices into a plain row-major S x S array.
__global__ __launch_bounds__(256) void untile_kernel(const double *__restrict__ G, int64_t S, int64_t nt, int TP,
                                                     int t, double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S * S) return;
    dst[e] = G[gidx(e / S, e % S, nt, TP, t)];
}

int launch_untile(const Ctx &c, int t, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(untile_kernel, dim3((unsigned)((c.S * c.S + 255) / 256)), dim3(256), 0, st, c.G, c.S, c.Gnt,
                       c.TP, t, dst);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------- launchers
int launch_stats(const Ctx &c, hipStream_t st) {
    phase_begin(c, SISSO_PHASE_STATS, st);
    const dim3 xg((unsigned)((c.S * c.T + 3) / 4));
    int vpt = 2;
    while (vpt <= SX_VPT && 64 * vpt < c.rows_max) vpt *= 2;
    switch (vpt) {
#define SX_LAUNCH(V)                                                                                            \
    hipLaunchKernelGGL(stats_y_kernel<V>, dim3(1), dim3(256), 0, st, c.y, c.off_dev, c.T, c.ybar, c.cyy, c.flags, \
                       c.tstar);                                                                                \
    hipLaunchKernelGGL(stats_x_kernel<V>, xg, dim3(256), 0, st, c.F, c.y, c.off_dev, c.n_total, c.S, c.T, c.TP,  \
                       c.ybar, c.mu, c.inv_s, c.bhat, c.flags);                                                 \
    break;
    case 2: SX_LAUNCH(2)
    case 4: SX_LAUNCH(4)
    case 8: SX_LAUNCH(8)
    case 16: SX_LAUNCH(16)
    case 32: SX_LAUNCH(32)
    default: SX_LAUNCH(0)  // longer tasks: streamed
#undef SX_LAUNCH
    }
    phase_end(c, SISSO_PHASE_STATS, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gram(const Ctx &c, hipStream_t st) {
    const int ntile = (int)((c.S + GRAM_TILE - 1) / GRAM_TILE);
    const int64_t blocks = (int64_t)c.nsplit * c.T * ntile * (ntile + 1) / 2;
    phase_begin(c, SISSO_PHASE_GRAM, st);
    if (c.lp_ns > 0) {
        if (launch_gram_lp(c, c.lp_ns, st)) return -1;
    } else {
        hipLaunchKernelGGL(gram_kernel, dim3((unsigned)blocks), dim3(256), 0, st, c.F, c.n_total, c.S,
                           c.off_dev, c.torder, c.T, c.mu, ntile, c.nsplit, c.part);
    }
    const int64_t npair64 = c.Gnt * (c.Gnt + 1) / 2;
    if (c.T > 1 && c.TP <= 16) {
        const size_t lds = (size_t)c.TP * (FR_T * GT + 1) * sizeof(double);
        hipLaunchKernelGGL(gram_finish_tasks_kernel, dim3((unsigned)(npair64 * (GT / FR_T))), dim3(256), lds, st,
                           c.part, c.S, c.T, c.TP, c.nsplit, c.inv_s, c.G, c.Gnt, c.G1 != c.G ? c.G1 : nullptr,
                           c.tstar);
    } else {
        hipLaunchKernelGGL(gram_finish_kernel, dim3((unsigned)(npair64 * c.T * (GT / FIN_ROWS))), dim3(256), 0, st,
                           c.part, c.S, c.T, c.TP, c.nsplit, c.inv_s, c.G, c.Gnt, c.G1 != c.G ? c.G1 : nullptr,
                           c.tstar);
    }
    phase_end(c, SISSO_PHASE_GRAM, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sl0
