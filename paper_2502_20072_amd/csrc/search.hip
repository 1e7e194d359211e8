// Exhaustive l0 search on gfx950: every D-tuple of the S features is scored
// by the SSE of its least-squares fit (intercept per task), and the k best
// by (SSE, lexicographic rank) are kept.
//
// The paper factorises each tuple's n x (D+1) descriptor matrix with
// Householder QR, one GPU thread per tuple.  Here the fits come from the
// correlation matrices G_t, b_t, c_t that the Gram step precomputed: for a
// tuple T = (P, k) with prefix P,
//     w = R_P^{-1} G[P,k],  d = 1 - |w|^2,  zeta = b_k - w.z_P,
//     SSE_t(T) = p_P - zeta^2 / d       (p_P = c_t - |z_P|^2 = SSE_t(P)),
// with R_P the Cholesky factor of G[P,P] and z_P = R_P^{-1} b_P.  d is the
// pivot of k (1 - R^2 of x_k on the intercept and P), which is also the
// rank test.  For a single task the comparison SSE <= theta needs no
// division: zeta^2 >= (p_P - theta) d.
//
// Work decomposition.  A tuple is (P', j, k): a sub-prefix P' of D-2
// indices, the (D-1)-th index j and the last index k.  A work item is a
// block of 64 consecutive j values together with a group of sub-prefixes
// (SUBP of them for one task, one when lanes are split over tasks).  The
// workgroup builds the Cholesky row of every (P', j) pair of the item in
// parallel (one thread each) into LDS; then each wave sweeps chunks of 64
// consecutive k (one per lane), keeps the k-dependent part of the
// sub-prefix solve in registers, and for every j loads one G[j][k] that
// serves all sub-prefixes of the item.  Items are handed out through an
// atomic counter in order of increasing j, i.e. largest first; sub-prefix
// groups are addressed by colexicographic rank (combinatorial number
// system), so item -> (j-block, sub-prefixes) is a bisection, not a table.
//
// Top-k.  Each wave keeps a sorted list of the KP best (SSE, rank) pairs in
// LDS; insertions happen only for tuples that pass the current bound, which
// is the minimum of a pre-pass bound theta0 (see pre_*), the wave's own
// KP-th entry and a device-wide bound that full lists publish with an
// atomic min.  Any list's KP-th entry bounds the global KP-th best, so the
// filter never drops a tuple of the global top-KP.  A merge kernel gathers
// the entries under the final bound, and every survivor is re-scored from F
// itself (explicit residuals in FP64), which fixes the reported SSE to the
// accuracy of a direct least-squares fit, before the final ordering.
#include <math.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sl0 {

constexpr int MAXD = SISSO_MAX_D;
constexpr double INF = __builtin_huge_val();
constexpr double THETA_SLACK = 1e-9;  // relative slack of the filter bound
constexpr double THETA_SLACK_F32 = 1e-5;  // FP32 solve form: absolute slack, in units of sum_t c_t
#ifndef SEARCH_JG
#define SEARCH_JG 8  // G rows per prefetch group (two groups in flight)
#endif

__device__ inline bool key_less(double s1, uint64_t r1, double s2, uint64_t r2) {
    return s1 < s2 || (s1 == s2 && r1 < r2);
}

__device__ inline double theta_load(const unsigned long long *p) {
    unsigned long long b = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)b);
}

__device__ inline void theta_publish(unsigned long long *p, double v) {
    // non-negative doubles order like their bit patterns
    if (v >= 0.0 && v < INF) atomicMin(p, (unsigned long long)__double_as_longlong(v));
}

// Values every lane holds identically (read from LDS or a uniform address)
// are moved to scalar registers, so address arithmetic on them stays scalar.
__device__ inline int64_t uni(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline uint64_t uni(uint64_t v) { return (uint64_t)uni((int64_t)v); }
__device__ inline double uni(double v) { return __longlong_as_double(uni((int64_t)__double_as_longlong(v))); }

// Lane permutation inside rows of 16 lanes (DPP), for both halves of a double.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// the same lane permutation for the FP32 form's sums
template <int CTRL>
__device__ inline float dpp_r(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_r(double v) { return dpp_f64<CTRL>(v); }
__device__ inline float rcp_r(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
}
__device__ inline double rcp_r(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}
// pivot ratio at or below which the solve of type R calls a tuple rank
// deficient: FP32 resolves 1 - |w|^2 only to a few units of 2^-23
template <typename R>
__device__ constexpr R rank_eps_r() { return sizeof(R) == 8 ? (R)RANK_EPS : (R)RANK_EPS_F32; }

__device__ inline int next_pow2_dev(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

__device__ inline double Gat(const Ctx &c, int64_t i, int64_t k, int t) {
    return c.G[gidx(i, k, c.Gnt, c.TP, t)];
}

// ----------------------------------------------------------------- helpers
// Normal-equation SSE of one sorted tuple summed over tasks, from the
// correlation matrices (Cholesky in increasing index order).  +inf when a
// pivot is <= RANK_EPS in some task.  Used by the threshold pre-pass.  All
// entries a task needs are loaded before any arithmetic, so the loads of one
// call overlap instead of forming a chain.
// SSE of one task from its tuple's correlation block g (lower triangle,
// sorted-index order), b and c = |y_c|^2; clears ok on a pivot <= RANK_EPS.
template <int D>
__device__ inline double ne_sse_core(const double (&g)[D][D], const double (&bv)[D], double cyy, bool &ok) {
    double L[D][D], z[D];
    double p = cyy;
#pragma unroll
    for (int m = 0; m < D; ++m) {
#pragma unroll
        for (int j = 0; j < m; ++j) {
            double s = g[m][j];
#pragma unroll
            for (int l = 0; l < j; ++l) s -= L[m][l] * L[j][l];
            L[m][j] = s / L[j][j];
        }
        double d = g[m][m];
#pragma unroll
        for (int l = 0; l < m; ++l) d -= L[m][l] * L[m][l];
        ok &= d > RANK_EPS;
        L[m][m] = sqrt(fmax(d, RANK_EPS));
        double zm = bv[m];
#pragma unroll
        for (int l = 0; l < m; ++l) zm -= L[m][l] * z[l];
        z[m] = zm / L[m][m];
        p -= z[m] * z[m];
    }
    return p;
}

template <int D>
__device__ double ne_sse_t(const Ctx &c, const int32_t *tup) {
    double total = 0.0;
    bool ok = true;
    for (int t = 0; t < c.T; ++t) {
        double g[D][D], bv[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
#pragma unroll
            for (int j = 0; j <= m; ++j) g[m][j] = Gat(c, tup[m], tup[j], t);
            bv[m] = c.bhat[(int64_t)tup[m] * c.TP + t];
        }
        total += ne_sse_core<D>(g, bv, c.cyy[t], ok);
    }
    return ok ? total : INF;
}

__device__ double ne_sse(const Ctx &c, int D, const int32_t *tup) {
    switch (D) {
        case 1: return ne_sse_t<1>(c, tup);
        case 2: return ne_sse_t<2>(c, tup);
        case 3: return ne_sse_t<3>(c, tup);
        default: return ne_sse_t<4>(c, tup);
    }
}

// Sorted per-wave list in LDS: entries e = lane + 64 m, m < KP/64.
// A wave's sorted list is written to global memory only up to its first
// empty (+inf) entry, which is written too as a terminator: readers stop
// there, so the (usually empty) tail of KP entries costs no traffic.
__device__ inline void list_store(double *__restrict__ ds, uint64_t *__restrict__ dr, const double *Ls,
                                  const uint64_t *Lr, int KP) {
    const int lane = threadIdx.x & 63;
    int nv = 0;
    for (int m = 0; m < KP; m += 64) nv += __popcll(__ballot(Ls[m + lane] < INF));
    for (int m = lane; m < KP && m <= nv; m += 64) {
        ds[m] = Ls[m];
        dr[m] = Lr[m];
    }
}

// Reads a list written by list_store into LDS (entries past the terminator
// are +inf).
__device__ inline void list_load(double *Ls, uint64_t *Lr, const double *__restrict__ ss,
                                 const uint64_t *__restrict__ sr, int KP) {
    const int lane = threadIdx.x & 63;
    bool end = false;
    for (int m = 0; m < KP; m += 64) {
        // the live entries are the prefix before the terminator; what lies
        // after it in the same chunk is stale and is not read as an entry
        const double v = end ? INF : ss[m + lane];
        const unsigned long long b = __ballot(v < INF);
        const int nlive = end ? 0 : (b == ~0ull ? 64 : __builtin_ctzll(~b));
        const bool live = lane < nlive;
        Ls[m + lane] = live ? v : INF;
        Lr[m + lane] = live ? sr[m + lane] : ~0ull;
        end = end || nlive < 64;
    }
}

__device__ void list_insert(double *Ls, uint64_t *Lr, int KP, double s, uint64_t r) {
    const int lane = threadIdx.x & 63;
    const int nper = KP >> 6;
    int pos = 0;
    for (int m = 0; m < nper; ++m) {
        const int e = lane + 64 * m;
        pos += __popcll(__ballot(key_less(Ls[e], Lr[e], s, r)));
    }
    if (pos >= KP) return;
    if (Ls[pos] == s && Lr[pos] == r) return;  // the same tuple, offered twice (list search)
    // shift the entries above pos up by one, highest chunk of 64 first: a
    // chunk is read whole before it is written, and its lowest lane reads the
    // top entry of the chunk below before that chunk is written (few live
    // registers, whatever the list length)
    for (int m = nper - 1; m >= 0 && 64 * m + 63 > pos; --m) {
        const int e = lane + 64 * m;
        const bool mv = e > pos;
        double vs = 0.0;
        uint64_t vr = 0;
        if (mv) {
            vs = Ls[e - 1];
            vr = Lr[e - 1];
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();
        if (mv) {
            Ls[e] = vs;
            Lr[e] = vr;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        Ls[pos] = s;
        Lr[pos] = r;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
}

// Sorts a wave's LDS list of KP (power of two) entries by (SSE, key).
__device__ void wave_sort_list(double *Ls, uint64_t *Lr, int KP) {
    const int lane = threadIdx.x & 63;
    for (int k = 2; k <= KP; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < KP; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const double a = Ls[i], b = Ls[ixj];
                    const uint64_t ra = Lr[i], rb = Lr[ixj];
                    if (key_less(b, rb, a, ra) == up) {
                        Ls[i] = b;
                        Ls[ixj] = a;
                        Lr[i] = rb;
                        Lr[ixj] = ra;
                    }
                }
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
        }
}

// ------------------------------------------------------------ init kernel
// Resets the per-search device state and tabulates the cumulative number
// of work items per j-block: block jb covers j in [JB*jb, N_jb) with
// N_jb = min(JB*(jb+1), S-1); its sub-prefixes are the q-combinations of
// {0..N_jb-2}, grouped R at a time.
__device__ void s3_tile_table(const Ctx &c);

__device__ void s4_tables(const Ctx &c);

// s3: 0 = work-item table of the general kernel, 4 = the D = 4 record-table
// tiles, other = the D = 3 record-table tiles
__device__ void search_init_body(const Ctx &c, int64_t e, bool leader, int D, int R, int JB, int s3,
                                 bool clear_pre = true) {
    if (e < (int64_t)(SISSO_MAX_D + 1) * (c.S + 1)) {
        const int r = (int)(e / (c.S + 1));
        const int64_t n = e % (c.S + 1);
        c.btab[e] = binom(n, r);
    }
    if (leader) {
        *c.work_counter = 0;
        *c.cand_counter = 0;
        *c.theta_bits = (unsigned long long)__double_as_longlong(INF);
        if (clear_pre) *c.pre_count = 0;  // (else the pre-pass selection runs beside and sets it)
        *c.merge_count = 0;
        *c.mtq_taken = 0;
        c.flags[FLAG_CAPACITY] = 0;
        c.flags[FLAG_BATCHQ] = 0;
        c.flags[FLAG_NLISTS] = 0;
        c.stats[1] = 0;
        if (s3 == 4) {
            s4_tables(c);
            return;
        }
        if (s3) {
            s3_tile_table(c);
            return;
        }
        const int q = D - 2;
        const int64_t nblk = (c.S - 1 + JB - 1) / JB;
        uint64_t acc = 0;
        c.cum[0] = 0;
        for (int64_t b = 0; b < nblk; ++b) {
            int64_t N = JB * (b + 1);
            if (N > c.S - 1) N = c.S - 1;
            // C(N - 1, q) in closed form (q = D - 2 <= 2)
            const uint64_t m1 = (uint64_t)(N - 1);
            const uint64_t nsub = q == 0 ? 1 : q == 1 ? m1 : (m1 * (m1 - 1)) / 2;
            acc += (nsub + R - 1) / R;
            c.cum[b + 1] = acc;
        }
    }
}

__global__ void search_init_kernel(Ctx c, int D, int R, int JB, int s3) {
    search_init_body(c, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, threadIdx.x == 0 && blockIdx.x == 0, D, R,
                     JB, s3);
}

// ----------------------------------------------------- threshold pre-pass
// The search starts from an upper bound theta0 of the KP-th best SSE, so
// that almost no tuple reaches the exact path.  It is built from a small,
// structured set of real tuples: the best (D-1)-subsets of the PRE_M most
// relevant features, each extended by every feature.  Any set of real
// tuples gives a valid bound (below), so the selections may be heuristic;
// they run as block-wide histogram thresholds, one thread per candidate.
constexpr int PRE_WG = 1024;      // threads of the pre-pass workgroups
constexpr int PRE_SORT = 4096;    // largest sorted candidate set
constexpr int PRE_KEEP = PRE_SORT / PRE_WG;  // candidates a thread keeps when S > PRE_SORT


// Fill key/id[0..N) with the candidates v(x) for x in [0, n): directly when
// n <= PRE_SORT, else each thread keeps its PRE_KEEP smallest.  Returns N.
template <class F>
__device__ int gather_candidates(double *key, int *id, int64_t n, F v) {
    const int tid = threadIdx.x;
    if (n <= PRE_SORT) {
        const int N = next_pow2_dev((int)n);
        for (int x = tid; x < N; x += PRE_WG) {
            key[x] = x < n ? v(x) : INF;
            id[x] = x;
        }
        return N;
    }
    double kv[PRE_KEEP];
    int ki[PRE_KEEP];
#pragma unroll
    for (int m = 0; m < PRE_KEEP; ++m) {
        kv[m] = INF;
        ki[m] = 0x7fffffff;
    }
    for (int64_t x = tid; x < n; x += PRE_WG) {
        double cv = v(x);
        int ci = (int)x;
#pragma unroll
        for (int m = 0; m < PRE_KEEP; ++m) {
            const bool less = cv < kv[m] || (cv == kv[m] && ci < ki[m]);
            const double tv = kv[m];
            const int ti = ki[m];
            kv[m] = less ? cv : tv;
            ki[m] = less ? ci : ti;
            cv = less ? tv : cv;
            ci = less ? ti : ci;
        }
    }
#pragma unroll
    for (int m = 0; m < PRE_KEEP; ++m) {
        key[tid * PRE_KEEP + m] = kv[m];
        id[tid * PRE_KEEP + m] = ki[m];
    }
    return PRE_SORT;
}

// Selections of the pre-pass without sorting: a histogram of 1024 bins over
// the order keys of the candidate values (IEEE doubles mapped to integers so
// that integer order = value order) finds, in a few barrier steps, a
// threshold t such that at least L candidates are <= t and t lies within one
// bin of the L-th smallest value.
constexpr int SEL_NB = PRE_WG;  // one histogram bin per thread
struct SelScratch {
    unsigned long long mn, mx;
    unsigned cnt;
    unsigned hist[SEL_NB];
    unsigned wsum[PRE_WG / 64];
    double res;
    int npick;
};

__device__ inline uint64_t okey(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double okey_inv(uint64_t t) {
    const uint64_t u = (t >> 63) ? (t & 0x7fffffffffffffffull) : ~t;
    return __longlong_as_double((long long)u);
}

// Block-wide inclusive prefix sum of one value per thread (PRE_WG threads).
__device__ inline unsigned block_scan(unsigned v, unsigned *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    __syncthreads();
    return incl + base;
}

// Threshold over key[0..n) (smaller is better, INF = not a candidate): a
// value t, equal to a bin's upper edge or to the largest candidate, with at
// least L candidates <= t; INF when fewer than L candidates exist.  Called
// by all PRE_WG threads.
__device__ double block_threshold(const double *key, int n, int L, SelScratch &sc) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        sc.mn = ~0ull;
        sc.mx = 0;
        sc.cnt = 0;
    }
    sc.hist[tid] = 0;
    __syncthreads();
    unsigned long long mn = ~0ull, mx = 0;
    unsigned cnt = 0;
    for (int x = tid; x < n; x += PRE_WG) {
        const double v = key[x];
        if (v < INF) {
            const uint64_t u = okey(v);
            mn = u < mn ? u : mn;
            mx = u > mx ? u : mx;
            ++cnt;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long a = (unsigned long long)__shfl_xor((long long)mn, o);
        const unsigned long long b = (unsigned long long)__shfl_xor((long long)mx, o);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        cnt += __shfl_xor(cnt, o);
    }
    if ((tid & 63) == 0) {
        atomicMin(&sc.mn, mn);
        atomicMax(&sc.mx, mx);
        atomicAdd(&sc.cnt, cnt);
    }
    __syncthreads();
    if (L < 1 || sc.cnt < (unsigned)L) return INF;
    const uint64_t lo = sc.mn, hi = sc.mx, span = hi - lo;
    int sh = 0;
    while ((span >> sh) >= (uint64_t)SEL_NB) ++sh;
    for (int x = tid; x < n; x += PRE_WG) {
        const double v = key[x];
        if (v < INF) atomicAdd(&sc.hist[(okey(v) - lo) >> sh], 1u);
    }
    __syncthreads();
    const unsigned h = sc.hist[tid];
    const unsigned incl = block_scan(h, sc.wsum);
    if (incl >= (unsigned)L && incl - h < (unsigned)L) {
        // the bin holding the L-th smallest: every candidate of bins <= tid is
        // <= its upper edge (the last occupied bin's edge is the maximum)
        const uint64_t top = span >> sh;
        const uint64_t edge = (uint64_t)tid + 1 > top ? hi : lo + (((uint64_t)tid + 1) << sh) - 1;
        sc.res = okey_inv(edge);
    }
    __syncthreads();
    return sc.res;
}

// The first (by position) up to M positions x < n with key[x] <= t, into
// out[]; returns how many.  Called by all PRE_WG threads.
__device__ int block_pick_first(const double *key, int n, double t, int M, int *out, SelScratch &sc) {
    int taken = 0;
    for (int base = 0; base < n && taken < M; base += PRE_WG) {
        const int x = base + (int)threadIdx.x;
        const bool f = x < n && key[x] < INF && key[x] <= t;
        const unsigned incl = block_scan(f ? 1u : 0u, sc.wsum);
        const int pos = taken + (int)incl - (f ? 1 : 0);
        if (f && pos < M) out[pos] = x;
        if (threadIdx.x == PRE_WG - 1) sc.npick = taken + (int)incl;
        __syncthreads();
        taken = sc.npick < M ? sc.npick : M;
        __syncthreads();
    }
    return taken;
}

// pre_select: relevance of feature j = sum over tasks of b_tj^2 (its D=1
// explained sum of squares); the PRE_M most relevant full-rank features;
// every (D-1)-subset of them scored; the PRE_Q best subsets become prefixes.
template <int D>
__device__ void pre_select_body(const Ctx &c) {
    __shared__ double key[PRE_SORT];
    __shared__ int id[PRE_SORT];
    __shared__ int pick[PRE_M > PRE_Q ? PRE_M : PRE_Q];
    __shared__ int sel[PRE_M];
    __shared__ SelScratch sc;
    const int tid = threadIdx.x;
    constexpr int q = D - 1;
    if (tid == 0) {
        *c.pre_count = 0;
        *c.pre_done = 0;
    }
    // 1. the PRE_M most relevant full-rank features (up to the last
    //    histogram bin), in increasing index order
    const int N = gather_candidates(key, id, c.S, [&](int64_t j) {
        double r = 0.0;
        bool ok = true;
        for (int t = 0; t < c.T; ++t) {
            ok &= Gat(c, j, j, t) == 1.0;
            const double b = c.bhat[j * c.TP + t];
            r += b * b;
        }
        return ok ? -r : INF;
    });
    __syncthreads();
    double th = block_threshold(key, N, PRE_M, sc);
    if (!(th < INF)) th = __DBL_MAX__;  // fewer than PRE_M full-rank features: take them all
    const int M = block_pick_first(key, N, th, PRE_M, pick, sc);
    // increasing feature index (positions are indices unless S > PRE_SORT)
    if (tid < M) {
        const int f = id[pick[tid]];
        int r = 0;
        for (int b2 = 0; b2 < M; ++b2) r += id[pick[b2]] < f;
        sel[r] = f;
    }
    __syncthreads();
    if (M < q) return;
    // 2. score every q-subset of the selection (<= C(16, 3) = 560 of them)
    const int nsub = (int)binom(M, q);
    for (int e = tid; e < nsub; e += PRE_WG) {
        int32_t loc[MAXD], tup[MAXD];
        colex_unrank_small((uint64_t)e, q, M, loc);
        for (int m = 0; m < q; ++m) tup[m] = sel[loc[m]];
        key[e] = ne_sse_t<(D > 1 ? D - 1 : 1)>(c, tup);
    }
    __syncthreads();
    // 3. PRE_Q of the best subsets (the first in subset order at or below
    //    the threshold of the PRE_Q-th best)
    double th2 = block_threshold(key, nsub, PRE_Q, sc);
    if (!(th2 < INF)) th2 = __DBL_MAX__;
    const int Q = block_pick_first(key, nsub, th2, PRE_Q, pick, sc);
    if (tid < Q) {
        int32_t loc[MAXD];
        colex_unrank_small((uint64_t)pick[tid], q, M, loc);
        for (int m = 0; m < q; ++m) c.pre_prefix[tid * MAXD + m] = sel[loc[m]];
    }
    if (tid == 0) *c.pre_count = Q;
}

template <int D>
__global__ __launch_bounds__(PRE_WG) void pre_select_kernel(Ctx c) {
    pre_select_body<D>(c);
}

// pre_extend: block qq scores every tuple prefix_qq + {k} that does not
// contain an earlier chosen prefix (so the tuples of different blocks are
// distinct) and lies in the searched rank range, and records the L-th
// smallest SSE among the candidates it kept.  Those are L distinct real
// tuples at or below that value, so Q*L >= KP of them at or below the
// maximum over blocks make that maximum an upper bound of the KP-th best
// SSE of the search.
template <int D>
__global__ __launch_bounds__(PRE_WG) void pre_extend_kernel(Ctx c, int ranged, uint64_t r0,
                                                            uint64_t r1, int L) {
    __shared__ double key[PRE_SORT];
    __shared__ int id[PRE_SORT];
    __shared__ SelScratch sc;
    const int qq = blockIdx.x;
    const int tid = threadIdx.x;
    const int Q = *c.pre_count;
    if (qq >= Q || L > PRE_SORT) {
        if (tid == 0) c.pre_bound[qq] = INF;
        return;
    }
    const int q = D - 1;
    int32_t P[MAXD];
    for (int m = 0; m < q; ++m) P[m] = c.pre_prefix[qq * MAXD + m];
    const int N = gather_candidates(key, id, c.S, [&](int64_t k) {
        int32_t tup[MAXD];
        bool inP = false;
        int n = 0;
        for (int m = 0; m < q; ++m) inP |= (P[m] == k);
        if (inP) return INF;
        bool placed = false;
        for (int m = 0; m < q; ++m) {
            if (!placed && k < P[m]) {
                tup[n++] = (int32_t)k;
                placed = true;
            }
            tup[n++] = P[m];
        }
        if (!placed) tup[n++] = (int32_t)k;
        for (int o = 0; o < qq; ++o) {
            int hit = 0;
            for (int m = 0; m < q; ++m) {
                const int32_t v = c.pre_prefix[o * MAXD + m];
                for (int u = 0; u < D; ++u) hit += (tup[u] == v);
            }
            if (hit == q) return INF;
        }
        if (ranged) {
            const uint64_t rk = lex_rank(BinomTab{c.btab, c.S}, c.S, D, tup);
            if (rk < r0 || rk >= r1) return INF;
        }
        return ne_sse_t<D>(c, tup);
    });
    __syncthreads();
    // at least L of the kept candidates (distinct real tuples) are <= the bound
    const double bound = block_threshold(key, N, L, sc);
    if (tid == 0) c.pre_bound[qq] = bound;
    if (c.T == 1) return;
    // several tasks: the tuples of all blocks are distinct, so the KP-th
    // smallest of their pooled scores is a bound as well, and usually far
    // below the largest per-block one (the weakest prefix no longer sets it).
    // The last block to finish computes it.
    const int nk = N < c.S ? N : (int)c.S;
    for (int x = tid; x < nk; x += PRE_WG) c.pre_sse[(int64_t)qq * c.S + x] = key[x];
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(c.pre_done, 1u) == (unsigned)Q - 1u;  // blocks qq >= Q left above
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int KP = c.KP;
    const int64_t npool = (int64_t)Q * c.S;
    const int NP = gather_candidates(key, id, npool, [&](int64_t x) {
        // (every block kept the same count nk)
        return x % c.S < nk ? __hip_atomic_load(&c.pre_sse[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : INF;
    });
    __syncthreads();
    const double pooled = block_threshold(key, NP, KP, sc);
    if (tid == 0 && pooled < INF) {
        double mx = 0.0;
        for (int b = 0; b < Q; ++b) mx = fmax(mx, c.pre_bound[b]);
        const double th = fmin(mx, pooled);
        for (int b = 0; b < Q; ++b) c.pre_bound[b] = th;
    }
}

template <class CtxT>
__device__ double theta0_from_prepass(const CtxT &c, int L, int KP) {
    const int Q = *c.pre_count;
    if ((int64_t)Q * L < KP) return INF;
    double th = 0.0;
    for (int q = 0; q < Q; ++q) th = fmax(th, c.pre_bound[q]);
    return th;
}

// --------------------------------------------------------- search kernel
constexpr int MT_RECS = 512;  // records per work item with many tasks (JB * TP)

struct SearchArgs {
    int D, TL, JB, R, KP, L, ranged;
    uint64_t r0, r1;
};


// LDS record of the Cholesky row of prefix (P', j) for one task:
//   v[0..q-1] = R_{P'}^{-1} G[P', j],  alpha = 1/d_j,  zs = z_j / s_j,
//   pi = p - theta_f (single task) ,  p = SSE of the prefix (P', j)
// z_j = (b_j - v.z') / s_j, s_j = sqrt(d_j), d_j = 1 - |v|^2.
// An invalid record has p = pi = NaN, which fails every comparison.

// k-dependent part of each sub-prefix solve for last index kc:
//   w' = R_{P'}^{-1} G[P', kc],  d' = 1 - |w'|^2,  zeta' = b_kc - w'.z'
// (sub-prefix factors read from LDS).  One set per sub-prefix (one task) or
// for the lane's task (many tasks).
template <int D, int NR, bool MT, typename R>
__device__ inline void hoist_k(const Ctx &c, const R *subf, const int32_t *sub, int64_t kc, int myt,
                               R (&wq)[NR][(D - 2) > 0 ? (D - 2) : 1], R (&dq)[NR], R (&zq)[NR]) {
    constexpr int q = D - 2;
    constexpr int QA = q > 0 ? q : 1;
    constexpr int SUBW = QA * QA + QA + 2;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int sid = MT ? myt : r;
        const R *f = subf + sid * SUBW;
        const int tt = MT ? myt : 0;
        R g[QA];
#pragma unroll
        for (int m = 0; m < q; ++m) {
            const int32_t pm = sub[(MT ? 0 : r) * QA + m];
            g[m] = (pm >= 0 && tt < c.T) ? (R)Gat(c, pm, kc, tt) : (R)0;
        }
        R dd = (tt < c.T) ? (R)Gat(c, kc, kc, tt) : (R)1;
        R zz = (tt < c.T) ? (R)c.bhat[kc * c.TP + tt] : (R)0;
#pragma unroll
        for (int m = 0; m < q; ++m) {
            R s = 0;
#pragma unroll
            for (int l = 0; l <= m; ++l) s += f[m * QA + l] * g[l];
            wq[r][m] = s;
            dd -= s * s;
            zz -= s * f[QA * QA + m];
        }
        dq[r] = dd;
        zq[r] = zz;
    }
}

// Rare path of the sweep: at least one lane passed the filter for (P', j, k).
// Recomputes the tuple terms exactly as the fast loop does, takes the SSE
// with a true division, applies the rank test and the current bound, and
// inserts the survivors into the wave's list.  Kept out of line so the fast
// loop's registers are not shaped by it.  Returns the wave's published bound.
template <int D, int NR, bool MT, typename R>
__device__ inline double slow_path(const Ctx &c, const SearchArgs &a, double *Ls, uint64_t *Lr,
                                         const R *recs, const R *subf, const int32_t *sub,
                                         const unsigned long long *smask, int64_t j, int jj, int64_t k,
                                         bool kin, bool flagged, int myt, int TL, double theta_f,
                                         double theta_pub, unsigned &offered) {
    constexpr int q = D - 2;
    constexpr int QA = q > 0 ? q : 1;
    constexpr int RECW = q + 4;
    const int KP = a.KP;
    const int lane = threadIdx.x & 63;
    const int64_t kc = kin ? k : c.S - 1;
    R wq[NR][QA], dq[NR], zq[NR];
    hoist_k<D, NR, MT, R>(c, subf, sub, kc, myt, wq, dq, zq);
    const bool lane_ok = kin && (k > j) && (MT || flagged);
    for (int r = 0; r < NR; ++r) {
        if (!MT && !((smask[r] >> jj) & 1ull)) continue;
        const R *rr = MT ? recs + (jj * TL + myt) * RECW : recs + (jj * NR + r) * RECW;
        const R g = (R)Gat(c, j, kc, MT ? myt : 0);
        R u = g;
        for (int x = 0; x < q; ++x) u = fma(-rr[x], wq[r][x], u);
        const R d = fma(-rr[q], u * u, dq[r]);
        const R z = fma(-rr[q + 1], u, zq[r]);
        double es;
        bool pass;
        if (MT) {
            R ex = 0;
            if (myt < c.T) ex = (d > rank_eps_r<R>()) ? rr[q + 3] - z * z / d : (R)INF;
            for (int o = 1; o < TL; o <<= 1) ex += __shfl_xor(ex, o);
            es = (double)ex;
            pass = (myt == 0);
        } else {
            es = (d > rank_eps_r<R>()) ? (double)(rr[q + 3] - z * z / d) : INF;
            pass = true;
        }
        const double thc = fmin(theta_f, Ls[KP - 1]);
        bool take = pass && lane_ok && (es <= thc);
        uint64_t rk = 0;
        if (take) {
            int32_t tup[MAXD];
            for (int m = 0; m < q; ++m) tup[m] = sub[(MT ? 0 : r) * QA + m];
            tup[q] = (int32_t)j;
            tup[q + 1] = (int32_t)k;
            rk = pack_tuple(tup, D);
            if (a.ranged) {
                const uint64_t lr = lex_rank(BinomTab{c.btab, c.S}, c.S, D, tup);
                if (lr < a.r0 || lr >= a.r1) take = false;
            }
        }
        unsigned long long m = __ballot(take);
        offered += (unsigned)__popcll(m);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const double cs = __shfl(es, src);
            const uint64_t cr = (uint64_t)__shfl((long long)rk, src);
            list_insert(Ls, Lr, KP, cs, cr);
        }
    }
    const double tw = Ls[KP - 1];
    if (tw < theta_pub) {
        theta_pub = tw;
        if (lane == 0) theta_publish(c.theta_bits, tw);
    }
    return theta_pub;
}

template <int D, bool MT, typename R>
__global__ __launch_bounds__(256) void search_kernel(Ctx c, SearchArgs a) {
    constexpr int q = D - 2;
    constexpr int QA = q > 0 ? q : 1;               // array extent
    constexpr int RECW = q + 4;                      // values per record
    constexpr int SUBW = QA * QA + QA + 2;           // Linv (QA x QA), z', p', valid
    constexpr int NR = MT ? 1 : SUBP;                // sub-prefixes per item

    extern __shared__ double smem[];
    const int KP = a.KP;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (kept in an SGPR)

    // LDS carve: per-wave lists, records [256][RECW], sub-prefix factors
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    R *recs = reinterpret_cast<R *>(smem + (size_t)SEARCH_WAVES * KP * 2);
    R *subf = recs + (MT ? a.JB * a.TL : SEARCH_WG) * RECW;  // [64][SUBW] (per r, or per task)
    __shared__ int32_t s_sub[SUBP][QA];                // sub-prefix indices per r
    __shared__ int s_iq[SUBP];                         // last sub-prefix index (or -1)
    __shared__ unsigned long long s_mask[SUBP > 64 ? SUBP : 64];  // record validity per r (ST) / per jj (MT)
    __shared__ uint64_t s_item;
    __shared__ double s_theta;
    __shared__ unsigned long long s_qmask[SEARCH_WAVES][JBLK];
    __shared__ int s_qj[SEARCH_WAVES][JBLK];

    for (int m = lane; m < KP; m += 64) {
        Ls[m] = INF;
        Lr[m] = ~0ull;
    }
    double theta_pub = INF;  // last value this wave published
    unsigned offered = 0;    // tuples offered to the list (diagnostics; one atomic per wave)
    const double theta0 = theta0_from_prepass(c, a.L, KP);
    // the FP32 form's filter bound is widened by an absolute margin (a
    // multiple of the FP32 rounding of SSEs of size up to c)
    double ctot = 0.0;
    if (sizeof(R) < 8)
        for (int t = 0; t < c.T; ++t) ctot += c.cyy[t];
    const double abs_slack = sizeof(R) < 8 ? THETA_SLACK_F32 * ctot : 0.0;

    const int TL = MT ? a.TL : 1;         // lanes per last index
    const int KL = 64 / TL;               // last indices per wave chunk
    const int JB = a.JB;                  // j values per item

    const uint64_t nitems = uni(c.cum[(c.S - 1 + JB - 1) / JB]);
    if (blockIdx.x == 0 && tid == 0) c.stats[1] = nitems;
    const double *__restrict__ Gbase = c.G;
    // items are dealt round-robin over the workgroups (largest first): a
    // shared counter would serialise on one address
    for (uint64_t next = blockIdx.x;; next += gridDim.x) {
        if (tid == 0) {
            s_item = next;
            const double ts = theta_load(c.theta_bits);
            s_theta = fmin(ts, theta0);
        }
        __syncthreads();
        const uint64_t item = uni(s_item);
        if (item >= nitems) break;
        const double theta_item = uni(s_theta);
        const double theta_f = theta_item < INF ? theta_item * (1.0 + THETA_SLACK) + abs_slack : INF;
        const R theta_r = (R)theta_f;

        // item -> (j-block, sub-prefix group) by bisection on the cumulative table
        int64_t lo = 0, hi = (c.S - 1 + JB - 1) / JB - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (c.cum[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int64_t jb = uni(lo);
        const uint64_t grp = uni(item - c.cum[jb]);
        int64_t Nj = JB * (jb + 1);
        if (Nj > c.S - 1) Nj = c.S - 1;
        const int64_t j0 = JB * jb;
        const uint64_t nsub = q > 0 ? binom(Nj - 1, q) : 1;

        // ---- records: thread -> (r, jj) for one task, (jj, t) for many (then
        //      JB * TL records, several per thread)
        for (int rid = tid; rid < (MT ? JB * TL : SEARCH_WG); rid += SEARCH_WG) {
            int r, jj, t;
            if (MT) {
                r = 0;
                jj = rid / TL;
                t = rid % TL;
            } else {
                r = tid >> 6;
                jj = tid & 63;
                t = 0;
            }
            const uint64_t sr = grp * NR + r;
            const bool rvalid = (r < NR) && (sr < nsub) && (jj < JB);
            int32_t P[QA];
            if (rvalid) {
                if (q > 0) colex_unrank_small(sr, q, Nj - 1, P);
            }
            // sub-prefix factorisation (normalised: unit diagonal)
            R Li[QA][QA], zp[QA], pp = 0;
            bool pvalid = rvalid && t < c.T;
            if (pvalid) {
                pp = (R)c.cyy[t];
                R Lf[QA][QA];
                for (int m = 0; m < q; ++m) {
                    for (int jx = 0; jx < m; ++jx) {
                        R s = (R)Gat(c, P[m], P[jx], t);
                        for (int l = 0; l < jx; ++l) s -= Lf[m][l] * Lf[jx][l];
                        Lf[m][jx] = s / Lf[jx][jx];
                    }
                    R d = (R)Gat(c, P[m], P[m], t);
                    for (int l = 0; l < m; ++l) d -= Lf[m][l] * Lf[m][l];
                    if (!(d > rank_eps_r<R>())) pvalid = false;
                    Lf[m][m] = sqrt(fmax(d, (R)0));
                }
                if (pvalid) {
                    // Li = Lf^{-1} (lower), z' = Li b_P', p' = c - |z'|^2
                    for (int m = 0; m < q; ++m) {
                        for (int jx = 0; jx <= m; ++jx) {
                            R s = (m == jx) ? (R)1 : (R)0;
                            for (int l = jx; l < m; ++l) s -= Lf[m][l] * Li[l][jx];
                            Li[m][jx] = s / Lf[m][m];
                        }
                        for (int jx = m + 1; jx < QA; ++jx) Li[m][jx] = 0;
                    }
                    for (int m = 0; m < q; ++m) {
                        R s = 0;
                        for (int l = 0; l <= m; ++l) s += Li[m][l] * (R)c.bhat[(int64_t)P[l] * c.TP + t];
                        zp[m] = s;
                        pp -= s * s;
                    }
                }
            }
            // publish the sub-prefix (one writer per r / per task)
            const int sid = MT ? t : r;
            const bool writer = MT ? (jj == 0 && t < 64) : (jj == 0 && r < NR);
            if (writer) {
                R *f = subf + sid * SUBW;
                for (int m = 0; m < QA; ++m)
                    for (int l = 0; l < QA; ++l) f[m * QA + l] = (pvalid && m < q) ? Li[m][l] : (R)0;
                for (int m = 0; m < QA; ++m) f[QA * QA + m] = (pvalid && m < q) ? zp[m] : (R)0;
                f[QA * QA + QA] = pvalid ? pp : (R)0;
                f[QA * QA + QA + 1] = pvalid ? (R)1 : (R)0;
                if (!MT) {
                    for (int m = 0; m < QA; ++m) s_sub[r][m] = (rvalid && m < q) ? P[m] : -1;
                    s_iq[r] = (rvalid && q > 0) ? P[q - 1] : (rvalid ? -1 : 1 << 30);
                } else if (t == 0) {
                    for (int m = 0; m < QA; ++m) s_sub[0][m] = (rvalid && m < q) ? P[m] : -1;
                    s_iq[0] = (rvalid && q > 0) ? P[q - 1] : (rvalid ? -1 : 1 << 30);
                }
            }
            // record of (P', j)
            const int64_t j = j0 + jj;
            const int iq = (q > 0 && rvalid) ? P[q - 1] : -1;
            bool jvalid = rvalid && (j > iq) && (j < Nj);
            R rec[RECW];
            for (int m = 0; m < RECW; ++m) rec[m] = 0;
            bool ok = false;
            if (jvalid && t < c.T && pvalid) {
                R v[QA];
                R d = (R)Gat(c, j, j, t);
                for (int m = 0; m < q; ++m) {
                    R s = 0;
                    for (int l = 0; l <= m; ++l) s += Li[m][l] * (R)Gat(c, P[l], j, t);
                    v[m] = s;
                    d -= s * s;
                }
                if (d > rank_eps_r<R>()) {
                    const R sj = sqrt(d);
                    R zn = (R)c.bhat[j * c.TP + t];
                    for (int m = 0; m < q; ++m) zn -= v[m] * zp[m];
                    zn /= sj;
                    const R p = pp - zn * zn;
                    for (int m = 0; m < q; ++m) rec[m] = v[m];
                    rec[q] = (R)1 / d;
                    rec[q + 1] = zn / sj;
                    rec[q + 2] = p - theta_r;
                    rec[q + 3] = p;
                    ok = true;
                }
            } else if (MT && jvalid && t >= c.T) {
                ok = true;  // padding task: contributes exactly zero
            }
            if (!ok) {
                rec[q + 2] = (R)__builtin_nan("");
                rec[q + 3] = (R)__builtin_nan("");
            }
            const int slot = MT ? (jj * TL + t) : (jj * NR + r);
            if (MT ? (jj < JB) : true) {
                R *dst = recs + slot * RECW;
                for (int m = 0; m < RECW; ++m) dst[m] = rec[m];
            }
            // validity masks: ST per r over jj; MT per jj over all tasks
            if (!MT) {
                const unsigned long long bal = __ballot(ok);
                if (lane == 0) s_mask[r] = bal;
            }
        }
        if (MT) {
            if (tid < 64) s_mask[tid] = 0;
        }
        __syncthreads();
        if (MT) {
            // a j is live if every real task has a valid record
            if (tid < JB) {
                bool all = true;
                for (int t = 0; t < c.T; ++t) {
                    const R *rr = recs + (tid * TL + t) * RECW;
                    all &= !__builtin_isnan(rr[q + 3]);
                }
                s_mask[tid] = all ? 1ull : 0ull;
            }
            __syncthreads();
        }

        // ---- sweep the last index k in chunks of KL per wave
        const int64_t jhi = (j0 + JB < Nj ? j0 + JB : Nj) - 1;  // largest j of the block
        const int64_t kstart = j0;  // chunks are aligned to KL, which divides the tile width
        const int tl = MT ? (lane % TL) : 0;
        const int kl = MT ? (lane / TL) : lane;
        const int myt = tl;
        unsigned long long *qmask = s_qmask[wave];
        int *qj = s_qj[wave];
        for (int64_t kb = kstart + (int64_t)wave * KL; kb < c.S; kb += (int64_t)SEARCH_WAVES * KL) {
            const int64_t k = kb + kl;
            const bool kin = k < c.S;
            const int64_t kc = kin ? k : c.S - 1;
            R wq[NR][QA], dq[NR], zq[NR];
            hoist_k<D, NR, MT, R>(c, subf, &s_sub[0][0], kc, myt, wq, dq, zq);
            const bool check = (kb <= jhi) || (kb + KL > c.S);
            // G rows of the tile (j-block, k-chunk): a uniform pointer to row j0
            // plus 32-bit row and lane offsets (one task: TP = 1).  Rows are
            // clamped to the block's last row, which lies inside the tile; lanes
            // past S read the tile's zero padding.
            const int TPk = MT ? c.TP : 1;
            const int rs = GT * TPk;
            const int ko = (int)(k & (GT - 1)) * TPk + myt;
            const int nrow = (int)(jhi - j0);            // last row of the block, < 64
            const int kr = (int)(k - j0);                // lane's k relative to j0 (> row means k > j)
            const double *__restrict__ gp =
                Gbase + ((((j0 >> 6) * c.Gnt + (kb >> 6)) << 12) + ((j0 & (GT - 1)) << 6)) * TPk;
            int nq = 0;  // steps of this chunk where some lane passed the filter
            // the j sweep, versioned on whether lanes need the k > j / k < S masks
            auto sweep = [&](auto checkc) {
                constexpr bool CHECK = decltype(checkc)::value;
                // records of one step: (P', j) for every sub-prefix (one task)
                typedef R RecSet[NR][q + 3];
                auto load_rv = [&](RecSet &rv, int jj) {
                    const R *rj = recs + jj * (NR * RECW);
#pragma unroll
                    for (int r = 0; r < NR; ++r)
#pragma unroll
                        for (int x = 0; x < q + 3; ++x) rv[r][x] = rj[r * RECW + x];
                };
                auto body = [&](int jj, R g, bool live, const RecSet &rvs) {
                    unsigned long long m = 0;
                    if (MT) {
                        // a j whose record is invalid in some task has p = NaN
                        // there, so its task sum fails the comparison
                        const R *rr = recs + (jj * TL + myt) * RECW;
                        R rv[q + 4];
#pragma unroll
                        for (int x = 0; x < q + 4; ++x) rv[x] = rr[x];
                        __asm__ volatile("" ::: "memory");
                        R u = g;
#pragma unroll
                        for (int x = 0; x < q; ++x) u = fma(-rv[x], wq[0][x], u);
                        const R d = fma(-rv[q], u * u, dq[0]);
                        const R z = fma(-rv[q + 1], u, zq[0]);
                        // p - z^2/d with a reciprocal refined by one Newton step
                        R sum = fma(-(z * z), rcp_r(d), rv[q + 3]);
                        for (int o = 1; o < TL; o <<= 1) sum += __shfl_xor(sum, o);
                        m = __ballot(sum <= theta_r && tl == 0);
                    } else {
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            R u = g;
#pragma unroll
                            for (int x = 0; x < q; ++x) u = fma(-rvs[r][x], wq[r][x], u);
                            const R d = fma(-rvs[r][q], u * u, dq[r]);
                            const R z = fma(-rvs[r][q + 1], u, zq[r]);
                            m |= __ballot(z * z >= rvs[r][q + 2] * d);
                        }
                    }
                    if (CHECK) m &= __ballot(kin && kr > jj);
                    m = live ? m : 0ull;
                    if (m) {
                        if (lane == 0) {
                            qmask[nq] = m;
                            qj[nq] = jj;
                        }
                        ++nq;
                    }
                };
                // rows are fetched a group of JG ahead into the other of two
                // register sets, so JG loads per wave are in flight while a
                // group is scored
                constexpr int JG = SEARCH_JG;
                R ga[JG], gb[JG];
                // a uniform 64-bit base plus a 32-bit byte offset per load
                // (uniform row part + per-lane column part)
                const char *__restrict__ gpc = reinterpret_cast<const char *>(gp);
                const uint32_t ko8 = (uint32_t)ko * 8u;
                auto fetch = [&](R (&dst)[JG], int jg) {
#pragma unroll
                    for (int x = 0; x < JG; ++x) {
                        const int jr = jg + x < nrow ? jg + x : nrow;
                        const uint32_t ro = (uint32_t)(jr * rs) * 8u;
                        dst[x] = (R)*reinterpret_cast<const double *>(gpc + (ro + ko8));
                    }
                };
                // every fetched row is scored (rows past the block repeat its
                // last row and are masked out), so no load is left pending on
                // a skipped path
                auto score = [&](const R (&src)[JG], int jg) {
                    if (MT) {
                        // many tasks: the task terms of all JG rows first (independent
                        // chains), then their sums over the TL task lanes of each last
                        // index, all rows at once (row-local DPP steps; wider groups
                        // by lane shuffles)
                        R sm[JG];
#pragma unroll
                        for (int x = 0; x < JG; ++x) {
                            const int jj = jg + x <= nrow ? jg + x : nrow;
                            const R *rr = recs + (jj * TL + myt) * RECW;
                            R u = src[x];
#pragma unroll
                            for (int xx = 0; xx < q; ++xx) u = fma(-rr[xx], wq[0][xx], u);
                            const R d = fma(-rr[q], u * u, dq[0]);
                            const R z = fma(-rr[q + 1], u, zq[0]);
                            sm[x] = fma(-(z * z), rcp_r(d), rr[q + 3]);
                        }
                        if (TL >= 2) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += dpp_r<0xB1>(sm[x]);  // lane ^ 1
                        }
                        if (TL >= 4) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += dpp_r<0x4E>(sm[x]);  // lane ^ 2
                        }
                        if (TL >= 8) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += dpp_r<0x141>(sm[x]);  // mirror in 8
                        }
                        if (TL >= 16) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += dpp_r<0x140>(sm[x]);  // mirror in 16
                        }
                        if (TL >= 32) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += __shfl_xor(sm[x], 16);
                        }
                        if (TL >= 64) {
#pragma unroll
                            for (int x = 0; x < JG; ++x) sm[x] += __shfl_xor(sm[x], 32);
                        }
#pragma unroll
                        for (int x = 0; x < JG; ++x) {
                            const int jj = jg + x <= nrow ? jg + x : nrow;
                            unsigned long long m = __ballot(sm[x] <= theta_r && tl == 0);
                            if (CHECK) m &= __ballot(kin && kr > jj);
                            m = (jg + x <= nrow) ? m : 0ull;
                            if (m) {
                                if (lane == 0) {
                                    qmask[nq] = m;
                                    qj[nq] = jj;
                                }
                                ++nq;
                            }
                        }
                        return;
                    }
#pragma unroll
                    for (int x = 0; x < JG; ++x) {
                        const int jj = jg + x <= nrow ? jg + x : nrow;
                        RecSet rv;
                        // all record reads of the step are issued before any use
                        load_rv(rv, jj);
                        __asm__ volatile("" ::: "memory");
                        body(jj, src[x], jg + x <= nrow, rv);
                    }
                };
                // drain the loads of the chunk set-up first, so that only the
                // row prefetches are outstanding when the sweep loop starts
                // (vmcnt(0); expcnt and lgkmcnt not waited on)
                __builtin_amdgcn_s_waitcnt(0x0F70);
                // one exit at the bottom: every path into the loop head has the
                // same loads outstanding, so the head needs no full drain
                fetch(ga, 0);
                for (int jg = 0;; jg += 2 * JG) {
                    fetch(gb, jg + JG);
                    score(ga, jg);
                    fetch(ga, jg + 2 * JG);
                    score(gb, jg + JG);
                    if (jg + 2 * JG > nrow) break;
                }
            };
            if (check) sweep(std::true_type{});
            else sweep(std::false_type{});
            // exact scoring of the queued steps (rare)
            for (int e = 0; e < nq; ++e) {
                const int jj = qj[e];
                const unsigned long long lm = qmask[e];
                theta_pub = slow_path<D, NR, MT, R>(c, a, Ls, Lr, recs, subf, &s_sub[0][0], s_mask, j0 + jj, jj, k,
                                                 kin, (lm >> lane) & 1ull, myt, TL, theta_f, theta_pub, offered);
            }
        }
        __syncthreads();
    }
    if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
    // write this wave's list
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// ------------------------------------------- D = 3, one task: record table
// With one task and D = 3 the Cholesky row of every pair (i1, j) is built
// once per search into a table (rec3_kernel), and the sweep reads the rows
// of four consecutive i1 for one j with scalar loads: lanes run over the
// last index k, so a record is the same for every lane and enters the FP64
// instructions as a scalar operand, at no LDS or vector-memory cost.  A
// work tile is (group of four i1, S3_JR rows j from j0, S3_KC columns k from
// j0 + 1 + S3_KC c); lane l takes k = kb + l and kb + 64 + l (one load of
// G[j][k] each serves 4 tuples), so only chunk 0 holds tuples with k <= j
// (in its first half), and a last chunk with at most 64 columns left runs
// its first half only.  Tiles are dealt to single waves round-robin, so no
// wave waits on another.  Per tuple the arithmetic is the same as search_kernel's
// single-task path: u = g - v w', d = d' - alpha u^2, zeta = zeta' - zs u,
// pass iff zeta^2 >= (p - theta) d.
constexpr int S3_NR = 4;              // i1 per tile (a group)
constexpr int S3_KC = 128;            // k per tile: two per lane, 64 apart
#ifndef S3_JR
#define S3_JR 64                      // j rows per tile (divides 64)
#endif
#ifndef S3_JG
#define S3_JG 2                       // G rows per prefetch group (two groups in flight)
#endif
constexpr int S3_XCDS = 8;            // XCDs of the chip
#ifndef S3_XCD_RUN
#define S3_XCD_RUN 64                 // consecutive tiles dealt within one XCD
#endif

// Rows of the record table: group g (i1 = S3_NR g .. S3_NR g + 3) holds rows
// j = S3_NR g + 1 .. S - 2, starting at row s3_rowoff(S, g).
__host__ __device__ inline int64_t s3_rowoff(int64_t S, int64_t g) {
    // sum over g' < g of (S - 2 - S3_NR g')
    return g * (S - 2) - (int64_t)S3_NR * (g * (g - 1) / 2);
}
__host__ __device__ inline int64_t s3_rows(int64_t S) {
    const int64_t ng = (S - 3) / S3_NR + 1;  // groups with at least one row (S >= 3)
    return s3_rowoff(S, ng);
}

// record of (i1, j), i1 = S3_NR g + r, in row R = s3_rowoff(S, g) + j - S3_NR g - 1:
//   rec[(R S3_NR + r) 4 + {0, 1, 2, 3}] = {v, 1/d_j, z_j / s_j, p}
// with v = G[i1][j], d_j = 1 - v^2, s_j = sqrt(d_j), z_j = (b_j - v b_i1) / s_j,
// p = c - b_i1^2 - z_j^2 (the SSE of the pair); p = NaN (fails every
// comparison) unless i1 < j, column i1 is live and d_j > RANK_EPS.
// (its grid also does the per-search initialisation of search_init_kernel)
// Grid: x over (j, r) of one group, y over groups (blockIdx.y = g).
// Launched with PRE_WG threads per workgroup and one workgroup column more
// than the records need: workgroup (last, 0) runs the pre-pass selection
// (independent of the table and of the initialisation, which leaves the
// pre-pass count to it), beside the record workgroups.
__global__ __launch_bounds__(PRE_WG) void rec3_kernel(Ctx c, double *__restrict__ rec) {
    const int64_t ex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t g = blockIdx.y;
    search_init_body(c, g * (int64_t)gridDim.x * blockDim.x + ex, ex == 0 && g == 0, 3, SUBP, JBLK, 1, false);
    if (blockIdx.x == gridDim.x - 1 && g == 0) {
        pre_select_body<3>(c);
        return;
    }
    const int64_t S = c.S;
    const int r = (int)(ex % S3_NR);
    const int64_t j = S3_NR * g + 1 + ex / S3_NR;
    if (g > (S - 3) / S3_NR || j > S - 2) return;
    const int64_t i1 = S3_NR * g + r;
    const int64_t e = (s3_rowoff(S, g) + j - S3_NR * g - 1) * S3_NR + r;
    // the filter task's pair (i1, j) (the only task when T = 1)
    const int ts = c.tstar[0];
    const double *G1 = c.G1;
    const int64_t nt = c.Gnt;
    double v = 0.0, al = 0.0, zs = 0.0, p = __builtin_nan("");
    if (i1 < j && G1[gidx(i1, i1, nt, 1, 0)] > RANK_EPS) {
        const double zp = c.bhat[i1 * c.TP + ts];
        const double pp = c.cyy[ts] - zp * zp;
        const double g = G1[gidx(i1, j, nt, 1, 0)];
        const double d = G1[gidx(j, j, nt, 1, 0)] - g * g;
        if (d > RANK_EPS) {
            const double sj = sqrt(d);
            const double zn = (c.bhat[j * c.TP + ts] - g * zp) / sj;
            v = g;
            al = 1.0 / d;
            zs = zn / sj;
            p = pp - zn * zn;
        }
    }
    double *o = rec + e * 4;
    o[0] = v;
    o[1] = al;
    o[2] = zs;
    o[3] = p;
}

// Tiles of j-block jb (j in [S3_JR jb, S3_JR jb + S3_JR) and j <= S - 2):
// nkb column chunks (k from j0 + 1 to S - 1) times groups g < ng (the
// group's first i1 lies below the block's last j).
__host__ __device__ inline void s3_block(int64_t S, int64_t jb, int64_t &nkb, int64_t &ng) {
    const int64_t j0 = jb * S3_JR;
    int64_t jmax = j0 + S3_JR - 1;
    if (jmax > S - 2) jmax = S - 2;
    nkb = (S - j0 - 1 + S3_KC - 1) / S3_KC;
    ng = jmax >= 1 ? (jmax - 1) / S3_NR + 1 : 0;
}
__host__ __device__ inline int64_t s3_nblocks(int64_t S) { return S >= 3 ? (S - 2) / S3_JR + 1 : 0; }

// tcum[jb] = tiles of the blocks before jb (tcum[nblocks] = all tiles)
__device__ void s3_tile_table(const Ctx &c) {
    const int64_t nb = s3_nblocks(c.S);
    uint64_t acc = 0;
    c.cum[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t nkb, ng;
        s3_block(c.S, b, nkb, ng);
        acc += (uint64_t)(nkb * ng);
        c.cum[b + 1] = acc;
    }
    c.stats[1] = acc;
}

int s3_rows_per_tile() { return S3_JR; }

uint64_t s3_tiles_host(int64_t S) {
    const int64_t nb = s3_nblocks(S);
    uint64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t nkb, ng;
        s3_block(S, b, nkb, ng);
        acc += (uint64_t)(nkb * ng);
    }
    return acc;
}

#ifndef S3_WPE
#define S3_WPE 4                      // waves per SIMD the register budget is sized for
#endif
// Several tasks, D = 3: the exact scoring of queued sweep steps, in two
// phases per wave.  mt_step_candidates redoes, for one step (row j of group
// g, column chunk kcx, the flag masks of the step's two columns per lane),
// the filter task's test per i1 and column with a true division, and appends
// the tuples that pass (key, filter-task SSE) to the wave's LDS buffer.
// mt_flush then takes up to 64 buffered tuples, one per lane: the second
// largest task's SSE is added (a tighter lower bound), and the survivors are
// scored over every task, 64 / LT tuples at a time with LT lanes each (lane
// q LT + l sums the tasks t = l mod LT of tuple q, then a butterfly sum and
// rank flag), and inserted into the wave's list.
constexpr int MT_BUF = 128;  // buffered tuples per wave (a flush takes 64)

__device__ __forceinline__ unsigned mt_flush(const Ctx &c, double *Ls, uint64_t *Lr, int KP, const uint64_t *bk,
                                             const double *be, int cnt, double theta_f) {
    const int lane = threadIdx.x & 63;
    const int TP = c.TP, t2 = c.tstar[1];
    auto task_sse = [&](const int32_t (&tq)[3], int t, bool &ok) {
        double gm[3][3], bv[3];
#pragma unroll
        for (int m2 = 0; m2 < 3; ++m2) {
#pragma unroll
            for (int j2 = 0; j2 <= m2; ++j2) gm[m2][j2] = Gat(c, tq[m2], tq[j2], t);
            bv[m2] = c.bhat[(int64_t)tq[m2] * TP + t];
        }
        return ne_sse_core<3>(gm, bv, c.cyy[t], ok);
    };
    bool take = lane < cnt;
    const uint64_t key = take ? bk[lane] : 0;
    int32_t tup[3] = {0, 1, 2};
    if (take) {
        unpack_tuple(key, 3, tup);
        if (t2 >= 0) {
            bool ok2 = true;
            const double e2 = task_sse(tup, t2, ok2);
            take = ok2 && be[lane] + e2 <= theta_f;
        }
    }
    const int LT = TP < 64 ? TP : 64;
    const int R = 64 / LT, slot = lane / LT;
    unsigned offered = 0;
    unsigned long long m = __ballot(take);
    while (m) {
        int src = -1;
        for (int q = 0; q < R; ++q) {
            const int sb = m ? __ffsll((long long)m) - 1 : -1;
            if (slot == q) src = sb;
            m &= m - 1;
        }
        const uint64_t kq = (uint64_t)__shfl((long long)key, src < 0 ? 0 : src);
        double part = 0.0;
        bool okp = true;
        if (src >= 0) {
            int32_t tq[3];
            unpack_tuple(kq, 3, tq);
            for (int t = lane % LT; t < c.T; t += LT) part += task_sse(tq, t, okp);
        }
        for (int o = 1; o < LT; o <<= 1) {
            part += __shfl_xor(part, o);
            okp = __shfl_xor((int)okp, o) != 0 && okp;
        }
        const double esv = okp ? part : INF;
        for (int q = 0; q < R; ++q) {
            if (__shfl(src, q * LT) < 0) break;
            const double v2 = __shfl(esv, q * LT);
            const uint64_t k2 = (uint64_t)__shfl((long long)kq, q * LT);
            if (v2 <= fmin(theta_f, Ls[KP - 1])) {
                ++offered;
                list_insert(Ls, Lr, KP, v2, k2);
            }
        }
    }
    return offered;
}

__device__ __forceinline__ unsigned mt_step(const Ctx &c, const SearchArgs &a, const double *__restrict__ rec,
                                            double *Ls, uint64_t *Lr, int KP, uint64_t *bk, double *be, int &nbuf,
                                            int64_t j, int64_t g, int64_t kcx, unsigned long long fm0,
                                            unsigned long long fm1, double theta_f) {
    const int lane = threadIdx.x & 63;
    const int64_t S = c.S, nt = c.Gnt;
    const int TP = c.TP, ts = c.tstar[0];
    const double *__restrict__ G1 = c.G1;
    const double *__restrict__ inv_st = c.inv_s + (int64_t)ts * S;
    const int64_t kb = j - j % S3_JR + 1 + kcx * S3_KC;  // the tile's first column
    const int64_t k0 = kb + lane, k1 = kb + 64 + lane;
    const bool kv0 = k0 < S, kv1 = k1 < S;
    const int64_t kk = kv0 ? k0 : S - 1, kd1 = kv1 ? k1 : S - 1;
    const double gvx = G1[gidx(j, kk, nt, 1, 0)], gvy = G1[gidx(j, kd1, nt, 1, 0)];
    const double gd0 = inv_st[kk] > 0.0 ? 1.0 : 0.0, gd1 = inv_st[kd1] > 0.0 ? 1.0 : 0.0;
    const double b0 = c.bhat[kk * TP + ts], b1 = c.bhat[kd1 * TP + ts];
    const double *rp = rec + (s3_rowoff(S, g) + j - S3_NR * g - 1) * (S3_NR * 4);
    unsigned offered = 0;
#pragma unroll
    for (int r = 0; r < S3_NR; ++r) {
        const int64_t i1 = S3_NR * g + r, i1c = i1 < S ? i1 : S - 1;
        const double v = rp[4 * r], al = rp[4 * r + 1], zs = rp[4 * r + 2], p = rp[4 * r + 3];
        const double zp = c.bhat[i1c * TP + ts];
        const double wvx = G1[gidx(i1c, kk, nt, 1, 0)], wvy = G1[gidx(i1c, kd1, nt, 1, 0)];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const double w = sl ? wvy : wvx, gg = sl ? gvy : gvx, gd = sl ? gd1 : gd0;
            const int64_t k = sl ? k1 : k0;
            const double dq = ((sl ? kv1 : kv0) && gd > RANK_EPS) ? gd - w * w : __builtin_nan("");
            const double zq = (sl ? b1 : b0) - w * zp;
            const double u = fma(-v, w, gg);
            const double d = fma(-al, u * u, dq);
            const double z = fma(-zs, u, zq);
            const double es = (d > RANK_EPS) ? p - z * z / d : INF;
            const int32_t tup[3] = {(int32_t)i1, (int32_t)j, (int32_t)k};
            bool take = (((sl ? fm1 : fm0) >> lane) & 1ull) && k < S && k > j && es <= theta_f;
            if (take && a.ranged) {
                const uint64_t lr = lex_rank(BinomTab{c.btab, c.S}, c.S, 3, tup);
                if (lr < a.r0 || lr >= a.r1) take = false;
            }
            const unsigned long long m = __ballot(take);
            if (m) {
                if (take) {
                    const int at = nbuf + __popcll(m & ((1ull << lane) - 1ull));
                    bk[at] = pack_tuple(tup, 3);
                    be[at] = es;
                }
                nbuf += __popcll(m);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_wave_barrier();
                if (nbuf >= 64) {
                    offered += mt_flush(c, Ls, Lr, KP, bk, be, 64, theta_f);
                    // keep the rest (fewer than 64) at the front
                    const int rest = nbuf - 64;
                    uint64_t kx = 0;
                    double ex = 0.0;
                    if (lane < rest) {
                        kx = bk[64 + lane];
                        ex = be[64 + lane];
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_wave_barrier();
                    if (lane < rest) {
                        bk[lane] = kx;
                        be[lane] = ex;
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_wave_barrier();
                    nbuf = rest;
                }
            }
        }
    }
    return offered;
}

// One tile of the D = 3 record-table sweep (see search3_kernel): the tile's
// k-dependent terms, the sweep over its rows, exact scoring of the flagged
// steps into the wave's list (one task) or their queueing (several tasks),
// and the publication of the wave's bound.  Shared by the one-problem kernel
// and the batched kernel.
// CtxT: Ctx (a kernel argument) or a Ctx in the constant address space (a
// copy in device memory, read by the batched kernel): both let the compiler
// read the fields with scalar loads into scalar registers.
template <bool MT, class CtxT>
__device__ __forceinline__ void s3_tile(const CtxT &c, const SearchArgs &a, const double *__restrict__ rec,
                                        const uint64_t *__restrict__ tcum, uint64_t t, double *Ls, uint64_t *Lr,
                                        double theta0, double &theta_pub, unsigned &offered, int &qchunk, int &qn,
                                        unsigned long long (*s_qw)[2], int *s_qjw) {
    const int KP = a.KP;
    const int lane = threadIdx.x & 63;
    const int64_t S = c.S;
    const int64_t nb = s3_nblocks(S);
    const int64_t nt = c.Gnt;
    const double *__restrict__ Gb = c.G1;
    const int TP = c.TP;
    const int ts = c.tstar[0];
    const double *__restrict__ inv_st = c.inv_s + (int64_t)ts * S;
    {
        // tile -> (j-block, column chunk, group)
        int64_t lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (tcum[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int64_t jb = lo;
        int64_t nkb, ng;
        s3_block(S, jb, nkb, ng);
        // column chunk fastest: the waves of a workgroup usually take chunks
        // of one (block, group) and share its records in the scalar cache;
        // a run of tiles on one XCD covers a few groups over the same chunks
        // of G
        const int64_t rem = (int64_t)(t - tcum[jb]);
        const int64_t kcx = rem % nkb;
        const int64_t g = rem / nkb;
        const int64_t j0 = jb * S3_JR;
        const int64_t jlo = j0 > S3_NR * g + 1 ? j0 : S3_NR * g + 1;
        const int64_t jhi = (j0 + S3_JR - 1 < S - 2) ? j0 + S3_JR - 1 : S - 2;
        const int nrow = (int)(jhi - jlo);  // steps 0..nrow
        const int64_t kb = j0 + 1 + kcx * S3_KC;
        const int64_t k0 = kb + lane, k1 = kb + 64 + lane;
        const bool kv0 = k0 < S, kv1 = k1 < S;
        // columns read for lanes past S: any valid one (never passes)
        const int64_t kk0 = kv0 ? k0 : S - 1, kk1 = kv1 ? k1 : S - 1;
        const bool diag = kcx == 0;            // k <= j only in chunk 0, first half
        const bool half = S - kb <= 64;        // no column in the second half

        double th = fmin(theta0, theta_load(c.theta_bits));
        th = fmin(th, Ls[KP - 1]);
        const double theta_f = th < INF ? th * (1.0 + THETA_SLACK) : INF;

        // k-dependent part of each i1's solve, for both columns of the lane
        double w[S3_NR][2], dq[S3_NR][2], zq[S3_NR][2];
        {
            // G[k][k] is 1 for a live column and 0 for a constant one; the
            // contiguous 1/|x - mean| row says which (0 = constant)
            const double gd0 = inv_st[kk0] > 0.0 ? 1.0 : 0.0;
            const double gd1 = inv_st[kk1] > 0.0 ? 1.0 : 0.0;
            const double b0 = c.bhat[kk0 * TP + ts], b1 = c.bhat[kk1 * TP + ts];
#pragma unroll
            for (int r = 0; r < S3_NR; ++r) {
                int64_t i1 = S3_NR * g + r;
                if (i1 > S - 1) i1 = S - 1;
                const double zp = c.bhat[i1 * TP + ts];
                const double2 wv = {Gb[gidx(i1, kk0, nt, 1, 0)], Gb[gidx(i1, kk1, nt, 1, 0)]};
                w[r][0] = wv.x;
                w[r][1] = wv.y;
                // a lane past S or on a constant column never passes
                dq[r][0] = (kv0 && gd0 > RANK_EPS) ? gd0 - wv.x * wv.x : __builtin_nan("");
                dq[r][1] = (kv1 && gd1 > RANK_EPS) ? gd1 - wv.y * wv.y : __builtin_nan("");
                zq[r][0] = b0 - wv.x * zp;
                zq[r][1] = b1 - wv.y * zp;
            }
        }
        // G[j][k] for the block's rows: j >> 6 is the same for the whole block
        // (S3_JR divides 64), so one uniform tile-row base plus 32-bit per-lane
        // byte offsets (column part + row j & 63) address every step
        const char *__restrict__ gtile =
            reinterpret_cast<const char *>(Gb + (((j0 >> 6) * nt) << 12));
        const uint32_t voff0 = (uint32_t)((((kk0 >> 6) << 12) + (kk0 & 63) + ((jlo & 63) << 6)) * 8);
        const uint32_t voff1 = (uint32_t)((((kk1 >> 6) << 12) + (kk1 & 63) + ((jlo & 63) << 6)) * 8);
        // records of row jlo + x are 128 bytes at recj + 128 x (uniform)
        const char *__restrict__ recj =
            reinterpret_cast<const char *>(rec + (size_t)(s3_rowoff(S, g) + jlo - S3_NR * g - 1) * (S3_NR * 4));
        int nq = 0;
        auto sweep = [&](auto diagc, auto halfc) {
            constexpr bool DIAG = decltype(diagc)::value;
            constexpr bool HALF = decltype(halfc)::value;
            constexpr int JG = S3_JG;
            double2 ga[JG], gb[JG];  // g(j, k0), g(j, k1)
            auto fetch = [&](double2 (&dst)[JG], int jg) {
#pragma unroll
                for (int x = 0; x < JG; ++x) {
                    const uint32_t jr = (uint32_t)(jg + x < nrow ? jg + x : nrow);
                    dst[x].x = *reinterpret_cast<const double *>(gtile + (voff0 + jr * 512u));
                    dst[x].y = HALF ? 0.0 : *reinterpret_cast<const double *>(gtile + (voff1 + jr * 512u));
                }
            };
            // records of one step are two halves of 64 bytes (i1 = 4g, 4g+1 and
            // 4g+2, 4g+3); each half is loaded while the other is scored.  Scalar
            // loads may return out of order, so the half in flight is waited for
            // (lgkmcnt(0)) before the next one is issued.
            auto load_half = [&](double (&rv)[8], int jr, int h) {
                const double *rp = reinterpret_cast<const double *>(recj + (size_t)jr * 128 + h * 64);
#pragma unroll
                for (int e = 0; e < 8; ++e) rv[e] = rp[e];
            };
            auto score_half = [&](const double (&rv)[8], const double2 gv, int h, unsigned long long &m0,
                                  unsigned long long &m1) {
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    const int r = 2 * h + rr;
                    const double pi = rv[4 * rr + 3] - theta_f;
                    {
                        const double u = fma(-rv[4 * rr], w[r][0], gv.x);
                        const double d = fma(-rv[4 * rr + 1], u * u, dq[r][0]);
                        const double z = fma(-rv[4 * rr + 2], u, zq[r][0]);
                        m0 |= __ballot(z * z >= pi * d);
                    }
                    if (!HALF) {
                        const double u = fma(-rv[4 * rr], w[r][1], gv.y);
                        const double d = fma(-rv[4 * rr + 1], u * u, dq[r][1]);
                        const double z = fma(-rv[4 * rr + 2], u, zq[r][1]);
                        m1 |= __ballot(z * z >= pi * d);
                    }
                }
            };
            double ra[8], rb[8];
            load_half(ra, 0, 0);
            auto score = [&](const double2 (&src)[JG], int jg) {
#pragma unroll
                for (int x = 0; x < JG; ++x) {
                    const int jr = jg + x;
                    const int jc = jr <= nrow ? jr : nrow;
                    unsigned long long m0 = 0, m1 = 0;
                    __builtin_amdgcn_s_waitcnt(0xC07F);
                    load_half(rb, jc, 1);
                    __builtin_amdgcn_sched_barrier(0);
                    score_half(ra, src[x], 0, m0, m1);
                    __builtin_amdgcn_s_waitcnt(0xC07F);
                    load_half(ra, jr + 1 <= nrow ? jr + 1 : nrow, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    score_half(rb, src[x], 1, m0, m1);
                    if (DIAG) m0 &= __ballot(k0 > jlo + jr);  // k1 > j0 + 64 > j
                    if (jr > nrow) m0 = m1 = 0;
                    if (m0 | m1) {
                        if (lane == 0) {
                            s_qw[nq][0] = m0;
                            s_qw[nq][1] = m1;
                            s_qjw[nq] = jr;
                        }
                        ++nq;
                    }
                }
            };
            __builtin_amdgcn_s_waitcnt(0x0F70);
            fetch(ga, 0);
            for (int jg = 0;; jg += 2 * JG) {
                fetch(gb, jg + JG);
                score(ga, jg);
                fetch(ga, jg + 2 * JG);
                score(gb, jg + JG);
                if (jg + 2 * JG > nrow) break;
            }
        };
        if (diag) {
            if (half) sweep(std::true_type{}, std::true_type{});
            else sweep(std::true_type{}, std::false_type{});
        } else {
            if (half) sweep(std::false_type{}, std::true_type{});
            else sweep(std::false_type{}, std::false_type{});
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();

        // exact scoring of the flagged steps (rare): the same terms, a true
        // division, the rank test and the current bound
        for (int e = 0; e < nq; ++e) {
            const int jr = s_qjw[e];
            const int64_t j = jlo + jr;
            const unsigned long long fm[2] = {s_qw[e][0], s_qw[e][1]};
            if (MT) {
                // several tasks: queue the step (row j of group g, chunk kcx,
                // the flags); a later, evenly spread kernel scores it.  The
                // pool holds a record per sweep step plus a partly filled
                // chunk per wave, so a take past its end cannot happen; it
                // would be reported, not dropped silently
                if (qchunk >= 0 && qn == MTQ_CHUNK) {
                    if (lane == 0) c.mtq_n[qchunk] = (uint32_t)qn;
                    unsigned got = 0;
                    if (lane == 0) got = atomicAdd(c.mtq_taken, 1u);
                    got = (unsigned)__shfl((int)got, 0) + gridDim.x * SEARCH_WAVES;
                    qchunk = got < (unsigned)c.mtq_chunks ? (int)got : -2;
                    if (qchunk == -2 && lane == 0) atomicOr(&c.flags[FLAG_CAPACITY], 1u);
                    qn = 0;
                }
                if (qchunk >= 0) {
                    if (lane < 3) {
                        const uint64_t w0 = ((uint64_t)j << 40) | ((uint64_t)g << 20) | (uint64_t)kcx;
                        c.mtq[((int64_t)qchunk * MTQ_CHUNK + qn) * 3 + lane] = lane == 0 ? w0 : lane == 1 ? fm[0] : fm[1];
                    }
                    ++qn;
                }
                continue;
            }
            const double *rp = reinterpret_cast<const double *>(recj + (size_t)jr * 128);
            const double2 gv = {*reinterpret_cast<const double *>(gtile + (voff0 + (uint32_t)jr * 512u)),
                                *reinterpret_cast<const double *>(gtile + (voff1 + (uint32_t)jr * 512u))};
            // (r, sl) are wave-uniform here: pick the k-data by selects, so
            // the arrays stay in registers (an indexed read would move them to
            // scratch memory, stored on every tile)
            auto pick = [&](const double (&arr)[S3_NR][2], int r, int sl) {
                double v = arr[0][0];
#pragma unroll
                for (int q = 0; q < S3_NR; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if (q == r && h == sl) v = arr[q][h];
                return v;
            };
            for (int r = 0; r < S3_NR; ++r) {
                const double v = rp[4 * r], al = rp[4 * r + 1], zs = rp[4 * r + 2], p = rp[4 * r + 3];
                for (int sl = 0; sl < 2; ++sl) {
                    const double gg = sl ? gv.y : gv.x;
                    const int64_t k = sl ? k1 : k0;
                    const double u = fma(-v, pick(w, r, sl), gg);
                    const double d = fma(-al, u * u, pick(dq, r, sl));
                    const double z = fma(-zs, u, pick(zq, r, sl));
                    const int32_t tup[3] = {(int32_t)(S3_NR * g + r), (int32_t)j, (int32_t)k};
                    // the step's flag covers all four i1 of the group: this
                    // i1's own terms decide (NaN records: i1 >= j or a rank
                    // deficient pair)
                    const double es = (d > RANK_EPS) ? p - z * z / d : INF;
                    bool take = ((fm[sl] >> lane) & 1ull) && k < S && k > j && es <= fmin(theta_f, Ls[KP - 1]);
                    if (take && a.ranged) {
                        const uint64_t lr = lex_rank(BinomTab{c.btab, c.S}, c.S, 3, tup);
                        if (lr < a.r0 || lr >= a.r1) take = false;
                    }
                    unsigned long long m = __ballot(take);
                    const uint64_t rk = take ? pack_tuple(tup, 3) : 0;
                    offered += (unsigned)__popcll(m);
                    while (m) {
                        const int src = __ffsll((long long)m) - 1;
                        m &= m - 1;
                        const double cs = __shfl(es, src);
                        const uint64_t cr = (uint64_t)__shfl((long long)rk, src);
                        list_insert(Ls, Lr, KP, cs, cr);
                    }
                }
            }
        }
        const double tw = Ls[KP - 1];
        if (tw < theta_pub) {
            theta_pub = tw;
            if (lane == 0) theta_publish(c.theta_bits, tw);
        }
    }
}

// MT: several tasks (the sweep filters on the filter task alone, the exact
// path sums every task); a template parameter so that the one-task kernel's
// registers are not shaped by the several-task exact path
template <bool MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S3_WPE))) void search3_kernel(Ctx c, SearchArgs a, const double *__restrict__ rec,
                                                      const uint64_t *__restrict__ tcum) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_q[SEARCH_WAVES][S3_JR][2];
    __shared__ int s_qj[SEARCH_WAVES][S3_JR];
    const int KP = a.KP;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    for (int m = lane; m < KP; m += 64) {
        Ls[m] = INF;
        Lr[m] = ~0ull;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    double theta_pub = INF;
    unsigned offered = 0;
    const double theta0 = theta0_from_prepass(c, a.L, KP);
    const uint64_t ntiles = tcum[s3_nblocks(c.S)];
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    // several tasks: flagged steps are queued in chunks of MTQ_CHUNK and scored
    // by a later, evenly spread kernel (the steps cluster in the few tiles of
    // the best features); wave gw owns chunk gw, further chunks come from the
    // pool above the launched waves' own, one atomic each
    int qchunk = MT ? (int)gw : -1, qn = 0;

    // Tiles are dealt round-robin over the waves (their costs are nearly
    // equal; a shared counter would serialise on one address), XCD-aware:
    // workgroups are placed on the eight XCDs in turn (workgroup b on XCD
    // b mod 8), and runs of S3_XCD_RUN consecutive tiles, which share blocks
    // of G, go to the waves of one XCD and its L2.
    const bool xa = (gridDim.x % S3_XCDS) == 0;
    const uint64_t xcd = xa ? blockIdx.x % S3_XCDS : 0;
    const uint64_t nx = xa ? S3_XCDS : 1;
    const uint64_t U = (uint64_t)gridDim.x / nx * SEARCH_WAVES;      // waves per XCD
    const uint64_t u0 = (uint64_t)blockIdx.x / nx * SEARCH_WAVES + wave;
    for (uint64_t sx = u0;; sx += U) {
        const uint64_t t = ((sx / S3_XCD_RUN) * nx + xcd) * S3_XCD_RUN + sx % S3_XCD_RUN;
        if (t >= ntiles) break;
        s3_tile<MT, Ctx>(c, a, rec, tcum, t, Ls, Lr, theta0, theta_pub, offered, qchunk, qn, s_q[wave], s_qj[wave]);
    }
    if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
    if (MT && qchunk >= 0 && lane == 0) c.mtq_n[qchunk] = (uint32_t)qn;
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// ---------------------------------------- batched D = 3 search (one task)
#ifndef S3B_WPE
#define S3B_WPE 3                     // waves per SIMD of the batched kernel (its per-problem state)
#endif
// Several independent one-task problems searched by one launch: the record
// tables and pre-pass bounds of every problem are built first (each problem
// on its own), then the waves of one persistent grid pull work items from a
// device queue -- item = a run of S3B_RUN consecutive tiles of one problem,
// problems ordered by decreasing tile count, so the largest start first and
// the small ones fill the tail.  A wave keeps one list per problem it works
// on: when its next item belongs to another problem it writes the list to
// that problem's next free list slot (a wave never returns to a problem, as
// items are taken in queue order) and starts an empty one.  Each problem's
// merge then reads the lists its waves wrote; the rest is the one-problem
// path, so the results equal those of separate searches bitwise.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S3B_WPE))) void search3_batch_kernel(
    BatchSearchArgs b) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_q[SEARCH_WAVES][S3_JR][2];
    __shared__ int s_qj[SEARCH_WAVES][S3_JR];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *Ls = smem + (size_t)wave * b.KPmax * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + b.KPmax);
    uint32_t *queue = b.ctx[0]->flags + FLAG_BATCHQ;
    const uint32_t nitems = b.item_end[b.P - 1];
    int cur = -1, qchunk = -1, qn = 0;
    const Ctx *cur_ctx = nullptr;
    double theta0 = INF, theta_pub = INF;
    unsigned offered = 0;
    SearchArgs a{};
    a.D = 3;
    auto flush = [&](const Ctx &c) {
        uint32_t slot = 0;
        if (lane == 0) slot = atomicAdd(c.flags + FLAG_NLISTS, 1u);
        slot = (uint32_t)__shfl((int)slot, 0);
        if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
        if (slot < (uint32_t)c.nwaves)
            list_store(c.list_sse + (int64_t)slot * a.KP, c.list_rank + (int64_t)slot * a.KP, Ls, Lr, a.KP);
    };
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(queue, 1u);
        it = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)__shfl((int)it, 0));
        if (it >= nitems) break;
        typedef const __attribute__((address_space(4))) uint32_t CU32;
        typedef const __attribute__((address_space(4))) uint64_t CU64;
        CU32 *ie = (CU32 *)(uintptr_t)b.item_end;
        int p = 0;
        while (ie[p] <= it) ++p;
        p = __builtin_amdgcn_readfirstlane(p);
        const uint32_t first = p ? ie[p - 1] : 0u;
        const Ctx *cp = (const Ctx *)(uintptr_t)((CU64 *)(uintptr_t)b.ctx)[p];
        typedef const __attribute__((address_space(4))) Ctx CCtx;
        CCtx &c = *(CCtx *)(uintptr_t)cp;
        if (p != cur) {
            if (cur >= 0) flush(*cur_ctx);
            cur_ctx = cp;
            cur = p;
            a.KP = c.KP;
            a.L = (c.KP + PRE_Q - 1) / PRE_Q;
            for (int m = lane; m < a.KP; m += 64) {
                Ls[m] = INF;
                Lr[m] = ~0ull;
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
            theta0 = theta0_from_prepass(c, a.L, a.KP);
            theta_pub = INF;
            offered = 0;
        }
        const uint64_t ntiles = c.cum[s3_nblocks(c.S)];
        const uint64_t t0 = (uint64_t)(it - first) * S3B_RUN;
        const uint64_t t1 = t0 + S3B_RUN < ntiles ? t0 + S3B_RUN : ntiles;
        for (uint64_t t = t0; t < t1; ++t)
            s3_tile<false, CCtx>(c, a, c.rec3, c.cum, t, Ls, Lr, theta0, theta_pub, offered, qchunk, qn, s_q[wave],
                                 s_qj[wave]);
    }
    if (cur >= 0) flush(*cur_ctx);
}

// ------------------------------------------- D = 4, one task: record table
// The D = 3 design one level up.  For every prefix (i1, i2, j) the Cholesky
// row of j against the pair is built once per search into a table
// (rec4_kernel); the sweep reads the rows of one pair group (four i1 with
// the same i2) for one j with scalar loads, so the records enter the FP64
// instructions as scalar operands.  A work tile is (pair group, S4_JR rows j
// from j0, S4_KC columns k from j0 + 1 + S4_KC c): lane l takes k = kb + l and
// kb + 64 + l, so only chunk 0 holds tuples with k <= j (in its first half),
// and a last chunk with at most 64 columns left runs its first half only.
// Per tuple, with the pair's
// k-dependent terms w0 = G[i1][k], w1 = (G[i2][k] - r w0) / s (r = G[i1][i2],
// s = sqrt(1 - r^2)), d' = G[k][k] - w0^2 - w1^2 and zeta' = b_k - w0 z0 -
// w1 z1 held in registers for the tile:
//   u = g - v0 w0 - v1 w1,  d = d' - alpha u^2,  zeta = zeta' - zs u,
//   pass iff zeta^2 >= (p - theta) d.
// Record of (i1, i2, j), i1 = 4 h + r in group (i2, h), row
// R = r4off[i2] + h (S - 2 - i2) + j - i2 - 1:
//   rec[(R S4_NR + r) S4_RECW + {0..4}] = {v0, v1, 1/d_j, z_j / s_j, p}
// with v0 = G[i1][j], v1 = (G[i2][j] - r v0) / s, d_j = G[j][j] - v0^2 - v1^2,
// z0 = b_i1, z1 = (b_i2 - r z0) / s, z_j = (b_j - v0 z0 - v1 z1) / s_j,
// s_j = sqrt(d_j), p = c - z0^2 - z1^2 - z_j^2 (the SSE of the triple);
// p = NaN (fails every comparison) unless i1 < i2 < j, column i1 is live,
// 1 - r^2 > RANK_EPS and d_j > RANK_EPS.
#ifndef S4_WPE
#define S4_WPE 3                      // waves per SIMD the register budget is sized for
#endif
#ifndef S4_WRUN
#define S4_WRUN 4                     // consecutive tiles per wave
#endif
// row block jb: nkb column chunks (k from j0 + 1 to S - 1) and ng pair groups
__host__ __device__ inline void s4_block(int64_t S, int64_t jb, int64_t &nkb, int64_t &ng) {
    const int64_t j0 = jb * S4_JR;
    int64_t jmax = j0 + S4_JR - 1;
    if (jmax > S - 2) jmax = S - 2;
    nkb = (S - j0 - 1 + S4_KC - 1) / S4_KC;
    ng = jmax >= 2 ? s4_groups_below(jmax) : 0;  // groups with i2 < jmax
}
__host__ __device__ inline int64_t s4_nblocks(int64_t S) { return S >= 4 ? (S - 2) / S4_JR + 1 : 0; }

// pair group index -> (i2, h): i2 is the largest index whose groups start at or before g
__device__ inline int64_t s4_group_i2(int64_t S, int64_t g) {
    int64_t lo = 1, hi = S - 3;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (s4_groups_below(mid) <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// tcum[jb] = tiles of the blocks before jb; r4off[i] = record rows of the
// groups with i2 < i (serial, leader thread of the initialisation)
__device__ void s4_tables(const Ctx &c) {
    const int64_t S = c.S;
    const int64_t nb = s4_nblocks(S);
    uint64_t acc = 0;
    c.cum[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t nkb, ng;
        s4_block(S, b, nkb, ng);
        acc += (uint64_t)(nkb * ng);
        c.cum[b + 1] = acc;
    }
    c.stats[1] = acc;
    int64_t rows = 0;
    for (int64_t i = 0; i <= S; ++i) {
        c.r4off[i] = rows;
        if (i >= 1 && i <= S - 3) rows += ((i + 3) / 4) * (S - 2 - i);
    }
}

uint64_t s4_tiles_host(int64_t S) {
    const int64_t nb = s4_nblocks(S);
    uint64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t nkb, ng;
        s4_block(S, b, nkb, ng);
        acc += (uint64_t)(nkb * ng);
    }
    return acc;
}

// first record row and row count of tile t
__device__ inline void s4_tile_rows(const Ctx &c, const uint64_t *__restrict__ tcum, int64_t nb, uint64_t t,
                                    int64_t &row, int64_t &nrows) {
    const int64_t S = c.S;
    int64_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (tcum[mid] <= t) lo = mid; else hi = mid - 1;
    }
    int64_t nkb, ng;
    s4_block(S, lo, nkb, ng);
    const int64_t grp = (int64_t)(t - tcum[lo]) / nkb;
    const int64_t i2 = s4_group_i2(S, grp);
    const int64_t hh = grp - s4_groups_below(i2);
    const int64_t j0 = lo * S4_JR;
    const int64_t jlo = j0 > i2 + 1 ? j0 : i2 + 1;
    const int64_t jhi = (j0 + S4_JR - 1 < S - 2) ? j0 + S4_JR - 1 : S - 2;
    row = c.r4off[i2] + hh * (S - 2 - i2) + (jlo - i2 - 1);
    nrows = jhi - jlo + 1;
}

__global__ void s4_init_kernel(Ctx c) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    search_init_body(c, e, e == 0, 4, SUBP, JBLK, 4);
}

// One thread per record, over the table in storage order: the row's pair
// group comes from a search of r4off (the threads of a workgroup share it
// but for the workgroups that straddle two values of i2).
// zs = z_j / s_j = e / d_j and z_j^2 = e^2 / d_j with e = b_j - v0 z0 - v1 z1,
// so a record takes one division and no root.
__global__ __launch_bounds__(256) void rec4_kernel(Ctx c, double *__restrict__ rec, int64_t nrec) {
    // the workgroup's records are staged in LDS and written out as
    // consecutive doubles (full cache lines), not as S4_RECW strided stores
    __shared__ double stage[256 * S4_RECW];
    const int64_t S = c.S;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t e = e0 + threadIdx.x;
    const int64_t ecl = e < nrec ? e : nrec - 1;  // a thread past the end computes the last record, unwritten
    const int r = (int)(ecl & (S4_NR - 1));
    const int64_t row = ecl / S4_NR;
    // i2: the largest index in [1, S - 3] whose rows start at or before row
    int64_t lo = 1, hi = S - 3;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (c.r4off[mid] <= row) lo = mid; else hi = mid - 1;
    }
    const int64_t i2 = lo;
    const int64_t nrow = S - 2 - i2;
    const int64_t loc = row - c.r4off[i2];
    const int64_t h = loc / nrow;
    const int64_t j = i2 + 1 + (loc - h * nrow);
    const int64_t i1 = S4_NR * h + r;
    const int64_t nt = c.Gnt;
    const double *__restrict__ G = c.G;
    double v0 = 0.0, v1 = 0.0, al = 0.0, zs = 0.0, p = __builtin_nan("");
    if (i1 < i2 && G[gidx(i1, i1, nt, 1, 0)] > RANK_EPS) {
        const double rr = G[gidx(i1, i2, nt, 1, 0)];
        const double s2 = G[gidx(i2, i2, nt, 1, 0)] - rr * rr;
        if (s2 > RANK_EPS) {
            const double isp = 1.0 / sqrt(s2);
            const double z0 = c.bhat[i1];
            const double z1 = (c.bhat[i2] - rr * z0) * isp;
            const double a0 = G[gidx(i1, j, nt, 1, 0)];
            const double a1 = (G[gidx(i2, j, nt, 1, 0)] - rr * a0) * isp;
            const double d = G[gidx(j, j, nt, 1, 0)] - a0 * a0 - a1 * a1;
            if (d > RANK_EPS) {
                const double id = 1.0 / d;
                const double ee = c.bhat[j] - a0 * z0 - a1 * z1;
                v0 = a0;
                v1 = a1;
                al = id;
                zs = ee * id;
                p = c.cyy[0] - z0 * z0 - z1 * z1 - ee * zs;
            }
        }
    }
    double *o = stage + threadIdx.x * S4_RECW;
    o[0] = v0;
    o[1] = v1;
    o[2] = al;
    o[3] = zs;
    o[4] = p;
    __syncthreads();
    const int64_t nvals = (nrec - e0 < 256 ? nrec - e0 : 256) * S4_RECW;
    double *out = rec + e0 * S4_RECW;
    for (int64_t q = threadIdx.x; q < nvals; q += 256) out[q] = stage[q];
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S4_WPE))) void search4_kernel(
    Ctx c, SearchArgs a, const double *__restrict__ rec, const uint64_t *__restrict__ tcum) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_q[SEARCH_WAVES][S4_JR][2];
    __shared__ int s_qj[SEARCH_WAVES][S4_JR];
    const int KP = a.KP;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    for (int m = lane; m < KP; m += 64) {
        Ls[m] = INF;
        Lr[m] = ~0ull;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    double theta_pub = INF;
    unsigned offered = 0;
    const double theta0 = theta0_from_prepass(c, a.L, KP);
    const int64_t S = c.S;
    const int64_t nb = s4_nblocks(S);
    const uint64_t ntiles = tcum[nb];
    const int64_t nt = c.Gnt;
    const double *__restrict__ Gb = c.G;
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    const double *__restrict__ inv_st = c.inv_s;

    // tiles dealt round-robin, XCD-aware, as in search3_kernel
    const bool xa = (gridDim.x % S3_XCDS) == 0;
    const uint64_t xcd = xa ? blockIdx.x % S3_XCDS : 0;
    const uint64_t nx = xa ? S3_XCDS : 1;
    const uint64_t U = (uint64_t)gridDim.x / nx * SEARCH_WAVES;
    const uint64_t u0 = (uint64_t)blockIdx.x / nx * SEARCH_WAVES + wave;
    // a wave takes S4_WRUN consecutive tiles (the column chunks of one pair
    // group and row block share its record rows, which the later ones find in
    // L2); runs are dealt round-robin and XCD-aware as tiles are in
    // search3_kernel
    for (uint64_t sx = u0;; sx += U) {
        const uint64_t run = ((sx / S3_XCD_RUN) * nx + xcd) * S3_XCD_RUN + sx % S3_XCD_RUN;
        if (run * S4_WRUN >= ntiles) break;
        const uint64_t tend = run * S4_WRUN + S4_WRUN < ntiles ? run * S4_WRUN + S4_WRUN : ntiles;
        for (uint64_t t = run * S4_WRUN; t < tend; ++t) {
        int64_t lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (tcum[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int64_t jb = lo;
        int64_t nkb, ng;
        s4_block(S, jb, nkb, ng);
        const int64_t rem = (int64_t)(t - tcum[jb]);
        const int64_t kcx = rem % nkb;
        const int64_t grp = uni(rem / nkb);
        const int64_t i2 = uni(s4_group_i2(S, grp));
        const int64_t hh = grp - s4_groups_below(i2);
        const int64_t j0 = jb * S4_JR;
        const int64_t jlo = j0 > i2 + 1 ? j0 : i2 + 1;
        const int64_t jhi = (j0 + S4_JR - 1 < S - 2) ? j0 + S4_JR - 1 : S - 2;
        const int nrow = (int)(jhi - jlo);  // steps 0..nrow (>= 0: i2 < jhi)
        // the next tile of this wave that starts a new pair group: touch each
        // 128-byte line of its record rows now, so that its scalar loads find
        // them in L2
        double pf = 0.0;
        {
            uint64_t tn = ~0ull;
            if (t + 1 < tend) {
                if ((rem + 1) % nkb == 0) tn = t + 1;
            } else {
                const uint64_t sn = sx + U;
                const uint64_t rn = ((sn / S3_XCD_RUN) * nx + xcd) * S3_XCD_RUN + sn % S3_XCD_RUN;
                if (rn * S4_WRUN < ntiles) tn = rn * S4_WRUN;
            }
            if (tn != ~0ull) {
                int64_t prow, pn;
                s4_tile_rows(c, tcum, nb, tn, prow, pn);
                const int64_t bytes = pn * S4_ROW * 8;
                if ((int64_t)lane * 128 < bytes)
                    pf = rec[(size_t)prow * S4_ROW + (size_t)lane * 16];
            }
        }
        const int64_t kb = j0 + 1 + kcx * S4_KC;
        const int64_t k0 = kb + lane, k1 = kb + 64 + lane;
        const bool kv0 = k0 < S, kv1 = k1 < S;
        // columns read for lanes past S: any valid one (never passes)
        const int64_t kk0 = kv0 ? k0 : S - 1, kk1 = kv1 ? k1 : S - 1;
        const bool diag = kcx == 0;            // k <= j only in chunk 0, first half
        const bool half = S - kb <= 64;        // no column in the second half

        double th = fmin(theta0, theta_load(c.theta_bits));
        th = fmin(th, Ls[KP - 1]);
        const double theta_f = th < INF ? th * (1.0 + THETA_SLACK) : INF;

        // k-dependent part of each pair's solve, for both columns of the lane
        double w0[S4_NR][2], w1[S4_NR][2], dq[S4_NR][2], zq[S4_NR][2];
        {
            const double gd0 = inv_st[kk0] > 0.0 ? 1.0 : 0.0;
            const double gd1 = inv_st[kk1] > 0.0 ? 1.0 : 0.0;
            const double b0 = c.bhat[kk0], b1 = c.bhat[kk1];
            const double w2x = Gb[gidx(i2, kk0, nt, 1, 0)], w2y = Gb[gidx(i2, kk1, nt, 1, 0)];
            const double zb2 = c.bhat[i2];
            const bool live2 = inv_st[i2] > 0.0;
#pragma unroll
            for (int r = 0; r < S4_NR; ++r) {
                int64_t i1 = S4_NR * hh + r;
                const bool pin = i1 < i2;
                if (!pin) i1 = i2;  // a void pair reads valid memory and never passes
                const double rr = Gb[gidx(i1, i2, nt, 1, 0)];
                const double s2 = (live2 ? 1.0 : 0.0) - rr * rr;
                const bool pv = pin && inv_st[i1] > 0.0 && s2 > RANK_EPS;
                const double isp = pv ? 1.0 / sqrt(s2) : 0.0;
                const double z0 = c.bhat[i1];
                const double z1 = (zb2 - rr * z0) * isp;
                const double a0 = Gb[gidx(i1, kk0, nt, 1, 0)], a1 = Gb[gidx(i1, kk1, nt, 1, 0)];
                const double c0 = (w2x - rr * a0) * isp, c1 = (w2y - rr * a1) * isp;
                w0[r][0] = a0;
                w0[r][1] = a1;
                w1[r][0] = c0;
                w1[r][1] = c1;
                // a lane past S, a constant column or a void pair never passes
                dq[r][0] = (pv && kv0 && gd0 > RANK_EPS) ? gd0 - a0 * a0 - c0 * c0 : __builtin_nan("");
                dq[r][1] = (pv && kv1 && gd1 > RANK_EPS) ? gd1 - a1 * a1 - c1 * c1 : __builtin_nan("");
                zq[r][0] = b0 - a0 * z0 - c0 * z1;
                zq[r][1] = b1 - a1 * z0 - c1 * z1;
            }
        }
        const char *__restrict__ gtile = reinterpret_cast<const char *>(Gb + (((j0 >> 6) * nt) << 12));
        // byte offsets of (jlo, k) in the 64 x 64 tile row of j0 (rows jlo .. jhi stay in it)
        const uint32_t voff0 = (uint32_t)((((kk0 >> 6) << 12) + (kk0 & 63) + ((jlo & 63) << 6)) * 8);
        const uint32_t voff1 = (uint32_t)((((kk1 >> 6) << 12) + (kk1 & 63) + ((jlo & 63) << 6)) * 8);
        // records of row jlo + x are S4_ROW doubles at recj + S4_ROW x (uniform)
        const double *__restrict__ recj =
            rec + (size_t)(c.r4off[i2] + hh * (S - 2 - i2) + (jlo - i2 - 1)) * S4_ROW;
        int nq = 0;
        auto sweep = [&](auto diagc, auto halfc) {
            constexpr bool DIAG = decltype(diagc)::value;
            constexpr bool HALF = decltype(halfc)::value;
            constexpr int JG = S3_JG;
            double2 ga[JG], gb[JG];  // g(j, k0), g(j, k1)
            auto fetch = [&](double2 (&dst)[JG], int jg) {
#pragma unroll
                for (int x = 0; x < JG; ++x) {
                    const uint32_t jr = (uint32_t)(jg + x < nrow ? jg + x : nrow);
                    dst[x].x = *reinterpret_cast<const double *>(gtile + (voff0 + jr * 512u));
                    dst[x].y = HALF ? 0.0 : *reinterpret_cast<const double *>(gtile + (voff1 + jr * 512u));
                }
            };
            // records of one step: two halves of two pairs (10 doubles each),
            // each loaded while the other is scored (scalar loads return out of
            // order, so the half in flight is waited for before the next issue)
            constexpr int HW = 2 * S4_RECW;
            auto load_half = [&](double (&rv)[HW], int jr, int h) {
                const double *rp = recj + (size_t)jr * S4_ROW + h * HW;
#pragma unroll
                for (int e = 0; e < HW; ++e) rv[e] = rp[e];
            };
            auto score_half = [&](const double (&rv)[HW], const double2 gv, int h, unsigned long long &m0,
                                  unsigned long long &m1) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int r = 2 * h + q;
                    const double *x = rv + q * S4_RECW;
                    const double pi = x[4] - theta_f;
                    {
                        const double u = fma(-x[1], w1[r][0], fma(-x[0], w0[r][0], gv.x));
                        const double d = fma(-x[2], u * u, dq[r][0]);
                        const double z = fma(-x[3], u, zq[r][0]);
                        m0 |= __ballot(z * z >= pi * d);
                    }
                    if (!HALF) {
                        const double u = fma(-x[1], w1[r][1], fma(-x[0], w0[r][1], gv.y));
                        const double d = fma(-x[2], u * u, dq[r][1]);
                        const double z = fma(-x[3], u, zq[r][1]);
                        m1 |= __ballot(z * z >= pi * d);
                    }
                }
            };
            double ra[HW], rb[HW];
            load_half(ra, 0, 0);
            auto score = [&](const double2 (&src)[JG], int jg) {
#pragma unroll
                for (int x = 0; x < JG; ++x) {
                    const int jr = jg + x;
                    const int jc = jr <= nrow ? jr : nrow;
                    unsigned long long m0 = 0, m1 = 0;
                    __builtin_amdgcn_s_waitcnt(0xC07F);
                    load_half(rb, jc, 1);
                    __builtin_amdgcn_sched_barrier(0);
                    score_half(ra, src[x], 0, m0, m1);
                    __builtin_amdgcn_s_waitcnt(0xC07F);
                    load_half(ra, jr + 1 <= nrow ? jr + 1 : nrow, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    score_half(rb, src[x], 1, m0, m1);
                    if (DIAG) m0 &= __ballot(k0 > jlo + jr);  // k1 > j0 + 64 > j
                    if (jr > nrow) m0 = m1 = 0;
                    if (m0 | m1) {
                        if (lane == 0) {
                            s_q[wave][nq][0] = m0;
                            s_q[wave][nq][1] = m1;
                            s_qj[wave][nq] = jr;
                        }
                        ++nq;
                    }
                }
            };
            __builtin_amdgcn_s_waitcnt(0x0F70);
            fetch(ga, 0);
            for (int jg = 0;; jg += 2 * JG) {
                fetch(gb, jg + JG);
                score(ga, jg);
                fetch(ga, jg + 2 * JG);
                score(gb, jg + JG);
                if (jg + 2 * JG > nrow) break;
            }
        };
        if (diag) {
            if (half) sweep(std::true_type{}, std::true_type{});
            else sweep(std::true_type{}, std::false_type{});
        } else {
            if (half) sweep(std::false_type{}, std::true_type{});
            else sweep(std::false_type{}, std::false_type{});
        }
        asm volatile("; prefetched %0" ::"v"(pf));  // the load stays (its value is not needed)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();

        // exact scoring of the flagged steps (rare): the same terms, a true
        // division, the rank test and the current bound
        auto pick = [&](const double (&arr)[S4_NR][2], int r, int sl) {
            double v = arr[0][0];
#pragma unroll
            for (int q = 0; q < S4_NR; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (q == r && h == sl) v = arr[q][h];
            return v;
        };
        for (int e = 0; e < nq; ++e) {
            const int jr = s_qj[wave][e];
            const int64_t j = jlo + jr;
            const unsigned long long fm[2] = {s_q[wave][e][0], s_q[wave][e][1]};
            const double *rp = recj + (size_t)jr * S4_ROW;
            const double gv0 = *reinterpret_cast<const double *>(gtile + (voff0 + (uint32_t)jr * 512u));
            const double gv1 = *reinterpret_cast<const double *>(gtile + (voff1 + (uint32_t)jr * 512u));
            for (int r = 0; r < S4_NR; ++r) {
                const double *x = rp + r * S4_RECW;
                const double v0 = x[0], v1 = x[1], al = x[2], zs = x[3], p = x[4];
                for (int sl = 0; sl < 2; ++sl) {
                    const double gg = sl ? gv1 : gv0;
                    const int64_t k = sl ? k1 : k0;
                    const double u = fma(-v1, pick(w1, r, sl), fma(-v0, pick(w0, r, sl), gg));
                    const double d = fma(-al, u * u, pick(dq, r, sl));
                    const double z = fma(-zs, u, pick(zq, r, sl));
                    const int32_t tup[4] = {(int32_t)(S4_NR * hh + r), (int32_t)i2, (int32_t)j, (int32_t)k};
                    const double es = (d > RANK_EPS) ? p - z * z / d : INF;
                    bool take = ((fm[sl] >> lane) & 1ull) && k < S && k > j && es <= fmin(theta_f, Ls[KP - 1]);
                    if (take && a.ranged) {
                        const uint64_t lr = lex_rank(BinomTab{c.btab, c.S}, c.S, 4, tup);
                        if (lr < a.r0 || lr >= a.r1) take = false;
                    }
                    unsigned long long m = __ballot(take);
                    const uint64_t rk = take ? pack_tuple(tup, 4) : 0;
                    offered += (unsigned)__popcll(m);
                    while (m) {
                        const int src = __ffsll((long long)m) - 1;
                        m &= m - 1;
                        const double cs = __shfl(es, src);
                        const uint64_t cr = (uint64_t)__shfl((long long)rk, src);
                        list_insert(Ls, Lr, KP, cs, cr);
                    }
                }
            }
        }
        const double tw = Ls[KP - 1];
        if (tw < theta_pub) {
            theta_pub = tw;
            if (lane == 0) theta_publish(c.theta_bits, tw);
        }
        }
    }
    if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// Several tasks, D = 3: exclusive prefix of the queued chunks' counts (one
// workgroup of PRE_WG threads, PRE_WG consecutive counts per pass).
__global__ __launch_bounds__(PRE_WG) void mt_scan_kernel(Ctx c, int nown) {
    __shared__ unsigned wsum[PRE_WG / 64];
    __shared__ unsigned long long carry;
    const int nreg = (int)min(*c.mtq_taken + (unsigned)nown, (unsigned)c.mtq_chunks);
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nreg; base += PRE_WG) {
        const int r = base + (int)threadIdx.x;
        const unsigned v = r < nreg ? c.mtq_n[r] : 0u;
        const unsigned incl = block_scan(v, wsum);
        const unsigned long long cy = carry;
        if (r < nreg) c.mtq_pre[r] = cy + incl - v;
        __syncthreads();
        if (threadIdx.x == PRE_WG - 1) carry = cy + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) c.mtq_pre[nreg] = carry;
}

// Several tasks, D = 3: scores the queued sweep steps.  The steps, in chunk
// order, are cut into equal contiguous runs, one per wave.  For each step the
// wave scores the steps with mt_step and mt_flush.  Wave gw starts from the
// sweep's list gw.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S3_WPE))) void mt_eval_kernel(
    Ctx c, SearchArgs a, const double *__restrict__ rec, int nown) {
    extern __shared__ double smem[];
    const int KP = a.KP;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    const int64_t nw = (int64_t)gridDim.x * SEARCH_WAVES;
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    list_load(Ls, Lr, c.list_sse + gw * KP, c.list_rank + gw * KP, KP);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    const int nreg = (int)min(*c.mtq_taken + (unsigned)nown, (unsigned)c.mtq_chunks);
    const uint64_t total = nreg > 0 ? c.mtq_pre[nreg] : 0;
    const uint64_t per = (total + nw - 1) / nw;
    const uint64_t e0 = (uint64_t)gw * per, e1 = e0 + per < total ? e0 + per : total;
    double th = fmin(theta0_from_prepass(c, a.L, KP), theta_load(c.theta_bits));
    const double theta_f = th < INF ? th * (1.0 + THETA_SLACK) : INF;
    __shared__ uint64_t s_bk[SEARCH_WAVES][MT_BUF];
    __shared__ double s_be[SEARCH_WAVES][MT_BUF];
    uint64_t *bk = s_bk[wave];
    double *be = s_be[wave];
    int nbuf = 0;
    unsigned offered = 0;
    if (e0 < e1) {
        int lo = 0, hi = nreg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (c.mtq_pre[mid] <= e0) lo = mid; else hi = mid - 1;
        }
        int reg = lo;
        for (uint64_t e = e0; e < e1; ++e) {
            while (reg + 1 <= nreg - 1 && c.mtq_pre[reg + 1] <= e) ++reg;
            const int64_t at = ((int64_t)reg * MTQ_CHUNK + (int64_t)(e - c.mtq_pre[reg])) * 3;
            const uint64_t w0 = c.mtq[at];
            offered += mt_step(c, a, rec, Ls, Lr, KP, bk, be, nbuf, (int64_t)(w0 >> 40),
                               (int64_t)((w0 >> 20) & 0xFFFFF), (int64_t)(w0 & 0xFFFFF), c.mtq[at + 1],
                               c.mtq[at + 2], theta_f);
        }
        if (nbuf > 0) offered += mt_flush(c, Ls, Lr, KP, bk, be, nbuf, theta_f);
    }
    if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// D = 1: every feature is a tuple; SSE = sum_t (c_t - b_t^2) over full-rank columns.
__global__ __launch_bounds__(256) void search_d1_kernel(Ctx c, SearchArgs a) {
    extern __shared__ double smem[];
    const int KP = a.KP;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    for (int m = lane; m < KP; m += 64) {
        Ls[m] = INF;
        Lr[m] = ~0ull;
    }
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    const int64_t nw = (int64_t)gridDim.x * SEARCH_WAVES;
    for (int64_t kb = gw * 64; kb < c.S; kb += nw * 64) {
        const int64_t k = kb + lane;
        double s = INF;
        if (k < c.S) {
            s = 0.0;
            for (int t = 0; t < c.T; ++t) {
                if (!(Gat(c, k, k, t) == 1.0)) {
                    s = INF;
                    break;
                }
                const double b = c.bhat[k * c.TP + t];
                s += c.cyy[t] - b * b;
            }
            if (a.ranged && ((uint64_t)k < a.r0 || (uint64_t)k >= a.r1)) s = INF;
        }
        unsigned long long m = __ballot(s < INF && s <= Ls[KP - 1]);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            list_insert(Ls, Lr, KP, __shfl(s, src), (uint64_t)(kb + src));
        }
    }
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// ------------------------------------------------- prefix-list evaluation
// Exact evaluation driven by a list of (D-1)-prefixes: every tuple P + {k}
// (k not in P) is scored by ne_sse on its sorted indices, so a tuple reached
// from several prefixes of the list gets bitwise the same SSE and key.

// Sorted tuple P + {k} (P sorted, k not in P); returns false if k is in P.
template <int M>
__device__ inline bool extend_sorted(const int32_t *P, int32_t k, int32_t *tup) {
    int n = 0;
    bool placed = false, dup = false;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        dup |= P[m] == k;
        if (!placed && k < P[m]) {
            tup[n++] = k;
            placed = true;
        }
        tup[n++] = P[m];
    }
    if (!placed) tup[n] = k;
    return !dup;
}

// Reads prefix p (M indices) and checks it: strictly increasing, in [0, S).
template <int M>
__device__ inline bool load_prefix(const Ctx &c, const int32_t *pre, int64_t p, int32_t *P) {
    bool ok = true;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        P[m] = pre[p * M + m];
        ok &= P[m] >= 0 && P[m] < c.S && (m == 0 || P[m] > P[m - 1]);
    }
    return ok;
}

// best[p] = min over k not in P of SSE(P + {k}); +inf if no extension is
// full rank, NaN for a malformed prefix.  One wavefront per prefix.
template <int M>
__global__ __launch_bounds__(256) void prefix_best_kernel(Ctx c, const int32_t *__restrict__ pre, int64_t n,
                                                          double *__restrict__ best) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < n; p += nw) {
        int32_t P[M];
        const bool ok = load_prefix<M>(c, pre, p, P);
        double mn = INF;
        if (ok)
            for (int64_t k = lane; k < c.S; k += 64) {
                int32_t tup[M + 1];
                if (extend_sorted<M>(P, (int32_t)k, tup)) mn = fmin(mn, ne_sse_t<M + 1>(c, tup));
            }
        for (int o = 32; o >= 1; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
        if (lane == 0) best[p] = ok ? mn : __builtin_nan("");
    }
}

// Top-k candidates over the extensions of a prefix list: persistent waves
// take prefixes in turn, lanes run over k, and each wave keeps its sorted
// list as in the exhaustive search (bound: own KP-th entry and the
// device-wide bound).  The lists feed the same merge, re-score and final
// ordering (merge removes tuples that several prefixes produced).
template <int M>
__global__ __launch_bounds__(256) void list_search_kernel(Ctx c, const int32_t *__restrict__ pre, int64_t n) {
    extern __shared__ double smem[];
    const int KP = c.KP;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *Ls = smem + (size_t)wave * KP * 2;
    uint64_t *Lr = reinterpret_cast<uint64_t *>(Ls + KP);
    for (int m = lane; m < KP; m += 64) {
        Ls[m] = INF;
        Lr[m] = ~0ull;
    }
    double theta_pub = INF;
    int fill = 0;  // entries appended while the list is filling (sorted once full)
    unsigned offered = 0;  // tuples offered to the list (diagnostics; one atomic per wave)
    const int64_t gw = (int64_t)blockIdx.x * SEARCH_WAVES + wave;
    const int64_t nw = (int64_t)gridDim.x * SEARCH_WAVES;
    for (int64_t p = gw; p < n; p += nw) {
        int32_t P[M];
        if (!load_prefix<M>(c, pre, p, P)) continue;
        // one task: the prefix's own factor (uniform) turns each extension
        // into an incremental filter (w = L^-1 G[P,k], d = G[k,k] - |w|^2,
        // SSE ~ p - zeta^2 / d); only extensions that pass it (or whose pivot
        // is too small to judge) are scored canonically
        double L[M][M], z[M], pp = 0.0;
        double gP[M][M], bP[M];  // the prefix's own correlation block and b (one task)
        bool pok = false;
        if (c.T == 1) {
            pp = c.cyy[0];
            pok = true;
#pragma unroll
            for (int a = 0; a < M; ++a) {
                bP[a] = c.bhat[(int64_t)P[a] * c.TP];
#pragma unroll
                for (int b2 = 0; b2 <= a; ++b2) gP[a][b2] = Gat(c, P[a], P[b2], 0);
            }
#pragma unroll
            for (int a = 0; a < M; ++a) {
#pragma unroll
                for (int b2 = 0; b2 < a; ++b2) {
                    double v = gP[a][b2];
#pragma unroll
                    for (int l = 0; l < b2; ++l) v -= L[a][l] * L[b2][l];
                    L[a][b2] = v / L[b2][b2];
                }
                double d = gP[a][a];
#pragma unroll
                for (int l = 0; l < a; ++l) d -= L[a][l] * L[a][l];
                pok &= d > RANK_EPS;
                L[a][a] = sqrt(fmax(d, RANK_EPS));
                double zz = bP[a];
#pragma unroll
                for (int l = 0; l < a; ++l) zz -= L[a][l] * z[l];
                z[a] = zz / L[a][a];
                pp -= z[a] * z[a];
            }
        }
        // the device-wide bound is read once per prefix (a memory round trip)
        const double th_dev = theta_load(c.theta_bits);
        for (int64_t kb = 0; kb < c.S; kb += 64) {
            const int64_t k = kb + lane;
            double sse = INF;
            uint64_t key = ~0ull;
            int32_t tup[M + 1];
            const double th = fmin(Ls[KP - 1], th_dev);
            bool score = k < c.S && extend_sorted<M>(P, (int32_t)k, tup);
            if (score && c.T == 1) {
                const int64_t kc = k;
                double gk[M];
#pragma unroll
                for (int a = 0; a < M; ++a) gk[a] = Gat(c, P[a], kc, 0);
                const double gkk = Gat(c, kc, kc, 0), bk = c.bhat[kc * c.TP];
                if (pok) {
                    double w[M], ww = 0.0, wz = 0.0;
#pragma unroll
                    for (int a = 0; a < M; ++a) {
                        double v = gk[a];
#pragma unroll
                        for (int l = 0; l < a; ++l) v -= L[a][l] * w[l];
                        w[a] = v / L[a][a];
                        ww += w[a] * w[a];
                        wz += w[a] * z[a];
                    }
                    const double d = gkk - ww;
                    const double zeta = bk - wz;
                    const double inc = d > 1e3 * RANK_EPS ? pp - zeta * zeta / d : -INF;
                    score = inc <= (th < INF ? th * (1.0 + 1e-8) + 1e-12 * c.cyy[0] : INF);
                }
                // (a tiny pivot in the prefix's own order says nothing certain about
                // the tuple's sorted order: such extensions are scored canonically)
                if (score) {
                    // canonical: the tuple's block in sorted-index order, from the
                    // values already loaded (G is bitwise symmetric)
                    int pos = 0;
#pragma unroll
                    for (int a = 0; a < M; ++a) pos += P[a] < kc;
                    // pos differs across lanes: the prefix values are picked by
                    // selects over constant indexes, so gP, bP and gk stay in
                    // registers (an indexed read would put them in scratch memory)
                    // (each candidate passes through an empty asm, so the
                    // compiler cannot fold the selects back into an indexed load)
                    auto opaque = [](double x) {
                        __asm__ volatile("" : "+v"(x));
                        return x;
                    };
                    auto pick1 = [&](const double (&arr)[M], int a) {
                        double r = opaque(arr[0]);
#pragma unroll
                        for (int q = 1; q < M; ++q) r = a == q ? opaque(arr[q]) : r;
                        return r;
                    };
                    auto pickg = [&](int a, int b) {  // b <= a (lower triangle)
                        double r = opaque(gP[0][0]);
#pragma unroll
                        for (int q = 1; q < M; ++q)
#pragma unroll
                            for (int q2 = 0; q2 <= q; ++q2) r = (a == q && b == q2) ? opaque(gP[q][q2]) : r;
                        return r;
                    };
                    double g4[M + 1][M + 1], b4[M + 1];
#pragma unroll
                    for (int u = 0; u <= M; ++u) {
                        const int au = u < pos ? u : u - 1;  // prefix slot of tuple slot u (u != pos)
                        b4[u] = u == pos ? bk : pick1(bP, au);
#pragma unroll
                        for (int v2 = 0; v2 <= u; ++v2) {
                            const int av = v2 < pos ? v2 : v2 - 1;
                            double val;
                            if (u == pos && v2 == pos) val = gkk;
                            else if (u == pos) val = pick1(gk, av);
                            else if (v2 == pos) val = pick1(gk, au);
                            else val = pickg(au, av);
                            g4[u][v2] = val;
                        }
                    }
                    bool ok = true;
                    const double v = ne_sse_core<M + 1>(g4, b4, c.cyy[0], ok);
                    sse = ok ? v : INF;
                    key = pack_tuple(tup, M + 1);
                }
            } else if (score) {
                sse = ne_sse_t<M + 1>(c, tup);
                key = pack_tuple(tup, M + 1);
            }
            unsigned long long m = __ballot(sse < INF && sse <= th);
            offered += (unsigned)__popcll(m);
            if (fill < KP && m) {
                // the list is not full: append (one slot per passing lane), and
                // sort once it is
                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                const int nfit = min(__popcll(m), KP - fill);
                const bool mine = ((m >> lane) & 1ull) && rank < nfit;
                if (mine) {
                    Ls[fill + rank] = sse;
                    Lr[fill + rank] = key;
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_wave_barrier();
                m &= ~__ballot(mine);
                fill += nfit;
                if (fill == KP) wave_sort_list(Ls, Lr, KP);
            }
            while (m) {
                const int src = __ffsll((long long)m) - 1;
                m &= m - 1;
                list_insert(Ls, Lr, KP, __shfl(sse, src), (uint64_t)__shfl((long long)key, src));
            }
            const double tw = Ls[KP - 1];
            if (tw < theta_pub) {
                theta_pub = tw;
                if (lane == 0) theta_publish(c.theta_bits, tw);
            }
        }
    }
    if (fill < KP) wave_sort_list(Ls, Lr, KP);  // unused slots hold +inf and sort last
    if (lane == 0 && offered) atomicAdd(c.cand_counter, offered);
    list_store(c.list_sse + gw * KP, c.list_rank + gw * KP, Ls, Lr, KP);
}

// Per-prefix features for the learned proposal (FP32, PROP_NF per prefix),
// dimension-agnostic so that a model trained on one prefix length applies
// to another: with r_i^2 = b_i^2 / c (squared correlation with y) and the
// prefix's own fit R^2 = 1 - SSE(P) / c (sums over tasks):
//   R^2, max r_i^2, min r_i^2, mean r_i^2, max |G_ij|, mean |G_ij|,
//   R^2 - max r_i^2 (gain over the best single feature), 1 / M.
// One thread per prefix.
template <int M>
__device__ void prefix_features(const Ctx &c, const int32_t *P, float *o) {
    double ctot = 0.0;
    for (int t = 0; t < c.T; ++t) ctot += c.cyy[t];
    const double ic = ctot > 0.0 ? 1.0 / ctot : 0.0;
    double r2max = 0.0, r2min = INF, r2sum = 0.0, gmax = 0.0, gsum = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double e = 0.0;
        for (int t = 0; t < c.T; ++t) {
            const double b = c.bhat[(int64_t)P[m] * c.TP + t];
            e += b * b;
        }
        e *= ic;
        r2max = fmax(r2max, e);
        r2min = fmin(r2min, e);
        r2sum += e;
#pragma unroll
        for (int l = 0; l < m; ++l) {
            double g = 0.0;
            for (int t = 0; t < c.T; ++t) g = fmax(g, fabs(Gat(c, P[m], P[l], t)));
            gmax = fmax(gmax, g);
            gsum += g;
        }
    }
    const double sse = ne_sse_t<M>(c, P);
    const double R2 = sse < INF ? 1.0 - sse * ic : 0.0;
    o[0] = (float)R2;
    o[1] = (float)r2max;
    o[2] = (float)r2min;
    o[3] = (float)(r2sum / M);
    o[4] = (float)gmax;
    o[5] = (float)(M > 1 ? gsum / (M * (M - 1) / 2) : 0.0);
    o[6] = (float)(R2 - r2max);
    o[7] = (float)(1.0 / M);
}

// Features of the prefixes of a list (one thread each).
template <int M>
__global__ __launch_bounds__(256) void prefix_features_kernel(Ctx c, const int32_t *__restrict__ pre, int64_t n,
                                                              float *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t P[M];
    float *o = out + p * PROP_NF;
    if (!load_prefix<M>(c, pre, p, P)) {
        for (int f = 0; f < PROP_NF; ++f) o[f] = __builtin_nanf("");
        return;
    }
    prefix_features<M>(c, P, o);
}

// Features of the M-subsets of {0..S-1} with colexicographic ranks
// r0 .. r0 + n - 1 (no prefix array needed for a full sweep).
template <int M>
__global__ __launch_bounds__(256) void prefix_features_range_kernel(Ctx c, uint64_t r0, int64_t n,
                                                                    float *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t P[M];
    colex_unrank_small(r0 + (uint64_t)p, M, c.S, P);
    prefix_features<M>(c, P, out + p * PROP_NF);
}

// ----------------------------------------------------------------- merge
// One workgroup: gather every list entry at or below the final bound, then
// select the KP smallest (SSE, rank) keys with bitonic sorts in LDS, a
// running top-KP carried across chunks when there are many.
constexpr int MERGE_THREADS = 1024;
constexpr int MERGE_CAP = 2048;

__device__ void bitonic_sort_lds(double *ks, uint64_t *kr, int N) {
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const double a = ks[i], b = ks[ixj];
                    const uint64_t ra = kr[i], rb = kr[ixj];
                    const bool gt = key_less(b, rb, a, ra);
                    if (gt == up) {
                        ks[i] = b;
                        ks[ixj] = a;
                        kr[i] = rb;
                        kr[ixj] = ra;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// merge_compact: one wave per list.  Lists are sorted ascending, so the
// entries at or below the bound are a prefix; its length is a ballot count
// and the prefix is appended to the candidate array at an atomically
// reserved offset.  The candidate set does not depend on the append order,
// and keys are unique, so the selection below is deterministic.
__device__ inline double merge_bound(const Ctx &c, int L, int KP, int use_pre) {
    double bound = theta_load(c.theta_bits);
    if (use_pre) bound = fmin(bound, theta0_from_prepass(c, L, KP));
    return bound < INF ? bound * (1.0 + THETA_SLACK) : INF;
}

// nl_dev (may be null): the number of lists written, read on the device (at
// most nlists; the batched search writes a variable number per problem)
__global__ __launch_bounds__(MERGE_THREADS) void merge_compact_kernel(Ctx c, int nlists, int KP, int L,
                                                                      int use_pre, const uint32_t *nl_dev) {
    const int lane = threadIdx.x & 63;
    const int64_t l = (int64_t)blockIdx.x * (MERGE_THREADS / 64) + (threadIdx.x >> 6);
    const int64_t nl = nl_dev ? (int64_t)min(*nl_dev, (uint32_t)nlists) : (int64_t)nlists;
    if (l >= nl) return;
    const double bound = merge_bound(c, L, KP, use_pre);
    const double *ls = c.list_sse + l * KP;
    const uint64_t *lr = c.list_rank + l * KP;
    // sorted: the entries at or below the bound are a prefix, which ends at
    // the list's terminator at the latest
    int n = 0;
    for (int m = 0; m < KP; m += 64) {
        const double v = ls[m + lane];
        const unsigned long long b = __ballot(v < INF && v <= bound);
        if (b != ~0ull) {
            n += __builtin_ctzll(~b);  // the prefix before the first entry that fails
            break;
        }
        n += 64;
    }
    if (n == 0) return;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(c.merge_count, (unsigned)n);
    base = __shfl(base, 0);
    for (int e = lane; e < n; e += 64) {
        c.cand_sse[base + e] = ls[e];
        c.cand_rank[base + e] = lr[e];
    }
}

// merge_select: one workgroup selects the KP smallest (SSE, key) pairs of
// the candidates with bitonic sorts in LDS, carrying a running top-KP across
// fills of the buffer when there are many.
// Marks the later copy of every adjacent equal (SSE, key) pair as empty and
// re-sorts (a prefix-list search can offer one tuple from several prefixes,
// always with bitwise the same SSE, so copies are adjacent after a sort).
__device__ void drop_adjacent_duplicates(double *ks, uint64_t *kr, int N) {
    bool dup[MERGE_CAP / MERGE_THREADS];
    int nd = 0;
    for (int i = threadIdx.x, u = 0; i < N; i += MERGE_THREADS, ++u) {
        dup[u] = i > 0 && ks[i] < INF && ks[i] == ks[i - 1] && kr[i] == kr[i - 1];
        nd += dup[u];
    }
    __syncthreads();
    for (int i = threadIdx.x, u = 0; i < N; i += MERGE_THREADS, ++u)
        if (dup[u]) {
            ks[i] = INF;
            kr[i] = ~0ull;
        }
    if (__syncthreads_or(nd)) bitonic_sort_lds(ks, kr, N);
}

__global__ __launch_bounds__(MERGE_THREADS) void merge_select_kernel(Ctx c, int KP, int L, int use_pre, int dedupe,
                                                                     int nlists, const uint32_t *nl_dev) {
    __shared__ double ks[MERGE_CAP];
    __shared__ uint64_t kr[MERGE_CAP];
    __shared__ int fill;
    const int tid = threadIdx.x;
    const int64_t total = *c.merge_count;
    if (tid == 0) {
        const double th0 = use_pre ? theta0_from_prepass(c, L, KP) : INF;
        c.stats[0] = *c.cand_counter;
        c.stats[2] = (uint64_t)__double_as_longlong(th0);
        c.stats[3] = (uint64_t)__double_as_longlong(theta_load(c.theta_bits));
    }
    // Few candidates (the usual case once the pre-pass bound is tight): the
    // KP smallest by rank counting, with no sort.  Without dedupe the keys are
    // distinct, so the ranks (candidates ordered before each one) are too,
    // and writing candidate x at position rank(x) < KP gives the sorted
    // prefix the sorting path below returns (the candidates are finite:
    // merge_compact appends only entries below INF); positions past the
    // candidates are empty (INF, ~0) as there.
    if (!dedupe && total <= MERGE_THREADS) {
        const int n = (int)total;
        if (tid < n) {
            ks[tid] = c.cand_sse[tid];
            kr[tid] = c.cand_rank[tid];
        }
        __syncthreads();
        if (tid < n) {
            const double v = ks[tid];
            const uint64_t r = kr[tid];
            // (SSE, key) order written without short-circuit evaluation, so
            // that the eight steps' LDS reads are all in flight together
            auto before = [&](int i) {
                const double a = ks[i];
                const uint64_t b = kr[i];
                return (int)((a < v) | ((a == v) & (b < r)));
            };
            int rank = 0, i = 0;
            for (; i + 8 <= n; i += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) rank += before(i + u);
            }
            for (; i < n; ++i) rank += before(i);
            if (rank < KP) {
                c.merged_sse[rank] = v;
                c.merged_rank[rank] = r;
            }
        }
        for (int i = n + tid; i < KP; i += MERGE_THREADS) {
            c.merged_sse[i] = INF;
            c.merged_rank[i] = ~0ull;
        }
        return;
    }
    auto clear_from = [&](int at) {
        for (int i = at + tid; i < MERGE_CAP; i += MERGE_THREADS) {
            ks[i] = INF;
            kr[i] = ~0ull;
        }
    };
    auto pow2_at_least = [&](int64_t need) {
        int N = 2 * KP;
        while (N < need) N <<= 1;
        return N;
    };
    clear_from(0);
    __syncthreads();
    const int chunk = MERGE_CAP - KP;
    // Many candidates: every list is sorted, so the KP-th smallest of the
    // lists' first entries bounds the KP-th smallest candidate (those KP
    // lists each hold an entry at or below it); only candidates at or below
    // that cut can be selected.  Not with dedupe: there one tuple can head
    // several lists, and KP first entries need not be KP tuples.
    double cut = INF;
    const int64_t nl = nl_dev ? (int64_t)min(*nl_dev, (uint32_t)nlists) : (int64_t)nlists;
    if (!dedupe && total > chunk && nl >= KP) {
        for (int64_t base = 0; base < nl; base += chunk) {
            const int64_t here = nl - base < chunk ? nl - base : chunk;
            const int N = pow2_at_least(KP + here);
            for (int i = tid; i < N - KP; i += MERGE_THREADS) {
                ks[KP + i] = i < here ? c.list_sse[(base + i) * KP] : INF;
                kr[KP + i] = 0;
            }
            __syncthreads();
            bitonic_sort_lds(ks, kr, N);
        }
        cut = ks[KP - 1];
        __syncthreads();
        clear_from(0);
        if (tid == 0) fill = 0;
        __syncthreads();
    } else if (tid == 0) {
        fill = 0;
    }
    __syncthreads();
    // the candidates at or below the cut are appended behind the KP kept in
    // front; the buffer is sorted (the KP smallest kept) before it could
    // overflow.  Append order does not matter: the sort is by (SSE, key).
    auto sort_keep = [&]() {
        const int N = pow2_at_least(KP + fill);
        bitonic_sort_lds(ks, kr, N);
        if (dedupe) drop_adjacent_duplicates(ks, kr, N);
        clear_from(KP);
        if (tid == 0) fill = 0;
        __syncthreads();
    };
    for (int64_t e = 0; e < total; e += MERGE_THREADS) {
        // sort only when this batch could overflow the buffer
        const int64_t batch = total - e < MERGE_THREADS ? total - e : MERGE_THREADS;
        if (fill + batch > chunk) sort_keep();
        const int64_t i = e + tid;
        if (i < total) {
            const double v = c.cand_sse[i];
            if (v <= cut) {
                const int at = atomicAdd(&fill, 1);
                ks[KP + at] = v;
                kr[KP + at] = c.cand_rank[i];
            }
        }
        __syncthreads();
    }
    sort_keep();
    for (int i = tid; i < KP; i += MERGE_THREADS) {
        c.merged_sse[i] = ks[i];
        c.merged_rank[i] = kr[i];
    }
}

// --------------------------------------------------------------- rescore
// One workgroup per candidate: for each task, the (D x D) normal equations
// of the centred columns are accumulated straight from F in a fixed order,
// solved by Cholesky (pivot-ratio rank test), and the SSE is taken as the
// squared norm of the explicit residual y_c - X_c beta.
template <int D>
__global__ __launch_bounds__(256) void rescore_kernel(Ctx c) {
    constexpr int NACC = D * (D + 1) / 2 + D;
    __shared__ double red[NACC][4];
    __shared__ double s_beta[D];
    __shared__ int s_ok;
    const int cand = blockIdx.x;
    const int tid = threadIdx.x;
    const int W = D + 1;
    double *coef = c.resc_coef + (int64_t)cand * c.T * (c.D_max + 1);
    if (!(c.merged_sse[cand] < INF)) {
        if (tid == 0) c.resc_sse[cand] = INF;
        for (int i = tid; i < c.T * (c.D_max + 1); i += 256) coef[i] = __builtin_nan("");
        return;
    }
    int32_t tup[MAXD];
    unpack_tuple(c.merged_rank[cand], D, tup);
    if (c.T > 1) {
        // several tasks: wave w takes tasks w, w + 4, ... on its own (wave
        // sums, the small solve repeated in every lane), then the four wave
        // totals are added in a fixed order
        __shared__ double wtot[4];
        __shared__ int wok[4];
        const int lane = tid & 63, wave = tid >> 6;
        double tw = 0.0;
        bool okw = true;
        for (int t = wave; t < c.T; t += 4) {
            const int64_t r0 = c.off_dev[t], r1 = c.off_dev[t + 1];
            const double ym = c.ybar[t];
            double mu[D];
#pragma unroll
            for (int m = 0; m < D; ++m) mu[m] = c.mu[(int64_t)t * c.S + tup[m]];
            double acc[NACC];
#pragma unroll
            for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
            for (int64_t i = r0 + lane; i < r1; i += 64) {
                double x[D];
#pragma unroll
                for (int m = 0; m < D; ++m) x[m] = c.F[(int64_t)tup[m] * c.n_total + i] - mu[m];
                const double yc = c.y[i] - ym;
                int e = 0;
#pragma unroll
                for (int m = 0; m < D; ++m)
#pragma unroll
                    for (int l = 0; l <= m; ++l) acc[e++] += x[m] * x[l];
#pragma unroll
                for (int m = 0; m < D; ++m) acc[e++] += x[m] * yc;
            }
#pragma unroll
            for (int i = 0; i < NACC; ++i)
                for (int o = 32; o > 0; o >>= 1) acc[i] += __shfl_xor(acc[i], o);
            double M[D][D], v[D], L[D][D], z[D], bt[D];
            int e = 0;
#pragma unroll
            for (int m = 0; m < D; ++m)
#pragma unroll
                for (int l = 0; l <= m; ++l) {
                    M[m][l] = acc[e];
                    M[l][m] = acc[e];
                    ++e;
                }
#pragma unroll
            for (int m = 0; m < D; ++m) v[m] = acc[e++];
            bool ok = true;
#pragma unroll
            for (int m = 0; m < D; ++m) {
#pragma unroll
                for (int jx = 0; jx < m; ++jx) {
                    double sm = M[m][jx];
#pragma unroll
                    for (int l = 0; l < jx; ++l) sm -= L[m][l] * L[jx][l];
                    L[m][jx] = sm / L[jx][jx];
                }
                double d = M[m][m];
#pragma unroll
                for (int l = 0; l < m; ++l) d -= L[m][l] * L[m][l];
                ok = ok && (M[m][m] > 0.0) && (d > RANK_EPS * M[m][m]);
                L[m][m] = ok ? sqrt(d) : 1.0;
            }
#pragma unroll
            for (int m = 0; m < D; ++m) {
                double sm = v[m];
#pragma unroll
                for (int l = 0; l < m; ++l) sm -= L[m][l] * z[l];
                z[m] = sm / L[m][m];
            }
#pragma unroll
            for (int m = D - 1; m >= 0; --m) {
                double sm = z[m];
#pragma unroll
                for (int l = m + 1; l < D; ++l) sm -= L[l][m] * bt[l];
                bt[m] = sm / L[m][m];
            }
            okw = okw && ok;
            double ss = 0.0;
            for (int64_t i = r0 + lane; i < r1; i += 64) {
                double er = c.y[i] - ym;
#pragma unroll
                for (int m = 0; m < D; ++m) er -= bt[m] * (c.F[(int64_t)tup[m] * c.n_total + i] - mu[m]);
                ss += er * er;
            }
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
            tw += ss;
            if (lane == 0) {
                double alpha = ym;
#pragma unroll
                for (int m = 0; m < D; ++m) alpha -= bt[m] * mu[m];
                coef[t * (c.D_max + 1)] = alpha;
#pragma unroll
                for (int m = 0; m < D; ++m) coef[t * (c.D_max + 1) + 1 + m] = bt[m];
            }
        }
        if (lane == 0) {
            wtot[wave] = tw;
            wok[wave] = okw ? 1 : 0;
        }
        __syncthreads();
        if (tid == 0) {
            const bool all = wok[0] && wok[1] && wok[2] && wok[3];
            c.resc_sse[cand] = all ? ((wtot[0] + wtot[1]) + wtot[2]) + wtot[3] : INF;
        }
        return;
    }
    double total = 0.0;
    bool valid = true;
    for (int t = 0; t < c.T; ++t) {
        const int64_t r0 = c.off_dev[t], r1 = c.off_dev[t + 1];
        const double ym = c.ybar[t];
        double mu[D];
        for (int m = 0; m < D; ++m) mu[m] = c.mu[(int64_t)t * c.S + tup[m]];
        double acc[NACC];
        for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
#pragma unroll 4
        for (int64_t i = r0 + tid; i < r1; i += 256) {
            double x[D];
            for (int m = 0; m < D; ++m) x[m] = c.F[(int64_t)tup[m] * c.n_total + i] - mu[m];
            const double yc = c.y[i] - ym;
            int e = 0;
            for (int m = 0; m < D; ++m)
                for (int l = 0; l <= m; ++l) acc[e++] += x[m] * x[l];
            for (int m = 0; m < D; ++m) acc[e++] += x[m] * yc;
        }
        constexpr int nacc = NACC;
        // wave butterflies, then the 4 wave sums in a fixed order
        for (int i = 0; i < nacc; ++i) {
            double v = acc[i];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if ((tid & 63) == 0) red[i][tid >> 6] = v;
        }
        __syncthreads();
        if (tid < nacc) red[tid][0] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
        __syncthreads();
        if (tid == 0) {
            // fully unrolled (D is fixed), so the small matrices stay in registers
            double M[D][D], v[D], L[D][D], z[D], bt[D];
            int e = 0;
#pragma unroll
            for (int m = 0; m < D; ++m)
#pragma unroll
                for (int l = 0; l <= m; ++l) {
                    M[m][l] = red[e][0];
                    M[l][m] = red[e][0];
                    ++e;
                }
#pragma unroll
            for (int m = 0; m < D; ++m) v[m] = red[e++][0];
            // Cholesky; once a pivot fails the rest is computed on a unit
            // pivot and discarded
            bool ok = true;
#pragma unroll
            for (int m = 0; m < D; ++m) {
#pragma unroll
                for (int jx = 0; jx < m; ++jx) {
                    double s = M[m][jx];
#pragma unroll
                    for (int l = 0; l < jx; ++l) s -= L[m][l] * L[jx][l];
                    L[m][jx] = s / L[jx][jx];
                }
                double d = M[m][m];
#pragma unroll
                for (int l = 0; l < m; ++l) d -= L[m][l] * L[m][l];
                ok = ok && (M[m][m] > 0.0) && (d > RANK_EPS * M[m][m]);
                L[m][m] = ok ? sqrt(d) : 1.0;
            }
            if (ok) {
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    double s = v[m];
#pragma unroll
                    for (int l = 0; l < m; ++l) s -= L[m][l] * z[l];
                    z[m] = s / L[m][m];
                }
#pragma unroll
                for (int m = D - 1; m >= 0; --m) {
                    double s = z[m];
#pragma unroll
                    for (int l = m + 1; l < D; ++l) s -= L[l][m] * bt[l];
                    bt[m] = s / L[m][m];
                }
#pragma unroll
                for (int m = 0; m < D; ++m) s_beta[m] = bt[m];
            }
            s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) {
            valid = false;
            __syncthreads();
            break;
        }
        double beta[D];
        for (int m = 0; m < D; ++m) beta[m] = s_beta[m];
        double ss = 0.0;
#pragma unroll 4
        for (int64_t i = r0 + tid; i < r1; i += 256) {
            double e = c.y[i] - ym;
            for (int m = 0; m < D; ++m) e -= beta[m] * (c.F[(int64_t)tup[m] * c.n_total + i] - mu[m]);
            ss += e * e;
        }
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
        if ((tid & 63) == 0) red[0][tid >> 6] = ss;
        __syncthreads();
        if (tid == 0) {
            total += ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
            double alpha = ym;
            for (int m = 0; m < D; ++m) alpha -= beta[m] * mu[m];
            coef[t * (c.D_max + 1)] = alpha;
            for (int m = 0; m < D; ++m) coef[t * (c.D_max + 1) + 1 + m] = beta[m];
        }
        __syncthreads();
    }
    if (tid == 0) c.resc_sse[cand] = valid ? total : INF;
    (void)W;
}

// ----------------------------------------------------------------- final
// Order the re-scored candidates by (SSE, rank) (rank by counting; invalid
// ones last in candidate order) and write the k best.  The KP keys are staged
// in LDS once, so each thread's count runs over LDS.
template <int D>
__global__ __launch_bounds__(1024) void final_kernel(Ctx c, int k, int KP) {
    // status words travel with the results (one readout transfer)
    if (threadIdx.x < 4) c.res_flags[threadIdx.x] = c.flags[threadIdx.x];
    __shared__ double fs[KP_MAX];
    __shared__ uint64_t fr[KP_MAX];
    __shared__ double ferr[1024 / 64];
    for (int i = threadIdx.x; i < KP; i += blockDim.x) {
        const double si = c.resc_sse[i];
        fs[i] = si < INF ? si : INF;
        fr[i] = c.merged_rank[i];
    }
    __syncthreads();
    double err = 0.0;  // largest relative gap between the ranked and the exact SSE of a result
    // rank by counting: FIN_SPLIT neighbouring lanes share one candidate and
    // count over interleaved slices of the others (short LDS chains), then
    // add their counts with shuffles
    constexpr int FIN_SPLIT = 8;
    for (int i0 = 0; i0 < KP; i0 += 1024 / FIN_SPLIT) {
        const int i = i0 + (int)(threadIdx.x / FIN_SPLIT);
        const int part = (int)(threadIdx.x % FIN_SPLIT);
        const bool have = i < KP;
        const double si = have ? fs[i] : INF;
        const uint64_t ri = have ? fr[i] : 0;
        const bool vi = si < INF;
        int pos = 0;
        if (have) {
#pragma unroll 4
            for (int j = part; j < KP; j += FIN_SPLIT) {
                const double sj = fs[j];
                const bool vj = sj < INF;
                bool before;
                if (vi && vj) before = key_less(sj, fr[j], si, ri);
                else if (vj) before = true;
                else if (vi) before = false;
                else before = j < i;
                pos += before;
            }
        }
        for (int o = 1; o < FIN_SPLIT; o <<= 1) pos += __shfl_xor(pos, o);
        if (have && part == 0 && pos < k) {
            if (vi) {
                const double a = c.merged_sse[i];
                err = fmax(err, si > 0.0 ? fabs(a - si) / si : fabs(a - si));
            }
            c.res_sse[pos] = vi ? si : INF;
            int32_t tup[MAXD];
            if (vi) unpack_tuple(ri, D, tup);
            for (int m = 0; m < D; ++m) c.res_idx[pos * D + m] = vi ? tup[m] : -1;
            for (int t = 0; t < c.T; ++t)
                for (int m = 0; m <= D; ++m)
                    c.res_coef[((int64_t)pos * c.T + t) * (D + 1) + m] =
                        vi ? c.resc_coef[((int64_t)i * c.T + t) * (c.D_max + 1) + m] : __builtin_nan("");
        }
    }
    for (int o = 32; o >= 1; o >>= 1) err = fmax(err, __shfl_xor(err, o));
    if ((threadIdx.x & 63) == 0) ferr[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) e = fmax(e, ferr[w]);
        c.err_bits[1] = (unsigned long long)__double_as_longlong(e);
    }
}

// -------------------------------------------------------------- launcher
// the small per-search kernels are compiled per D (short code, no runtime
// dimension loops)
static void launch_rescore_final(const Ctx &c, int D, int k, hipStream_t st) {
    phase_begin(c, SISSO_PHASE_RESCORE, st);
    switch (D) {
        case 1: hipLaunchKernelGGL((rescore_kernel<1>), dim3(c.KP), dim3(256), 0, st, c); break;
        case 2: hipLaunchKernelGGL((rescore_kernel<2>), dim3(c.KP), dim3(256), 0, st, c); break;
        case 3: hipLaunchKernelGGL((rescore_kernel<3>), dim3(c.KP), dim3(256), 0, st, c); break;
        default: hipLaunchKernelGGL((rescore_kernel<4>), dim3(c.KP), dim3(256), 0, st, c); break;
    }
    phase_end(c, SISSO_PHASE_RESCORE, st);
    phase_begin(c, SISSO_PHASE_FINAL, st);
    switch (D) {
        case 1: hipLaunchKernelGGL((final_kernel<1>), dim3(1), dim3(1024), 0, st, c, k, c.KP); break;
        case 2: hipLaunchKernelGGL((final_kernel<2>), dim3(1), dim3(1024), 0, st, c, k, c.KP); break;
        case 3: hipLaunchKernelGGL((final_kernel<3>), dim3(1), dim3(1024), 0, st, c, k, c.KP); break;
        default: hipLaunchKernelGGL((final_kernel<4>), dim3(1), dim3(1024), 0, st, c, k, c.KP); break;
    }
    phase_end(c, SISSO_PHASE_FINAL, st);
}

template <int D>
static void launch_prepass(const Ctx &c, const SearchCall &sc, int L, hipStream_t st, bool select = true) {
    if (select) hipLaunchKernelGGL((pre_select_kernel<D>), dim3(1), dim3(PRE_WG), 0, st, c);
    hipLaunchKernelGGL((pre_extend_kernel<D>), dim3(PRE_Q), dim3(PRE_WG), 0, st, c, sc.ranged, sc.r0, sc.r1, L);
}

template <int D, bool MT>
static void launch_one(const Ctx &c, const SearchArgs &a, size_t lds, hipStream_t st) {
    if (c.fp32)
        hipLaunchKernelGGL((search_kernel<D, MT, float>), dim3(c.search_wgs), dim3(SEARCH_WG), lds, st, c, a);
    else
        hipLaunchKernelGGL((search_kernel<D, MT, double>), dim3(c.search_wgs), dim3(SEARCH_WG), lds, st, c, a);
}

static void launch_merge(const Ctx &c, int nlists, int L, int use_pre, hipStream_t st, int dedupe = 0,
                         const uint32_t *nl_dev = nullptr) {
    const int per = MERGE_THREADS / 64;
    hipLaunchKernelGGL(merge_compact_kernel, dim3((nlists + per - 1) / per), dim3(MERGE_THREADS), 0, st, c, nlists,
                       c.KP, L, use_pre, nl_dev);
    hipLaunchKernelGGL(merge_select_kernel, dim3(1), dim3(MERGE_THREADS), 0, st, c, c.KP, L, use_pre, dedupe, nlists,
                       nl_dev);
}

// The one-task D = 3 record-table path applies (it also needs the table in
// the workspace and fewer than 2^31 tiles).
bool s3_batchable(const Ctx &c, int D) {
    return D == 3 && c.T == 1 && !c.fp32 && c.rec3 != nullptr && s3_tiles_host(c.S) < (1ull << 31);
}

// record table + initialisation + pre-pass selection (one launch), then the
// pre-pass extension: everything before the sweep of the one-task D = 3 path
static void s3_prologue(const Ctx &c, const SearchCall &sc, int L, hipStream_t st) {
    const unsigned init_blocks = (unsigned)(((SISSO_MAX_D + 1) * (c.S + 1) + 255) / 256);
    const int64_t ngr = (c.S - 3) / S3_NR + 1;
    int64_t bx = ((c.S - 2) * S3_NR + PRE_WG - 1) / PRE_WG;
    const int64_t ninit = (int64_t)init_blocks * 256;
    if (bx * PRE_WG * ngr < ninit) bx = (ninit / ngr + PRE_WG - 1) / PRE_WG + 1;
    // one more column: its first workgroup runs the pre-pass selection
    hipLaunchKernelGGL(rec3_kernel, dim3((unsigned)(bx + 1), (unsigned)ngr), dim3(PRE_WG), 0, st, c, c.rec3);
    launch_prepass<3>(c, sc, L, st, false);
}

int launch_batch_prologue(const Ctx &c, const SearchCall &sc, hipStream_t st) {
    s3_prologue(c, sc, (c.KP + PRE_Q - 1) / PRE_Q, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_search3(const BatchSearchArgs &b, int wgs, hipStream_t st) {
    // one resident round: S3B_WPE waves on each of the 4 SIMDs of 256 CUs
    if (wgs <= 0 || wgs > S3B_WPE * 256) wgs = S3B_WPE * 256;
    const size_t lds = (size_t)SEARCH_WAVES * b.KPmax * 2 * sizeof(double);
    hipLaunchKernelGGL(search3_batch_kernel, dim3((unsigned)wgs), dim3(SEARCH_WG), lds, st, b);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_epilogue(const Ctx &c, const SearchCall &sc, hipStream_t st) {
    launch_merge(c, c.nwaves, (c.KP + PRE_Q - 1) / PRE_Q, 1, st, 0, c.flags + FLAG_NLISTS);
    launch_rescore_final(c, 3, sc.k, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_search(const Ctx &c, const SearchCall &sc, hipStream_t st) {
    const int D = sc.D;
    const bool MT = c.T > 1;
    SearchArgs a{};
    a.D = D;
    a.KP = c.KP;
    a.ranged = sc.ranged;
    a.r0 = sc.r0;
    a.r1 = sc.r1;
    a.TL = MT ? c.TP : 1;
    // many tasks: JB * TP <= MT_RECS records of the item in LDS (JB <= 64)
    a.JB = MT ? (64 < MT_RECS / c.TP ? 64 : MT_RECS / c.TP) : JBLK;
    a.R = MT ? 1 : SUBP;
    a.L = (c.KP + PRE_Q - 1) / PRE_Q;
    const int q = D - 2;
    const int RECW = q + 4;
    const int QA = q > 0 ? q : 1;
    const int SUBW = QA * QA + QA + 2;
    const size_t lds_lists = (size_t)SEARCH_WAVES * c.KP * 2 * sizeof(double);
    const unsigned init_blocks = (unsigned)(((SISSO_MAX_D + 1) * (c.S + 1) + 255) / 256);

    if (D == 1) {
        int wgs = (int)((c.S + SEARCH_WG - 1) / SEARCH_WG);
        if (wgs > c.search_wgs) wgs = c.search_wgs;
        phase_begin(c, SISSO_PHASE_PREPASS, st);
        hipLaunchKernelGGL(search_init_kernel, dim3(init_blocks), dim3(256), 0, st, c, 2, 1, JBLK, 0);
        phase_end(c, SISSO_PHASE_PREPASS, st);
        phase_begin(c, SISSO_PHASE_SEARCH, st);
        hipLaunchKernelGGL(search_d1_kernel, dim3(wgs), dim3(SEARCH_WG), lds_lists, st, c, a);
        phase_end(c, SISSO_PHASE_SEARCH, st);
        phase_begin(c, SISSO_PHASE_MERGE, st);
        launch_merge(c, wgs * SEARCH_WAVES, a.L, 0, st);
        phase_end(c, SISSO_PHASE_MERGE, st);
    } else {
        phase_begin(c, SISSO_PHASE_PREPASS, st);
        // one task, D = 3: record table + tile sweep (tile count within the 32-bit work counter)
        // D = 3: the record-table sweep, on the filter task's matrix when
        // there are several tasks
        const bool s3 = D == 3 && !c.fp32 && c.rec3 != nullptr && s3_tiles_host(c.S) < (1ull << 31) &&
                        (!MT || c.mtq_chunks > 0);
        // one task, D = 4: the pair-group record table (sized at create only
        // while it stays within S4_TABLE_MAX and 2^31 tiles)
        const bool s4 = D == 4 && !MT && !c.fp32 && c.rec4 != nullptr;
        if (s4) {
            hipLaunchKernelGGL(s4_init_kernel, dim3(init_blocks), dim3(256), 0, st, c);
        } else if (s3) {
            // record table + initialisation in one launch (its grid covers the binomial table)
            // x: the rows of one group (j, r); y: groups; the grid also covers
            // the binomial table of the initialisation
            const int64_t ngr = (c.S - 3) / S3_NR + 1;
            int64_t bx = ((c.S - 2) * S3_NR + PRE_WG - 1) / PRE_WG;
            const int64_t ninit = (int64_t)init_blocks * 256;
            if (bx * PRE_WG * ngr < ninit) bx = (ninit / ngr + PRE_WG - 1) / PRE_WG + 1;
            // one more column: its first workgroup runs the pre-pass selection
            hipLaunchKernelGGL(rec3_kernel, dim3((unsigned)(bx + 1), (unsigned)ngr), dim3(PRE_WG), 0, st, c, c.rec3);
        } else {
            hipLaunchKernelGGL(search_init_kernel, dim3(init_blocks), dim3(256), 0, st, c, D, a.R, a.JB, 0);
        }
        switch (D) {
            case 2: launch_prepass<2>(c, sc, a.L, st); break;
            case 3: launch_prepass<3>(c, sc, a.L, st, !s3); break;
            default: launch_prepass<4>(c, sc, a.L, st); break;
        }
        if (s4) {
            // the pair-group record table (part of the set-up, like rec3 above)
            const int64_t nrec = s4_rows_below(c.S, c.S - 2) * S4_NR;
            hipLaunchKernelGGL(rec4_kernel, dim3((unsigned)((nrec + 255) / 256)), dim3(256), 0, st, c, c.rec4, nrec);
        }
        phase_end(c, SISSO_PHASE_PREPASS, st);
        phase_begin(c, SISSO_PHASE_SEARCH, st);
        const size_t nrec = MT ? (size_t)a.JB * c.TP : (size_t)SEARCH_WG;
        const size_t lds = lds_lists + nrec * RECW * sizeof(double) + (size_t)64 * SUBW * sizeof(double);
        if (s4) {
            hipLaunchKernelGGL(search4_kernel, dim3(c.search_wgs), dim3(SEARCH_WG), lds_lists, st, c, a,
                               (const double *)c.rec4, (const uint64_t *)c.cum);
        } else if (s3 && MT) {
            hipLaunchKernelGGL(search3_kernel<true>, dim3(c.search_wgs), dim3(SEARCH_WG), lds_lists, st, c, a,
                               (const double *)c.rec3, (const uint64_t *)c.cum);
            const int nown = c.search_wgs * SEARCH_WAVES;  // the sweep waves' own chunks
            hipLaunchKernelGGL(mt_scan_kernel, dim3(1), dim3(PRE_WG), 0, st, c, nown);
            hipLaunchKernelGGL(mt_eval_kernel, dim3(c.search_wgs), dim3(SEARCH_WG), lds_lists, st, c, a,
                               (const double *)c.rec3, nown);
        }
        else if (s3)
            hipLaunchKernelGGL(search3_kernel<false>, dim3(c.search_wgs), dim3(SEARCH_WG), lds_lists, st, c, a,
                               (const double *)c.rec3, (const uint64_t *)c.cum);
        else switch (D) {
            case 2: MT ? launch_one<2, true>(c, a, lds, st) : launch_one<2, false>(c, a, lds, st); break;
            case 3: MT ? launch_one<3, true>(c, a, lds, st) : launch_one<3, false>(c, a, lds, st); break;
            case 4: MT ? launch_one<4, true>(c, a, lds, st) : launch_one<4, false>(c, a, lds, st); break;
            default: return -1;
        }
        phase_end(c, SISSO_PHASE_SEARCH, st);
        phase_begin(c, SISSO_PHASE_MERGE, st);
        launch_merge(c, c.search_wgs * SEARCH_WAVES, a.L, 1, st);
        phase_end(c, SISSO_PHASE_MERGE, st);
    }
    launch_rescore_final(c, D, sc.k, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}


int launch_prefix_best(const Ctx &c, int M, const int32_t *pre, int64_t n, double *best, hipStream_t st) {
    const unsigned wgs = (unsigned)(n < 4096 ? (n + 3) / 4 : 1024);
    switch (M) {
        case 1: hipLaunchKernelGGL((prefix_best_kernel<1>), dim3(wgs), dim3(256), 0, st, c, pre, n, best); break;
        case 2: hipLaunchKernelGGL((prefix_best_kernel<2>), dim3(wgs), dim3(256), 0, st, c, pre, n, best); break;
        case 3: hipLaunchKernelGGL((prefix_best_kernel<3>), dim3(wgs), dim3(256), 0, st, c, pre, n, best); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Training target of a prefix from its best extension's SSE:
// -log10(best / sum_t |y_t - mean|^2), the fraction clamped to [1e-12, 1];
// a prefix with no full-rank extension (best = +inf) or a malformed row
// (NaN) gets 0 (fraction 1).
__global__ void prefix_target_kernel(const double *__restrict__ cyy, int T, const double *__restrict__ best,
                                     int64_t n, float *__restrict__ target) {
    double ctot = 0.0;
    for (int t = 0; t < T; ++t) ctot += cyy[t];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double b = best[i];
        double frac = b / ctot;
        frac = frac < 1e-12 ? 1e-12 : (frac > 1.0 ? 1.0 : frac);
        if (!(b <= 1.7976931348623157e308)) frac = 1.0;  // +inf or NaN
        target[i] = (float)(-log10(frac));
    }
}

int launch_prefix_target(const Ctx &c, const double *best, int64_t n, float *target, hipStream_t st) {
    const unsigned blocks = (unsigned)(n < 262144 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(prefix_target_kernel, dim3(blocks), dim3(256), 0, st, c.cyy, c.T, best, n, target);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Every extension of each listed prefix: thread (p, t) writes the sorted
// (M + 1)-tuple P + {j}, j the t-th index of {0..S-1} not in P (walking the
// sorted prefix: each member at or below the running index pushes it up by
// one).  A malformed prefix row gives rows of -1.
template <int M>
__global__ __launch_bounds__(256) void prefix_extend_kernel(int64_t S, const int32_t *__restrict__ pre, int64_t n,
                                                            int32_t *__restrict__ out) {
    const int64_t w = S - M;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * w) return;
    const int64_t p = e / w, t = e - p * w;
    int32_t P[M];
    bool ok = true;
    for (int q = 0; q < M; ++q) {
        P[q] = pre[p * M + q];
        ok &= P[q] >= 0 && P[q] < S && (q == 0 || P[q] > P[q - 1]);
    }
    int32_t *o = out + e * (M + 1);
    if (!ok) {
        for (int q = 0; q <= M; ++q) o[q] = -1;
        return;
    }
    int64_t j = t;
    for (int q = 0; q < M; ++q) j += P[q] <= j ? 1 : 0;
    int q = 0, x = 0;
    for (; q < M && P[q] < j; ++q) o[x++] = P[q];
    o[x++] = (int32_t)j;
    for (; q < M; ++q) o[x++] = P[q];
}

int launch_prefix_extend(const Ctx &c, int M, const int32_t *pre, int64_t n, int32_t *out, hipStream_t st) {
    const int64_t tot = n * (c.S - M);
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    switch (M) {
        case 1: hipLaunchKernelGGL((prefix_extend_kernel<1>), dim3(blocks), dim3(256), 0, st, c.S, pre, n, out); break;
        case 2: hipLaunchKernelGGL((prefix_extend_kernel<2>), dim3(blocks), dim3(256), 0, st, c.S, pre, n, out); break;
        case 3: hipLaunchKernelGGL((prefix_extend_kernel<3>), dim3(blocks), dim3(256), 0, st, c.S, pre, n, out); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prefix_features(const Ctx &c, int M, const int32_t *pre, int64_t n, float *out, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (M) {
        case 1: hipLaunchKernelGGL((prefix_features_kernel<1>), dim3(blocks), dim3(256), 0, st, c, pre, n, out); break;
        case 2: hipLaunchKernelGGL((prefix_features_kernel<2>), dim3(blocks), dim3(256), 0, st, c, pre, n, out); break;
        case 3: hipLaunchKernelGGL((prefix_features_kernel<3>), dim3(blocks), dim3(256), 0, st, c, pre, n, out); break;
        case 4: hipLaunchKernelGGL((prefix_features_kernel<4>), dim3(blocks), dim3(256), 0, st, c, pre, n, out); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prefix_features_range(const Ctx &c, int M, uint64_t r0, int64_t n, float *out, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (M) {
        case 1: hipLaunchKernelGGL((prefix_features_range_kernel<1>), dim3(blocks), dim3(256), 0, st, c, r0, n, out); break;
        case 2: hipLaunchKernelGGL((prefix_features_range_kernel<2>), dim3(blocks), dim3(256), 0, st, c, r0, n, out); break;
        case 3: hipLaunchKernelGGL((prefix_features_range_kernel<3>), dim3(blocks), dim3(256), 0, st, c, r0, n, out); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_search(const Ctx &c, int D, int k, const int32_t *pre, int64_t n, hipStream_t st) {
    const unsigned init_blocks = (unsigned)(((SISSO_MAX_D + 1) * (c.S + 1) + 255) / 256);
    phase_begin(c, SISSO_PHASE_PREPASS, st);
    hipLaunchKernelGGL(search_init_kernel, dim3(init_blocks), dim3(256), 0, st, c, 2, 1, JBLK, 0);
    phase_end(c, SISSO_PHASE_PREPASS, st);
    int64_t wgs = (n + SEARCH_WAVES - 1) / SEARCH_WAVES;
    if (wgs > c.search_wgs) wgs = c.search_wgs;
    if (wgs < 1) wgs = 1;
    const size_t lds = (size_t)SEARCH_WAVES * c.KP * 2 * sizeof(double);
    phase_begin(c, SISSO_PHASE_SEARCH, st);
    switch (D - 1) {
        case 1: hipLaunchKernelGGL((list_search_kernel<1>), dim3((unsigned)wgs), dim3(SEARCH_WG), lds, st, c, pre, n); break;
        case 2: hipLaunchKernelGGL((list_search_kernel<2>), dim3((unsigned)wgs), dim3(SEARCH_WG), lds, st, c, pre, n); break;
        case 3: hipLaunchKernelGGL((list_search_kernel<3>), dim3((unsigned)wgs), dim3(SEARCH_WG), lds, st, c, pre, n); break;
        default: return -1;
    }
    phase_end(c, SISSO_PHASE_SEARCH, st);
    phase_begin(c, SISSO_PHASE_MERGE, st);
    launch_merge(c, (int)wgs * SEARCH_WAVES, 1, 0, st, 1);
    phase_end(c, SISSO_PHASE_MERGE, st);
    launch_rescore_final(c, D, k, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sl0
