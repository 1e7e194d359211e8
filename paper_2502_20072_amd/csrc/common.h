// Shared definitions of the gfx950 l0 library: workspace layout, launch
// parameters, and host/device helpers for the combinatorial number system.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sisso_l0.h"

namespace sl0 {

constexpr int WAVE = 64;               // CDNA wavefront width
constexpr double RANK_EPS = 1e-10;     // pivot ratio at or below which a tuple is rank-deficient
constexpr double RANK_EPS_F32 = 1e-5;  // the same for the FP32 solve form (a few hundred units of 2^-23)
constexpr int GRAM_TILE = 128;         // Gram output tile (rows = cols)
#ifndef GRAM_KC_SAMPLES
#define GRAM_KC_SAMPLES 16
#endif
constexpr int GRAM_KC = GRAM_KC_SAMPLES;  // samples per LDS stage of the Gram (divides 256)
constexpr int SEARCH_WG = 256;         // threads per search workgroup (4 waves)
constexpr int SEARCH_WAVES = SEARCH_WG / WAVE;
constexpr int SEARCH_WGS_MAX = 2048;   // largest persistent search grid (lists are sized for it)
constexpr int SEARCH_WGS_DEFAULT = 1024;
constexpr int JBLK = 64;               // (D-1)-th indices per search work item (one per lane)
constexpr int SUBP = 4;                // sub-prefixes sharing one Gram load (single task)
constexpr int PRE_M = 16;              // features the threshold pre-pass starts from
constexpr int PRE_Q = 8;               // best prefixes the pre-pass extends by every feature
constexpr int KP_MAX = 512;            // longest per-wave candidate list
constexpr int LP_XC = 256;             // precision form: samples per slice-exponent chunk
constexpr int PROP_NF = 8;             // learned proposal: features per prefix

// ---------------------------------------------------------------- binomials
// C(n, r) exactly in 64-bit arithmetic, saturating at UINT64_MAX (never
// reached for accepted sizes, which keep C(S, D) < 2^63).  Multiplicative
// formula c <- c (n - r + i) / i with the division done first: with
// g = gcd(c, i), i/g divides n - r + i, so no intermediate exceeds the result.
__host__ __device__ inline uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

__host__ __device__ inline uint64_t binom(int64_t n, int r) {
    if (r < 0 || n < r) return 0;
    if (r == 0) return 1;
    if (r > n - r) r = (int)(n - r);
    uint64_t c = 1;
    for (int i = 1; i <= r; ++i) {
        const uint64_t g = gcd_u64(c, (uint64_t)i);
        const uint64_t m = (uint64_t)(n - r + i) / ((uint64_t)i / g);
        c /= g;
        if (c > UINT64_MAX / m) return UINT64_MAX;
        c *= m;
    }
    return c;
}

// Binomials from a table tab[r * (S + 1) + n], r <= SISSO_MAX_D, n <= S,
// filled on the device once per search (lookups replace the arithmetic in
// kernels); the host uses binom() directly.
struct BinomTab {
    const uint64_t *tab;
    int64_t S;
    __host__ __device__ uint64_t operator()(int64_t n, int r) const {
        return (r < 0 || n < r) ? 0 : tab[(int64_t)r * (S + 1) + n];
    }
};
struct BinomCalc {
    __host__ __device__ uint64_t operator()(int64_t n, int r) const { return binom(n, r); }
};

// Lexicographic rank of a sorted tuple (i_1 < ... < i_D) of {0..S-1}:
// tuples with a smaller first index come first, then by the second, etc.
// rank = sum_m [C(S - i_{m-1} - 1, D - m + 1) - C(S - i_m, D - m + 1)], i_0 = -1
// (the hockey-stick sum of the tuples skipped at position m).
template <class BF>
__host__ __device__ inline uint64_t lex_rank(const BF &bf, int64_t S, int D, const int32_t *t) {
    uint64_t r = 0;
    int64_t prev = -1;
    for (int m = 1; m <= D; ++m) {
        int64_t im = t[m - 1];
        r += bf(S - prev - 1, D - m + 1) - bf(S - im, D - m + 1);
        prev = im;
    }
    return r;
}

// Inverse of lex_rank: position by position, the m-th index is the largest
// x with count(x) <= r, where count(x) = C(S - prev - 1, k) - C(S - x, k)
// (k = D - m + 1) counts the tuples whose m-th index lies in (prev, x);
// found by bisection on that monotone count.
template <class BF>
__host__ __device__ inline void lex_unrank(const BF &bf, int64_t S, int D, uint64_t r, int32_t *t) {
    int64_t prev = -1;
    for (int m = 1; m <= D; ++m) {
        const int k = D - m + 1;
        const uint64_t base = bf(S - prev - 1, k);
        int64_t lo = prev + 1, hi = S - k;  // answer in [lo, hi]
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            uint64_t before = base - bf(S - mid, k);
            if (before <= r) lo = mid; else hi = mid - 1;
        }
        r -= base - bf(S - lo, k);
        t[m - 1] = (int32_t)lo;
        prev = lo;
    }
}

// Colexicographic unranking of a q-combination of {0..N-1}: the q-th element
// is the largest c with C(c, q) <= r, then recurse on r - C(c, q).  Used to
// hand out groups of sub-prefixes: colex ranks below C(N, q) are exactly the
// combinations inside {0..N-1}.
template <class BF>
__host__ __device__ inline void colex_unrank(const BF &bf, uint64_t r, int q, int64_t N, int32_t *t) {
    int64_t hi = N - 1;
    for (int m = q; m >= 1; --m) {
        int64_t lo = m - 1, h = hi;  // largest c in [m-1, hi] with C(c, m) <= r
        while (lo < h) {
            int64_t mid = (lo + h + 1) / 2;
            if (bf(mid, m) <= r) lo = mid; else h = mid - 1;
        }
        t[m - 1] = (int32_t)lo;
        r -= bf(lo, m);
        hi = lo - 1;
    }
}

// Top-k key of a sorted tuple: the indices packed most significant first,
// 64/D bits each, so integer order of keys is lexicographic order of tuples
// (equivalently, order of lexicographic rank).  Needs S <= 2^(64/D); no
// valid tuple packs to ~0 (indices are strictly increasing), which marks an
// empty slot.
__host__ __device__ inline int key_bits(int D) { return 64 / D; }
__host__ __device__ inline uint64_t pack_tuple(const int32_t *t, int D) {
    if (D == 1) return (uint64_t)(uint32_t)t[0];
    const int b = 64 / D;
    uint64_t k = 0;
    for (int m = 0; m < D; ++m) k = (k << b) | (uint64_t)(uint32_t)t[m];
    return k;
}
__host__ __device__ inline void unpack_tuple(uint64_t k, int D, int32_t *t) {
    if (D == 1) {
        t[0] = (int32_t)k;
        return;
    }
    const int b = 64 / D;
    const uint64_t mask = (1ull << b) - 1;
    for (int m = D - 1; m >= 0; --m) {
        t[m] = (int32_t)(k & mask);
        k >>= b;
    }
}

// ------------------------------------------------------ tiled Gram layout
// The correlation matrices are stored in 64 x 64 tiles (row-major inside a
// tile, tiles row-major, padded with zeros to a multiple of 64), task
// fastest: element (i, k) of task t is at gidx(i, k, nt, TP, t) with
// nt = ceil(S / 64).  A search step reads one row of one tile, so a chunk of
// 64 steps stays inside 32 KB of contiguous memory.
constexpr int GT = 64;
constexpr int MTQ_CHUNK = 256;  // queued sweep steps per pool chunk (several tasks, D = 3)
constexpr unsigned long long MTQ_POOL_MAX = 8ull << 30;  // largest pool of queued steps (bytes)
__host__ __device__ inline int64_t gidx(int64_t i, int64_t k, int64_t nt, int TP, int t) {
    return ((((i >> 6) * nt + (k >> 6)) << 12) + ((i & 63) << 6) + (k & 63)) * TP + t;
}

// Colexicographic unranking for the small sub-prefix lengths of the search
// (q <= 2 in closed form, larger q by bisection), no table lookups.
__host__ __device__ inline void colex_unrank_small(uint64_t r, int q, int64_t N, int32_t *t) {
    if (q == 1) {
        t[0] = (int32_t)r;
        return;
    }
    if (q == 3) {
        // largest c with c (c - 1) (c - 2) / 6 <= r, then the pair below it
        int64_t c = (int64_t)cbrt(6.0 * (double)r) + 2;
        auto c3 = [](int64_t x) { return x < 3 ? (uint64_t)0 : (uint64_t)(x * (x - 1) / 2) * (uint64_t)(x - 2) / 3; };
        while (c > 2 && c3(c) > r) --c;
        while (c3(c + 1) <= r) ++c;
        t[2] = (int32_t)c;
        colex_unrank_small(r - c3(c), 2, c, t);
        return;
    }
    if (q == 2) {
        // largest c with c (c - 1) / 2 <= r
        int64_t c = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)r)) * 0.5);
        while (c > 1 && (uint64_t)(c * (c - 1) / 2) > r) --c;
        while ((uint64_t)((c + 1) * c / 2) <= r) ++c;
        t[1] = (int32_t)c;
        t[0] = (int32_t)(r - (uint64_t)(c * (c - 1) / 2));
        return;
    }
    colex_unrank(BinomCalc{}, r, q, N, t);
}

// ----------------------------------------- D = 4, one task: record table
// Pairs (i1, i2) of a D = 4 prefix are grouped four at a time: group
// (i2, h) holds i1 = 4h .. 4h + 3 (those >= i2 are void), so a group exists
// for h < ceil(i2 / 4).  Groups are ordered by i2, then h.
constexpr int S4_NR = 4;        // pairs per group
constexpr int S4_RECW = 5;      // doubles per pair record: v0, v1, 1/d_j, z_j / s_j, p
constexpr int S4_ROW = S4_NR * S4_RECW;  // doubles per record row (160 bytes)
constexpr int S4_KC = 128;      // k per tile: two adjacent per lane
constexpr int S4_JR = 32;       // j rows per tile (divides 64)
constexpr size_t S4_TABLE_MAX = (size_t)4 << 30;  // largest record table kept in the workspace

// groups with i2 < i: sum over i' < i of ceil(i' / 4)
__host__ __device__ inline int64_t s4_groups_below(int64_t i) {
    if (i <= 1) return 0;
    const int64_t N = i - 1, a = N / 4, b = N % 4;
    return (i - 1) + 2 * a * (a - 1) + b * a;
}
// record rows of the groups with i2 < i: sum over i' < i of ceil(i'/4) (S - 2 - i')
__host__ __device__ inline int64_t s4_rows_below(int64_t S, int64_t i) {
    int64_t acc = 0;
    for (int64_t x = 1; x < i && x <= S - 3; ++x) acc += ((x + 3) / 4) * (S - 2 - x);
    return acc;
}

// -------------------------------------------------------- workspace layout
// Every region is 256-byte aligned; offsets in bytes from the workspace base.
struct Layout {
    size_t off_dev;    // int64 [T+1]
    size_t torder;     // int32 [T] tasks by decreasing row count (the Gram's launch order)
    size_t ybar;       // double [T]
    size_t cyy;        // double [T]   |y_t - ybar_t|^2
    size_t mu;         // double [T][S] column means per task
    size_t inv_s;      // double [T][S] 1/|x - mean| (0 for a constant column)
    size_t bhat;       // double [S][TP] normalised F_t^T y_t
    size_t G;          // double [S][S][TP] correlation matrices, task fastest
    size_t part;       // double [nsplit][T][S][S] raw centred Gram partial sums
    size_t flags;      // uint32 [64] device status words
    size_t lp_cbase;   // int32 [T+1] precision form: first chunk of each task
    size_t lp_exp;     // int32 [S][nchunk] precision form: chunk exponents
    size_t lp_slices;  // bf16 [NS][S][nchunk * LP_XC] precision form: slices
    size_t stat_bits;  // uint64 [4] error report scratch
    size_t pre;        // pre-pass scratch
    size_t rec3;       // D = 3: pair records of the filter task, double [ceil(S/4)][S][4][4] (0 bytes otherwise)
    size_t rec3_bytes;
    size_t G1;         // D = 3, several tasks: the filter task's matrix alone, double [S][S] tiled (0 bytes otherwise)
    size_t G1_bytes;
    size_t rec4;       // D = 4, one task: pair-group records, double [rows][S4_ROW] (0 bytes otherwise)
    size_t rec4_bytes;
    size_t self;       // a device copy of the handle's Ctx (read by the batched search)
    size_t btab;       // batched search: item prefix and context table, when this handle leads a batch
    size_t r4off;      //   int64 [S + 1] record rows of the groups below each i2
    size_t mtq;        // D = 3, several tasks: flagged sweep steps, uint64 [mtq_chunks][MTQ_CHUNK][3]
    size_t mtq_n;      //   uint32 [mtq_chunks] keys per chunk
    size_t mtq_pre;    //   uint64 [mtq_chunks + 1] exclusive prefix of the counts
    int mtq_chunks;    //   chunks in the pool (0: no queue)
    size_t lists;      // per-wave top lists: (double sse, uint64 rank) [nwaves][KP]
    size_t merged;     // merged candidates [KP] (sse, rank)
    size_t rescored;   // rescored candidates [KP] (sse, rank)
    size_t coef;       // double [KP][T][D_max+1]
    size_t res;        // result block, read back by one copy: status words uint32 [4], then
    size_t res_sse;    //   double [k_max],
    size_t res_idx;    //   int32 [k_max][D_max] (padded to 8 bytes),
    size_t res_coef;   //   double [k_max][T][D_max+1]
    size_t res_bytes;  // block size without / with the coefficients: res_coef - res, res_bytes
    size_t total;
    int TP;            // tasks padded to a power of two
    int nsplit;        // split-K factor of the Gram
    int KP;            // list length per wave (power of two >= k_max + margin)
    int nwaves;        // persistent search waves
    int search_wgs;    // persistent search workgroups
    int lp_ns;         // precision form: slices per value (0 = FP64 Gram)
    int fp32;          // FP32 solve form (FP64 Gram, per-tuple solves in FP32)
    int lp_nchunk;     // precision form: chunks over all tasks
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// device status flag indices
enum {
    FLAG_NONFINITE = 0,
    FLAG_CAPACITY = 1,
    FLAG_CAND = 2,
    FLAG_THETA = 4,   /* uint64 at 4..5 */
    FLAG_BATCHQ = 8,  /* batched search: next queue item (read on the batch's first problem) */
    FLAG_NLISTS = 9   /* batched search: lists this problem's waves have written */
};

}  // namespace sl0
