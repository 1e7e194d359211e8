// The small network of the learned proposal: FP32 training kernels
// (forward, backward with ordered reductions, Adam) and a BF16 MFMA
// inference kernel.  Layout and semantics: include/sisso_mlp.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/sisso_l0.h"
#include "../../include/sisso_mlp.h"
#include "common.h"

namespace sl0 {
namespace {

constexpr int IN = SISSO_MLP_IN;
constexpr int H = SISSO_MLP_HIDDEN;
constexpr int NP = SISSO_MLP_NPARAM;
constexpr int OW1 = 0, OB1 = IN * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
static_assert(OB3 + 1 == NP, "parameter layout");
constexpr int FB = 16;  // samples per forward / hidden-gradient block
constexpr int GB = 64;  // samples per weight-gradient block (one partial row each)

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Ws {
    float *h1, *h2, *o, *dz2, *dz1, *dout, *part;
};

Ws carve(void *base, int64_t n) {
    char *p = (char *)base;
    Ws w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = p + off;
        off = al(off + bytes);
        return (float *)q;
    };
    w.h1 = take((size_t)n * H * 4);
    w.h2 = take((size_t)n * H * 4);
    w.o = take((size_t)n * 4);
    w.dz2 = take((size_t)n * H * 4);
    w.dz1 = take((size_t)n * H * 4);
    w.dout = take((size_t)n * 4);
    w.part = take((size_t)((n + GB - 1) / GB) * (NP + 1) * 4);
    return w;
}

size_t ws_bytes(int64_t n) {
    return al((size_t)n * H * 4) * 4 + al((size_t)n * 4) * 2 + al((size_t)((n + GB - 1) / GB) * (NP + 1) * 4) + 256;
}

// ------------------------------------------------------------- forward
// Block: FB samples; thread (s, g) owns hidden units 8g..8g+7 of sample s.
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ P, const float *__restrict__ x,
                                                          int64_t n, float *__restrict__ h1g, float *__restrict__ h2g,
                                                          float *__restrict__ out) {
    __shared__ float h1s[FB][H];
    const int tid = threadIdx.x, s = tid >> 4, g = tid & 15;
    const int64_t i = (int64_t)blockIdx.x * FB + s;
    const bool live = i < n;
    float xi[IN];
#pragma unroll
    for (int a = 0; a < IN; ++a) xi[a] = live ? x[i * IN + a] : 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int j = 8 * g + u;
        float z = P[OB1 + j];
#pragma unroll
        for (int a = 0; a < IN; ++a) z = fmaf(xi[a], P[OW1 + a * H + j], z);
        z = fmaxf(z, 0.f);
        h1s[s][j] = z;
        if (live) h1g[i * H + j] = z;
    }
    __syncthreads();
    float o = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int j = 8 * g + u;
        float z = P[OB2 + j];
        for (int k = 0; k < H; ++k) z = fmaf(h1s[s][k], P[OW2 + k * H + j], z);
        z = fmaxf(z, 0.f);
        if (live) h2g[i * H + j] = z;
        o = fmaf(z, P[OW3 + j], o);
    }
    for (int m = 8; m >= 1; m >>= 1) o += __shfl_xor(o, m);  // the 16 threads of sample s
    if (g == 0 && live) out[i] = o + P[OB3];
}

// ------------------------------------------------------------ backward
__global__ void mlp_dout_kernel(const float *__restrict__ o, const float *__restrict__ y, int64_t n,
                                float *__restrict__ dout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dout[i] = 2.f * (o[i] - y[i]) / (float)n;
}

// dz2[i][j] = dout[i] W3[j] [h2 > 0]
__global__ void mlp_dz2_kernel(const float *__restrict__ P, const float *__restrict__ h2, const float *__restrict__ dout,
                               int64_t n, float *__restrict__ dz2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * H) return;
    const int64_t i = e / H;
    const int j = (int)(e % H);
    dz2[e] = h2[e] > 0.f ? dout[i] * P[OW3 + j] : 0.f;
}

// dz1[i][k] = (sum_j dz2[i][j] W2[k][j]) [h1 > 0]; block of FB samples
__global__ __launch_bounds__(256) void mlp_dz1_kernel(const float *__restrict__ P, const float *__restrict__ h1,
                                                      const float *__restrict__ dz2, int64_t n, float *__restrict__ dz1) {
    __shared__ float d2[FB][H];
    const int tid = threadIdx.x, s = tid >> 4, g = tid & 15;
    const int64_t i = (int64_t)blockIdx.x * FB + s;
    const bool live = i < n;
#pragma unroll
    for (int u = 0; u < 8; ++u) d2[s][8 * g + u] = live ? dz2[i * H + 8 * g + u] : 0.f;
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int k = 8 * g + u;
        float z = 0.f;
        for (int j = 0; j < H; ++j) z = fmaf(d2[s][j], P[OW2 + k * H + j], z);
        dz1[i * H + k] = h1[i * H + k] > 0.f ? z : 0.f;
    }
}

// Per-block partial sums over GB samples (fixed order) of every parameter
// gradient and of the squared error; row b of part has NP + 1 entries.
__global__ __launch_bounds__(256) void mlp_grad_partial_kernel(const float *__restrict__ x, const float *__restrict__ h1,
                                                               const float *__restrict__ h2, const float *__restrict__ o,
                                                               const float *__restrict__ y, const float *__restrict__ dz1,
                                                               const float *__restrict__ dz2, const float *__restrict__ dout,
                                                               int64_t n, float *__restrict__ part) {
    __shared__ float sh1[GB][H + 1], sd2[GB][H + 1];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * GB;
    const int cnt = (int)(n - i0 < GB ? n - i0 : GB);
    for (int e = tid; e < GB * H; e += 256) {
        const int s = e / H, k = e % H;
        sh1[s][k] = s < cnt ? h1[(i0 + s) * H + k] : 0.f;
        sd2[s][k] = s < cnt ? dz2[(i0 + s) * H + k] : 0.f;
    }
    __syncthreads();
    float *row = part + (int64_t)blockIdx.x * (NP + 1);
    for (int p = tid; p < NP + 1; p += 256) {
        float acc = 0.f;
        if (p < OB1) {  // W1[a][k]: x[a] dz1[k]
            const int a = p / H, k = p % H;
            for (int s = 0; s < cnt; ++s) acc = fmaf(x[(i0 + s) * IN + a], dz1[(i0 + s) * H + k], acc);
        } else if (p < OW2) {  // b1[k]
            const int k = p - OB1;
            for (int s = 0; s < cnt; ++s) acc += dz1[(i0 + s) * H + k];
        } else if (p < OB2) {  // W2[k][j]: h1[k] dz2[j]
            const int k = (p - OW2) / H, j = (p - OW2) % H;
            for (int s = 0; s < cnt; ++s) acc = fmaf(sh1[s][k], sd2[s][j], acc);
        } else if (p < OW3) {  // b2[j]
            const int j = p - OB2;
            for (int s = 0; s < cnt; ++s) acc += sd2[s][j];
        } else if (p < OB3) {  // W3[j]: h2[j] dout
            const int j = p - OW3;
            for (int s = 0; s < cnt; ++s) acc = fmaf(h2[(i0 + s) * H + j], dout[i0 + s], acc);
        } else if (p == OB3) {
            for (int s = 0; s < cnt; ++s) acc += dout[i0 + s];
        } else {  // squared error
            for (int s = 0; s < cnt; ++s) {
                const float d = o[i0 + s] - y[i0 + s];
                acc = fmaf(d, d, acc);
            }
        }
        row[p] = acc;
    }
}

__global__ void mlp_reduce_kernel(const float *__restrict__ part, int nb, int64_t n, float *__restrict__ grad,
                                  float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * (NP + 1) + p];
    if (p < NP) grad[p] = acc;
    else loss[0] = acc / (float)n;
}

__global__ void mlp_adam_kernel(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, int step, float lr) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mi = b1 * m[p] + (1.f - b1) * g[p];
    const float vi = b2 * v[p] + (1.f - b2) * g[p] * g[p];
    m[p] = mi;
    v[p] = vi;
    const float mh = mi / (1.f - powf(b1, (float)step));
    const float vh = vi / (1.f - powf(b2, (float)step));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------- BF16 MFMA inference
// Block: 4 waves, persistent over groups of 64 samples (16 per wave).  Both
// hidden layers run on v_mfma_f32_16x16x32_bf16 (A[i][k] in lane i + 16
// (k / 8), element k % 8; B[k][j] in lane j + 16 (k / 8); D[i][j] in lane
// j + 16 (i / 4), register i % 4), the output layer in FP32.
//  - layer 1 is computed transposed, h1^T = W1^T x^T (inputs padded from 8
//    to the MFMA's 32), so each lane receives 4 consecutive hidden units of
//    one sample from each 16-row block;
//  - layer 2 takes those as its A operand directly: in K-step s, element e
//    of lane i + 16 g is hidden unit hid(s, g, e) = 32 s + 4 g + e (e < 4) or
//    32 s + 16 + 4 g + (e - 4) (e >= 4), and W2 is staged in LDS in the same
//    unit order, so the contraction is over all 128 units exactly once.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int WT = H + 8;  // LDS row stride of the staged W2 (BF16 elements)

template <int CTRL>
__device__ inline float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ inline int hid_of(int s, int g, int e) { return 32 * s + (e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4)); }

// Register budget for two waves per SIMD (the W2 fragments are reused by
// every sample group; one wave per SIMD left every load latency exposed).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void mlp_infer_bf16_kernel(
    const float *__restrict__ P, const float *__restrict__ x,
                                                             int64_t n, float *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) __bf16 w2t[H][WT];  // [output j][MFMA k order]
    for (int e = threadIdx.x; e < H * H; e += 256) {
        const int j = e / H, kk = e % H;  // kk = 32 s + 8 g + el
        const int s = kk >> 5, g = (kk >> 3) & 3, el = kk & 7;
        w2t[j][kk] = (__bf16)P[OW2 + hid_of(s, g, el) * H + j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    // layer-1 operands that do not change with the samples: W1^T blocks
    // (rows = hidden units, k = inputs; only lanes of k-group 0 hold inputs)
    // and the bias as the accumulator's start value
    bf16x8 A1[H / 32][2];
    f32x4 B1init[H / 32][2];
#pragma unroll
    for (int s = 0; s < H / 32; ++s)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const int row = 32 * s + 16 * hf + r16;
#pragma unroll
            for (int e = 0; e < 8; ++e) A1[s][hf][e] = (__bf16)(g == 0 && e < IN ? P[OW1 + e * H + row] : 0.f);
#pragma unroll
            for (int r = 0; r < 4; ++r) B1init[s][hf][r] = P[OB1 + 32 * s + 16 * hf + 4 * g + r];
        }
    float b2r[H / 16], w3r[H / 16];
#pragma unroll
    for (int cb = 0; cb < H / 16; ++cb) {
        b2r[cb] = P[OB2 + 16 * cb + r16];
        w3r[cb] = P[OW3 + 16 * cb + r16];
    }
    const float b3 = P[OB3];
    // the inputs of the next group of samples are loaded while this one is
    // computed (lanes of k-group 0 hold the 8 inputs of sample r16)
    auto load_x = [&](int64_t gs, float4 &lo, float4 &hi) {
        const int64_t i = gs + wave * 16 + r16;
        lo = (float4){0.f, 0.f, 0.f, 0.f};
        hi = (float4){0.f, 0.f, 0.f, 0.f};
        if (g == 0 && i < n) {
            lo = reinterpret_cast<const float4 *>(x + i * IN)[0];
            hi = reinterpret_cast<const float4 *>(x + i * IN)[1];
        }
    };
    float4 xlo, xhi;
    load_x((int64_t)blockIdx.x * 64, xlo, xhi);
    for (int64_t g0 = (int64_t)blockIdx.x * 64; g0 < n; g0 += (int64_t)gridDim.x * 64) {
        const int64_t i0 = g0 + wave * 16;
        // x^T as the B operand
        bf16x8 Bx;
        Bx[0] = (__bf16)xlo.x; Bx[1] = (__bf16)xlo.y; Bx[2] = (__bf16)xlo.z; Bx[3] = (__bf16)xlo.w;
        Bx[4] = (__bf16)xhi.x; Bx[5] = (__bf16)xhi.y; Bx[6] = (__bf16)xhi.z; Bx[7] = (__bf16)xhi.w;
        load_x(g0 + (int64_t)gridDim.x * 64, xlo, xhi);
        bf16x8 A2[H / 32];
#pragma unroll
        for (int s = 0; s < H / 32; ++s)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[s][hf], Bx, B1init[s][hf], 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) A2[s][4 * hf + r] = (__bf16)fmaxf(acc[r], 0.f);
            }
        // eight independent accumulators, K-steps outermost, so consecutive
        // MFMAs do not wait on each other
        f32x4 acc[H / 16];
#pragma unroll
        for (int cb = 0; cb < H / 16; ++cb) acc[cb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < H / 32; ++s)
#pragma unroll
            for (int cb = 0; cb < H / 16; ++cb) {
                const bf16x8 Bw = *reinterpret_cast<const bf16x8 *>(&w2t[16 * cb + r16][32 * s + 8 * g]);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[s], Bw, acc[cb], 0, 0, 0);
            }
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int cb = 0; cb < H / 16; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[r] = fmaf(fmaxf(acc[cb][r] + b2r[cb], 0.f), w3r[cb], part[r]);
        // sum over the 16 columns of a row: row-local DPP steps (lane ^ 1,
        // lane ^ 2, mirror in 8, mirror in 16); every lane gets the row sum
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            part[r] += dpp_f32<0xB1>(part[r]);
            part[r] += dpp_f32<0x4E>(part[r]);
            part[r] += dpp_f32<0x141>(part[r]);
            part[r] += dpp_f32<0x140>(part[r]);
        }
        if (r16 == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 4 * g + r;
                if (i < n) out[i] = part[r] + b3;
            }
        }
    }
}

// ------------------------------------------------------ top-K selection
// Scores are mapped to order-preserving unsigned keys.  A 4096-bin
// histogram of the top 12 key bits finds the bin holding the K-th largest
// score; a second histogram of the next 12 bits inside that bin refines the
// cut, and every score whose key is at or above it is selected (count >= K,
// exceeding K only by scores within 2^8 key units of the K-th; the set does
// not depend on scheduling).
constexpr int SEL_BINS = 4096;
__device__ inline uint32_t okey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // larger float -> larger key
}

struct SelState {
    unsigned long long count;  // selected so far (compaction)
    unsigned long long above;  // scores in level-0 bins above the cut bin
    unsigned int b1;           // level-0 cut bin
    unsigned int thr;          // final key threshold
};

// level 0: all scores, bin = key >> 20; level 1: scores in bin b1, bin = (key >> 8) & 0xfff
__global__ void sel_hist_kernel(const float *__restrict__ sc, int64_t n, int level, const SelState *__restrict__ st,
                                unsigned int *__restrict__ hist) {
    __shared__ unsigned int h[SEL_BINS];
    for (int b = threadIdx.x; b < SEL_BINS; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const unsigned b1 = level ? st->b1 : 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float f = sc[i];
        if (f != f) continue;  // NaN scores are never selected
        const uint32_t k = okey(f);
        if (level == 0) atomicAdd(&h[k >> 20], 1u);
        else if ((k >> 20) == b1) atomicAdd(&h[(k >> 8) & 0xfffu], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < SEL_BINS; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// one thread: the highest bin at which the count from the top reaches the target
__global__ void sel_threshold_kernel(const unsigned int *__restrict__ hist, int64_t K, int level,
                                     SelState *__restrict__ st) {
    const int64_t target = level ? K - (int64_t)st->above : K;
    int64_t acc = 0;
    int b = SEL_BINS - 1;
    for (; b > 0; --b) {
        if (acc + (int64_t)hist[b] >= target) break;
        acc += hist[b];
    }
    if (level == 0) {
        st->b1 = (unsigned)b;
        st->above = (unsigned long long)acc;
    } else {
        st->thr = (st->b1 << 20) | ((unsigned)b << 8);
        st->count = 0ull;
    }
}

__global__ void sel_compact_kernel(const float *__restrict__ sc, int64_t n, SelState *__restrict__ st,
                                   uint64_t *__restrict__ out, int64_t cap) {
    const uint32_t thr = st->thr;
    const int lane = threadIdx.x & 63;
    // one atomic per wave: the selected lanes take consecutive slots
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const float f = i < n ? sc[i] : __builtin_nanf("");
        const bool take = f == f && okey(f) >= thr;
        const unsigned long long m = __ballot(take);
        if (!m) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&st->count, (unsigned long long)__popcll(m));
        base = __shfl(base, 0);
        const unsigned long long at = base + __popcll(m & ((1ull << lane) - 1ull));
        if (take && (int64_t)at < cap) out[at] = (uint64_t)i;
    }
}

__global__ void sel_clear_kernel(unsigned int *__restrict__ hist) {
    for (int b = threadIdx.x; b < SEL_BINS; b += blockDim.x) hist[b] = 0u;
}

// Colexicographic unranking (q <= 3) of a rank list into prefix rows,
// each row sorted ascending.
__global__ void colex_unrank_kernel(int m, const uint64_t *__restrict__ ranks, int64_t n, int32_t *__restrict__ pre) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t t[4];
    colex_unrank_small(ranks[i], m, (int64_t)1 << 30, t);
    for (int a = 0; a < m; ++a) pre[i * m + a] = t[a];
}

int32_t launched() { return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_EDEVICE; }

}  // namespace
}  // namespace sl0

using namespace sl0;

extern "C" size_t sisso_mlp_workspace_bytes(int64_t n) { return n < 1 ? 0 : ws_bytes(n); }

extern "C" int32_t sisso_mlp_forward(const float *params, const float *x, int64_t n, float *out, void *workspace,
                                     size_t workspace_bytes, void *stream) {
    if (!params || !x || !out || !workspace || n < 1 || workspace_bytes < ws_bytes(n)) return SISSO_EINVAL;
    const Ws w = carve(workspace, n);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + FB - 1) / FB)), dim3(256), 0, st, params, x, n, w.h1,
                       w.h2, w.o);
    if (hipMemcpyAsync(out, w.o, (size_t)n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) return SISSO_EDEVICE;
    return launched();
}

extern "C" int32_t sisso_mlp_backward(const float *params, const float *x, const float *target, int64_t n, float *grad,
                                      float *loss, void *workspace, size_t workspace_bytes, void *stream) {
    if (!params || !x || !target || !grad || !loss || !workspace || n < 1 || workspace_bytes < ws_bytes(n))
        return SISSO_EINVAL;
    const Ws w = carve(workspace, n);
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((n + GB - 1) / GB);
    hipLaunchKernelGGL(mlp_dout_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w.o, target, n, w.dout);
    hipLaunchKernelGGL(mlp_dz2_kernel, dim3((unsigned)((n * H + 255) / 256)), dim3(256), 0, st, params, w.h2, w.dout, n,
                       w.dz2);
    hipLaunchKernelGGL(mlp_dz1_kernel, dim3((unsigned)((n + FB - 1) / FB)), dim3(256), 0, st, params, w.h1, w.dz2, n,
                       w.dz1);
    hipLaunchKernelGGL(mlp_grad_partial_kernel, dim3((unsigned)nb), dim3(256), 0, st, x, w.h1, w.h2, w.o, target, w.dz1,
                       w.dz2, w.dout, n, w.part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, w.part, nb, n, grad, loss);
    return launched();
}

extern "C" int32_t sisso_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                                  void *stream) {
    if (!params || !grad || !m || !v || step < 1) return SISSO_EINVAL;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                       step, lr);
    return launched();
}

extern "C" int32_t sisso_mlp_infer_bf16(const float *params, const float *x, int64_t n, float *out, void *stream) {
    if (!params || !x || !out || n < 1) return SISSO_EINVAL;
    const int64_t groups = (n + 63) / 64;
    hipLaunchKernelGGL(mlp_infer_bf16_kernel, dim3((unsigned)(groups < 1024 ? groups : 1024)), dim3(256), 0,
                       (hipStream_t)stream, params, x, n, out);
    return launched();
}

extern "C" size_t sisso_select_workspace_bytes(void) { return SEL_BINS * sizeof(unsigned int) + 256; }

static thread_local const char *g_select_err = "";

static int32_t select_fail(int32_t code, const char *msg) {
    g_select_err = msg;
    return code;
}

// The selection on a scratch area of sisso_select_workspace_bytes() bytes:
// the level histograms (cleared by a kernel before each level) and the state
// (every field written before it is read).
static int32_t select_top(const float *scores, int64_t n, int64_t K, uint64_t *out, int64_t cap, int64_t *count,
                          void *scratch_area, hipStream_t st) {
    unsigned int *hist = (unsigned int *)scratch_area;  // [SEL_BINS], then the state
    SelState *ss = (SelState *)((char *)scratch_area + SEL_BINS * sizeof(unsigned int));
    const unsigned grid = (unsigned)(n / 1024 + 1 < 2048 ? n / 1024 + 1 : 2048);
    for (int level = 0; level < 2; ++level) {
        hipLaunchKernelGGL(sel_clear_kernel, dim3(1), dim3(1024), 0, st, hist);
        hipLaunchKernelGGL(sel_hist_kernel, dim3(grid), dim3(1024), 0, st, scores, n, level, ss, hist);
        hipLaunchKernelGGL(sel_threshold_kernel, dim3(1), dim3(1), 0, st, hist, K, level, ss);
    }
    hipLaunchKernelGGL(sel_compact_kernel, dim3(grid), dim3(1024), 0, st, scores, n, ss, out, cap);
    unsigned long long h = 0;
    if (hipMemcpyAsync(&h, &ss->count, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return select_fail(SISSO_EDEVICE, "a HIP call of the selection failed");
    *count = (int64_t)h;
    if (launched() != SISSO_OK) return select_fail(SISSO_EDEVICE, "a selection kernel failed to launch");
    if ((int64_t)h > cap) return select_fail(SISSO_EINVAL, "more scores selected than cap");
    return SISSO_OK;
}

static bool select_args_ok(const float *scores, int64_t n, int64_t K, const uint64_t *out, int64_t cap,
                           const int64_t *count) {
    return scores && out && count && n >= 1 && K >= 1 && K <= n && cap >= 1;
}

extern "C" int32_t sisso_select_top(const float *scores, int64_t n, int64_t K, uint64_t *out, int64_t cap,
                                    int64_t *count, void *workspace, size_t workspace_bytes, void *stream) {
    g_select_err = "";
    if (!select_args_ok(scores, n, K, out, cap, count) || !workspace)
        return select_fail(SISSO_EINVAL, "null pointer, or n, K, cap out of range");
    if (workspace_bytes < sisso_select_workspace_bytes())
        return select_fail(SISSO_EINVAL, "workspace smaller than sisso_select_workspace_bytes()");
    return select_top(scores, n, K, out, cap, count, workspace, (hipStream_t)stream);
}

// ---------------------------------------------- selection without a workspace
// For callers that cannot allocate device memory: the selection's scratch
// lives in this fixed device array.  Every GPU holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is not a
// device address in host code).
constexpr size_t SEL_SCRATCH_BYTES = SEL_BINS * sizeof(unsigned int) + 256;
static __device__ __align__(256) unsigned char scratch[SEL_SCRATCH_BYTES];
static_assert(sizeof(SelState) <= 256, "selection state fits its slot");

constexpr int SEL_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SEL_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
static int32_t scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return select_fail(SISSO_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= SEL_MAX_DEVICES) return select_fail(SISSO_ENOTSUP, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return select_fail(SISSO_EDEVICE, "hipGetSymbolAddress of the selection scratch failed");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SISSO_OK;
}

extern "C" size_t sisso_select_noalloc_scratch_bytes(void) { return SEL_SCRATCH_BYTES; }

extern "C" int32_t sisso_select_top_noalloc(const float *scores, int64_t n, int64_t K, uint64_t *out, int64_t cap,
                                            int64_t *count, void *stream) {
    g_select_err = "";
    if (!select_args_ok(scores, n, K, out, cap, count))
        return select_fail(SISSO_EINVAL, "null pointer, or n, K, cap out of range");
    if (sisso_select_workspace_bytes() > SEL_SCRATCH_BYTES)
        return select_fail(SISSO_ENOMEM, "the selection needs more scratch than the fixed device array holds");
    hipStream_t st = (hipStream_t)stream;
    int cur = -1, sdev = -1;
    if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(st, &sdev) != hipSuccess)
        return select_fail(SISSO_EDEVICE, "cannot query the current device or the stream's device");
    if (sdev != cur) return select_fail(SISSO_EINVAL, "the stream must belong to the current device");
    void *area = nullptr;
    const int32_t rc = scratch_address(&area);
    if (rc != SISSO_OK) return rc;
    return select_top(scores, n, K, out, cap, count, area, st);
}

extern "C" const char *sisso_select_last_error(void) { return g_select_err; }

extern "C" int32_t sisso_colex_unrank(int32_t m, const uint64_t *ranks, int64_t n, int32_t *prefixes, void *stream) {
    if (m < 1 || m > 3 || !ranks || !prefixes || n < 0) return SISSO_EINVAL;
    if (n == 0) return SISSO_OK;
    hipLaunchKernelGGL(colex_unrank_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, m, ranks,
                       n, prefixes);
    return launched();
}
