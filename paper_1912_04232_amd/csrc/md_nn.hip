// Neural pair potential on gfx950: radial descriptors, a per-atom MLP on BF16 MFMA, forces.
//
// The model (the paper's neural-network energies, Sec. 3.2.4 / 4.1, with forces F = -grad E, Sec. 3.3.2):
//   G_i^k = sum_{j != i, r_ij < r_c} g_k(r_ij),  g_k(r) = exp(-eta (r - mu_k)^2) fc(r),
//   fc(r) = (cos(pi r / r_c) + 1)/2,  mu_k = mu0 + k (mu1 - mu0)/(K - 1)
//   x = (G - m)/s,  h1 = sp(W1 x + b1),  h2 = sp(W2 h1 + b2),  E_i = w3 . h2 + b3,  sp = softplus
//   F_i = -sum_j sum_k (e_i^k + e_j^k) g_k'(r_ij) (r_i - r_j)/r_ij,  e_i = dE_i/dG_i
// K = 16, H = 64.
//
//   k_nn_descriptor  W lanes per atom walk its neighbor list (the ELL list of md_core) and sum the 16
//                    basis functions; lanes meet through __shfl_xor.
//   k_nn_mlp         one wave per tile of 32 atoms: X W1^T, H1 W2^T (forward) and D2 W2, D1 W1 (the input
//                    gradient e) as v_mfma_f32_32x32x16_bf16 products with BF16 operands staged in LDS and
//                    FP32 accumulation; activation derivatives stay in registers in the accumulator layout.
//   k_nn_force       W lanes per atom gather e_j and sum the pair terms.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

constexpr int kK = 16;
constexpr int kH = 64;
constexpr int kTile = 32;          // atoms per wave tile
constexpr int kMlpWaves = 4;
constexpr int kMlpThreads = 64 * kMlpWaves;

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

struct NNDev {
    float mu0, dmu, r_c, eta;
    const uint16_t *W1;  // [H][K]
    const uint16_t *W2;  // [H][H]
    const float *b1, *b2, *w3;
    float b3;
    const float *m, *s;  // [K]
};

// g_k(r) for k = 0..15 and, when DERIV, g_k'(r).
template <bool DERIV>
__device__ __forceinline__ void rbf(const NNDev &p, float r, float *g, float *dg)
{
    const float pi = 3.14159265358979f;
    float c = __cosf(pi * r / p.r_c);
    float fc = 0.5f * (c + 1.0f);
    float dfc = DERIV ? -0.5f * pi / p.r_c * __sinf(pi * r / p.r_c) : 0.0f;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        float t = r - (p.mu0 + k * p.dmu);
        float gauss = __expf(-p.eta * t * t);
        g[k] = gauss * fc;
        if (DERIV) dg[k] = gauss * (dfc - 2.0f * p.eta * t * fc);
    }
}

template <int D>
__device__ __forceinline__ float pair_r(const uint32_t *ui, const uint32_t *uj, const DevBox &b, float *d)
{
    float r2 = 0.0f;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        d[q] = tdisp(ui[q], uj[q], b.s[q]);
        r2 = __builtin_fmaf(d[q], d[q], r2);
    }
    return r2;
}

template <int D, int W>
__global__ __launch_bounds__(kBlock) void k_nn_descriptor(DevBox b, NNDev p, const uint32_t *__restrict__ pos, int N,
                                                          const int32_t *__restrict__ idx,
                                                          const int32_t *__restrict__ count, int capW,
                                                          float *__restrict__ G)
{
    int gt = blockIdx.x * kBlock + threadIdx.x;
    int i = gt / W, l = gt % W;
    bool live = i < N;
    int ii = live ? i : N - 1;
    uint32_t ui[D];
    load_pos<D>(pos, ii, ui);
    float acc[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) acc[k] = 0.0f;
    int n = live ? min(count[(size_t)ii * W + l], capW) : 0;
    float rc2 = p.r_c * p.r_c;
    for (int t = 0; t < n; ++t) {
        int j = idx[((size_t)t * N + ii) * W + l];
        uint32_t uj[D];
        load_pos<D>(pos, j, uj);
        float d[D];
        float r2 = pair_r<D>(ui, uj, b, d);
        if (r2 < rc2) {
            float g[kK];
            rbf<false>(p, sqrtf(r2), g, nullptr);
#pragma unroll
            for (int k = 0; k < kK; ++k) acc[k] += g[k];
        }
    }
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
#pragma unroll
        for (int k = 0; k < kK; ++k) acc[k] += __shfl_xor(acc[k], o);
    }
    if (live && l == 0) {
#pragma unroll
        for (int k = 0; k < kK; ++k) G[(size_t)i * kK + k] = acc[k];
    }
}

template <int D, int W>
__global__ __launch_bounds__(kBlock) void k_nn_force(DevBox b, NNDev p, const uint32_t *__restrict__ pos, int N,
                                                     const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ count, int capW,
                                                     const float *__restrict__ e, float *__restrict__ force,
                                                     int32_t *flags)
{
    int gt = blockIdx.x * kBlock + threadIdx.x;
    int i = gt / W, l = gt % W;
    bool live = i < N;
    int ii = live ? i : N - 1;
    uint32_t ui[D];
    load_pos<D>(pos, ii, ui);
    float ei[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) ei[k] = e[(size_t)ii * kK + k];
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    int n = live ? min(count[(size_t)ii * W + l], capW) : 0;
    float rc2 = p.r_c * p.r_c;
    for (int t = 0; t < n; ++t) {
        int j = idx[((size_t)t * N + ii) * W + l];
        uint32_t uj[D];
        load_pos<D>(pos, j, uj);
        float d[D];
        float r2 = pair_r<D>(ui, uj, b, d);
        if (r2 < rc2) {
            float r = sqrtf(r2);
            float g[kK], dg[kK];
            rbf<true>(p, r, g, dg);
            float coef = 0.0f;
#pragma unroll
            for (int k = 0; k < kK; ++k) coef = __builtin_fmaf(ei[k] + e[(size_t)j * kK + k], dg[k], coef);
            float fr = -coef / r;
#pragma unroll
            for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fr, d[q], F[q]);
        }
    }
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] += __shfl_xor(F[q], o);
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < D; ++q) bad = bad || !isfinite(F[q]);
    uint64_t m = __ballot(live && bad);
    if (m && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) flags[MD_FLAG_NONFINITE] = 1;
    if (live && l == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) force[(size_t)i * D + q] = F[q];
    }
}

// ---------------------------------------------------------------------------------------------
// MFMA helpers.  v_mfma_f32_32x32x16_bf16 on a 32 x 16 A tile and a 16 x 32 B tile: lane l supplies
// A row (l % 32), k = 8 (l / 32) .. +7 and B column (l % 32), the same k; accumulator register r of lane
// l holds C[row][col] with col = l % 32, row = (r % 4) + 4 (l / 32) + 8 (r / 4).

__device__ __forceinline__ int acc_row(int r, int lane)
{
    return (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
}

// C[32][32 * half .. +32] = A[32][K] (row-major bf16, LDS, row stride lda) x B where B column n is row
// (32 * half + n) of a row-major bf16 matrix Bt (LDS, row stride ldb): C = A Bt^T.
template <int K>
__device__ __forceinline__ f32x16 mfma_tile(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, int half)
{
    int lane = threadIdx.x & 63;
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = 0.0f;
#pragma unroll
    for (int kk = 0; kk < K; kk += 16) {
        const uint16_t *ap = A + (lane & 31) * lda + kk + 8 * (lane >> 5);
        const uint16_t *bp = Bt + (32 * half + (lane & 31)) * ldb + kk + 8 * (lane >> 5);
        bf16x8 av, bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            av[q] = (short)ap[q];
            bv[q] = (short)bp[q];
        }
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
    return c;
}

__device__ __forceinline__ float softplus(float z)
{
    return fmaxf(z, 0.0f) + __logf(1.0f + __expf(-fabsf(z)));
}

__device__ __forceinline__ float sigmoid(float z)
{
    return 1.0f / (1.0f + __expf(-z));
}

struct MlpLds {
    uint16_t W1[kH * kK];        // [H][K]
    uint16_t W1t[32 * kH];       // [32][H]: rows k < K hold column k of W1, rows K..31 are zero
    uint16_t W2[kH * kH];        // [H][H]
    uint16_t W2t[kH * kH];       // [H][H] transposed
    float b1[kH], b2[kH], w3[kH], m[kK], s[kK];
    uint16_t X[kMlpWaves][kTile * kK];
    uint16_t T[kMlpWaves][kTile * kH];
    float Erow[kMlpWaves][kTile];
};

// Per-atom energies E_i and input gradients e_i = dE_i/dG_i for atoms [0, N), 32 per wave tile.
__global__ __launch_bounds__(kMlpThreads) void k_nn_mlp(NNDev p, const float *__restrict__ G, int N,
                                                        float *__restrict__ Ei, float *__restrict__ e)
{
    __shared__ MlpLds s;
    int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int q = t; q < kH * kK; q += kMlpThreads) s.W1[q] = p.W1[q];
    for (int q = t; q < 32 * kH; q += kMlpThreads) {
        int k = q / kH, h = q % kH;
        s.W1t[q] = k < kK ? p.W1[h * kK + k] : (uint16_t)0;
    }
    for (int q = t; q < kH * kH; q += kMlpThreads) {
        s.W2[q] = p.W2[q];
        s.W2t[q] = p.W2[(q % kH) * kH + q / kH];
    }
    for (int q = t; q < kH; q += kMlpThreads) {
        s.b1[q] = p.b1[q];
        s.b2[q] = p.b2[q];
        s.w3[q] = p.w3[q];
    }
    for (int q = t; q < kK; q += kMlpThreads) {
        s.m[q] = p.m[q];
        s.s[q] = p.s[q];
    }
    __syncthreads();
    int ntiles = (N + kTile - 1) / kTile;
    // every wave of the block runs the same iterations (workgroup barriers inside); a wave past the last
    // tile works on zero rows and stores nothing
    for (int base = blockIdx.x * kMlpWaves; base < ntiles; base += gridDim.x * kMlpWaves) {
        int tile = base + w;
        int a0 = tile * kTile;
        // X = (G - m)/s in bf16, rows beyond N are zero
        for (int q = lane; q < kTile * kK; q += 64) {
            int row = q / kK, k = q % kK;
            int a = a0 + row;
            float x = a < N ? (G[(size_t)a * kK + k] - s.m[k]) / s.s[k] : 0.0f;
            s.X[w][q] = f2bf(x);
        }
        __syncthreads();
        // layer 1: z1 = X W1^T + b1; h1 = sp(z1) -> T (bf16); a1 = sp'(z1) kept in registers
        float a1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mfma_tile<kK>(s.X[w], kK, s.W1, kK, hf);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int row = acc_row(r, lane), col = 32 * hf + (lane & 31);
                float z = c[r] + s.b1[col];
                a1[hf][r] = sigmoid(z);
                s.T[w][row * kH + col] = f2bf(softplus(z));
            }
        }
        __syncthreads();
        // layer 2: z2 = H1 W2^T + b2; E_i = w3 . sp(z2) + b3; d2 = sp'(z2) * w3 -> T
        float d2[2][16];
        float erow[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) erow[r] = 0.0f;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mfma_tile<kH>(s.T[w], kH, s.W2, kH, hf);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int col = 32 * hf + (lane & 31);
                float z = c[r] + s.b2[col];
                erow[r] += s.w3[col] * softplus(z);
                d2[hf][r] = sigmoid(z) * s.w3[col];
            }
        }
        // row sums of w3 . h2 over the 64 columns: 32 lanes of a half hold one row's columns
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float v = erow[r];
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
            erow[r] = v;
        }
        if ((lane & 31) == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) s.Erow[w][acc_row(r, lane)] = erow[r];
        }
        __syncthreads();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int row = acc_row(r, lane), col = 32 * hf + (lane & 31);
                s.T[w][row * kH + col] = f2bf(d2[hf][r]);
            }
        }
        __syncthreads();
        if (lane < kTile && a0 + lane < N) Ei[a0 + lane] = s.Erow[w][lane] + p.b3;
        // d1 = a1 * (D2 W2): B column k of W2 is row k of W2t
        float d1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mfma_tile<kH>(s.T[w], kH, s.W2t, kH, hf);
#pragma unroll
            for (int r = 0; r < 16; ++r) d1[hf][r] = c[r] * a1[hf][r];
        }
        __syncthreads();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int row = acc_row(r, lane), col = 32 * hf + (lane & 31);
                s.T[w][row * kH + col] = f2bf(d1[hf][r]);
            }
        }
        __syncthreads();
        // e = (D1 W1) / s: B column k of W1 is row k of W1t (rows >= K are zero)
        f32x16 c = mfma_tile<kH>(s.T[w], kH, s.W1t, kH, 0);
        int col = lane & 31;
        if (col < kK) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int a = a0 + acc_row(r, lane);
                if (a < N) e[(size_t)a * kK + col] = c[r] / s.s[col];
            }
        }
        __syncthreads();
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// host

static bool make_nn(const md_nn_params *q, NNDev &p)
{
    if (!q || q->K != kK || q->H != kH || !q->W1 || !q->W2 || !q->b1 || !q->b2 || !q->w3 || !q->m || !q->s)
        return false;
    if (!(q->r_c > 0.0f) || !(q->mu1 > q->mu0)) return false;
    p.mu0 = q->mu0;
    p.dmu = (q->mu1 - q->mu0) / (kK - 1);
    p.r_c = q->r_c;
    p.eta = 1.0f / (2.0f * p.dmu * p.dmu);
    p.W1 = q->W1;
    p.W2 = q->W2;
    p.b1 = q->b1;
    p.b2 = q->b2;
    p.w3 = q->w3;
    p.b3 = q->b3;
    p.m = q->m;
    p.s = q->s;
    return true;
}

#define NN_LANES(W_, ...)                                                    \
    do {                                                                     \
        switch (W_) {                                                        \
        case 1: { constexpr int W = 1; __VA_ARGS__; } break;                 \
        case 2: { constexpr int W = 2; __VA_ARGS__; } break;                 \
        case 4: { constexpr int W = 4; __VA_ARGS__; } break;                 \
        default: { constexpr int W = 8; __VA_ARGS__; } break;                \
        }                                                                    \
    } while (0)

static md_status nn_checks(md_ctx *ctx, const md_box *box, const md_nn_params *q, const uint32_t *pos, int32_t N,
                           const md_nlist *nl, DevBox &b, NNDev &p)
{
    if (!ctx || !box || box->dim != 3 || !pos || N < 0 || !make_nn(q, p)) return MD_ERR_ARG;
    if (!nl || nl->N != N || !nl->idx || !nl->count || !(nl->lanes == 1 || nl->lanes == 2 || nl->lanes == 4 ||
                                                         nl->lanes == 8))
        return MD_ERR_ARG;
    if (nl->r_list < q->r_c) return MD_ERR_ARG;
    for (int k = 0; k < 3; ++k)
        if (!(nl->r_list < 0.5f * box->L[k])) return MD_ERR_BOX;
    memset(&b, 0, sizeof(b));
    for (int k = 0; k < 3; ++k) {
        b.s[k] = box->L[k] / 4294967296.0f;
        b.inv_s[k] = 4294967296.0f / box->L[k];
        b.sd[k] = (double)box->L[k] / 4294967296.0;
    }
    return MD_OK;
}

extern "C" {

md_status nn_descriptors(md_ctx *ctx, const md_box *box, const md_nn_params *q, const uint32_t *pos, int32_t N,
                         const md_nlist *nl, float *G, void *stream)
{
    DevBox b;
    NNDev p;
    md_status st = nn_checks(ctx, box, q, pos, N, nl, b, p);
    if (st != MD_OK) return st;
    if (!G) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    int W = nl->lanes, capW = nl->capacity / W;
    int grid = (int)(((int64_t)N * W + kBlock - 1) / kBlock);
    NN_LANES(W, hipLaunchKernelGGL((k_nn_descriptor<3, W>), dim3(grid), dim3(kBlock), 0, s, b, p, pos, N, nl->idx,
                                   nl->count, capW, G));
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_mlp(md_ctx *ctx, const md_nn_params *q, const float *G, int32_t N, float *Ei, float *e, void *stream)
{
    NNDev p;
    if (!ctx || !make_nn(q, p) || !G || !Ei || !e || N < 0) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    int ntiles = (N + kTile - 1) / kTile;
    int grid = (ntiles + kMlpWaves - 1) / kMlpWaves;
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(k_nn_mlp, dim3(grid), dim3(kMlpThreads), 0, (hipStream_t)stream, p, G, N, Ei, e);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_forces(md_ctx *ctx, const md_box *box, const md_nn_params *q, const uint32_t *pos, int32_t N,
                    const md_nlist *nl, const float *e, float *force, void *stream)
{
    DevBox b;
    NNDev p;
    md_status st = nn_checks(ctx, box, q, pos, N, nl, b, p);
    if (st != MD_OK) return st;
    if (!e || !force || !nl->flags) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    int W = nl->lanes, capW = nl->capacity / W;
    int grid = (int)(((int64_t)N * W + kBlock - 1) / kBlock);
    NN_LANES(W, hipLaunchKernelGGL((k_nn_force<3, W>), dim3(grid), dim3(kBlock), 0, s, b, p, pos, N, nl->idx,
                                   nl->count, capW, e, force, nl->flags));
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
