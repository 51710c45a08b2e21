// Neural pair potential on gfx950: radial descriptors, a per-atom MLP on BF16 MFMA, forces, and the
// training pass (loss, pair adjoint, weight gradient, Adam).
//
// The model (the paper's neural-network energies, Sec. 3.2.4 / 4.1, with forces F = -grad E, Sec. 3.3.2):
//   G_i^k = sum_{j != i, r_ij < r_c} g_k(r_ij),  g_k(r) = exp(-eta (r - mu_k)^2) fc(r),
//   fc(r) = (cos(pi r / r_c) + 1)/2,  mu_k = mu0 + k (mu1 - mu0)/(K - 1)
//   x = (G - m)/s,  h1 = sp(W1 x + b1),  h2 = sp(W2 h1 + b2),  E_i = w3 . h2 + b3,  sp = softplus
//   F_i = -sum_j sum_k (e_i^k + e_j^k) g_k'(r_ij) (r_i - r_j)/r_ij,  e_i = dE_i/dG_i
// K = 16, H = 64.  Training (Sec. 4.1) minimises
//   L = (1/S) sum_s ((E_s - E^_s)/n)^2 + lam_F/(3N) sum_i |F_i - F^_i|^2
// over S configurations of n atoms (N = S n).  With lam_i = dL/dF_i, the force term reaches the weights
// through the pair adjoint  ebar_i = dL/de_i = -sum_j g'(r_ij) u_ij . (lam_i - lam_j)  and the tangent
// (forward-mode) pass of each atom's network along ebar_i / s, whose reverse pass gives the weight gradient.
//
//   k_nn_descriptor  W lanes per atom walk its neighbor list and sum the 16 basis functions.
//   k_nn_mlp         one wave per tile of 32 atoms: X W1^T, H1 W2^T (forward) and D2 W2, D1 W1 (the input
//                    gradient e) as v_mfma_f32_32x32x16_bf16 products.  Weights are BF16 (the model's own
//                    values); activations enter as a BF16 pair hi + lo (hi = bf16(a), lo = bf16(a - hi)), two
//                    products per layer, so the activation side keeps ~16 mantissa bits; FP32 accumulation.
//   k_nn_force       W lanes per atom gather e_j and sum the pair terms.
//   k_nn_adjoint     the same walk with lam_j: ebar_i.
//   k_nn_train       one wave per tile: the forward pass again, the tangent pass along ebar/s, the reverse
//                    pass, and the weight gradients as MFMA products over the tile's atoms (per-unit adjoints
//                    transposed times the layer inputs, BF16), accumulated across tiles in registers; one
//                    partial gradient per wave, summed in a fixed order by k_nn_grad_reduce.
//   k_nn_loss_*      per-system energy residuals, force residuals lam_i and the loss (double, fixed order).
//   k_nn_adam        Adam on FP32 master weights; writes the BF16 copies the other kernels read.
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
constexpr int kTile = 32;  // atoms per wave tile
// flat parameter vector: W1 [H][K], b1 [H], W2 [H][H], b2 [H], w3 [H], b3
constexpr int oW1 = 0, ob1 = kH * kK, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH, ob3 = ow3 + kH;
constexpr int kNP = ob3 + 1;
static_assert(kNP == kNNParams, "parameter layout");
constexpr int kTrainWaves = kNNTrainWaves;  // partial gradients (one per wave of a training launch)

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

__device__ __forceinline__ void split_bf(float x, uint16_t &hi, uint16_t &lo)
{
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

struct NNDev {
    float mu0, dmu, r_c, eta;
    const uint16_t *W1;  // [H][K]
    const uint16_t *W2;  // [H][H]
    const float *b1, *b2, *w3, *b3;
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
    const float nel2 = -p.eta * 1.4426950408889634f;  // -eta log2(e): exp(-eta t^2) = 2^(nel2 t^2)
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        float t = r - (p.mu0 + k * p.dmu);
        float gauss = __builtin_amdgcn_exp2f(nel2 * t * t);
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
    // the next entry's index and position are loaded while the current pair is evaluated
    int jn = n > 0 ? idx[(size_t)ii * W + l] : ii;
    uint32_t un[D];
    load_pos<D>(pos, jn, un);
    for (int t = 0; t < n; ++t) {
        uint32_t uj[D];
#pragma unroll
        for (int q = 0; q < D; ++q) uj[q] = un[q];
        if (t + 1 < n) {
            jn = idx[((size_t)(t + 1) * N + ii) * W + l];
            load_pos<D>(pos, jn, un);
        }
        asm volatile("" ::: "memory");  // keep the loads above ahead of the arithmetic below
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
    // the next entry's index, position and e row are loaded while the current pair is evaluated
    int jn = n > 0 ? idx[(size_t)ii * W + l] : ii;
    uint32_t un[D];
    load_pos<D>(pos, jn, un);
    float4 en[kK / 4];
#pragma unroll
    for (int k = 0; k < kK / 4; ++k) en[k] = ((const float4 *)(e + (size_t)jn * kK))[k];
    for (int t = 0; t < n; ++t) {
        uint32_t uj[D];
#pragma unroll
        for (int q = 0; q < D; ++q) uj[q] = un[q];
        float4 ej[kK / 4];
#pragma unroll
        for (int k = 0; k < kK / 4; ++k) ej[k] = en[k];
        if (t + 1 < n) {
            jn = idx[((size_t)(t + 1) * N + ii) * W + l];
            load_pos<D>(pos, jn, un);
#pragma unroll
            for (int k = 0; k < kK / 4; ++k) en[k] = ((const float4 *)(e + (size_t)jn * kK))[k];
        }
        asm volatile("" ::: "memory");  // keep the loads above ahead of the arithmetic below
        float d[D];
        float r2 = pair_r<D>(ui, uj, b, d);
        if (r2 < rc2) {
            float r = sqrtf(r2);
            float g[kK], dg[kK];
            rbf<true>(p, r, g, dg);
            const float *ejf = (const float *)ej;
            float coef = 0.0f;
#pragma unroll
            for (int k = 0; k < kK; ++k) coef = __builtin_fmaf(ei[k] + ejf[k], dg[k], coef);
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

// ebar_i^k = -sum_j g_k'(r_ij) u_ij . (lam_i - lam_j), u_ij = (r_i - r_j)/r_ij: the transpose of the force map
// F(e) at fixed positions applied to lam.
template <int D, int W>
__global__ __launch_bounds__(kBlock) void k_nn_adjoint(DevBox b, NNDev p, const uint32_t *__restrict__ pos, int N,
                                                       const int32_t *__restrict__ idx,
                                                       const int32_t *__restrict__ count, int capW,
                                                       const float *__restrict__ lam, float *__restrict__ ebar)
{
    int gt = blockIdx.x * kBlock + threadIdx.x;
    int i = gt / W, l = gt % W;
    bool live = i < N;
    int ii = live ? i : N - 1;
    uint32_t ui[D];
    load_pos<D>(pos, ii, ui);
    float li[D];
#pragma unroll
    for (int q = 0; q < D; ++q) li[q] = lam[(size_t)ii * D + q];
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
            float r = sqrtf(r2);
            float g[kK], dg[kK];
            rbf<true>(p, r, g, dg);
            float tt = 0.0f;
#pragma unroll
            for (int q = 0; q < D; ++q) tt = __builtin_fmaf(d[q], li[q] - lam[(size_t)j * D + q], tt);
            tt = -tt / r;
#pragma unroll
            for (int k = 0; k < kK; ++k) acc[k] = __builtin_fmaf(dg[k], tt, acc[k]);
        }
    }
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
#pragma unroll
        for (int k = 0; k < kK; ++k) acc[k] += __shfl_xor(acc[k], o);
    }
    if (live && l == 0) {
#pragma unroll
        for (int k = 0; k < kK; ++k) ebar[(size_t)i * kK + k] = acc[k];
    }
}

// ---------------------------------------------------------------------------------------------
// MFMA.  v_mfma_f32_32x32x16_bf16 on a 32 x 16 A tile and a 16 x 32 B tile: lane l supplies A row (l % 32),
// k = 8 (l / 32) .. +7 and B column (l % 32), the same k; accumulator register r of lane l holds C[row][col]
// with col = l % 32, row = (r % 4) + 4 (l / 32) + 8 (r / 4).  The products are C = A Bt^T with A and Bt
// row-major in LDS, K contiguous, rows padded by 8 elements against bank conflicts; or C = A M with the B
// columns read down a row-major M.

__device__ __forceinline__ int acc_row(int r, int lane)
{
    return (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p)
{
    return *(const bf16x8 *)p;  // 16-byte aligned: row strides and k offsets are multiples of 8 elements
}

template <int K>
__device__ __forceinline__ f32x16 mma(f32x16 c, const uint16_t *A, int lda, const uint16_t *Bt, int ldb)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int kk = 0; kk < K; kk += 16) {
        bf16x8 av = ld8(A + (lane & 31) * lda + kk + 8 * (lane >> 5));
        bf16x8 bv = ld8(Bt + (lane & 31) * ldb + kk + 8 * (lane >> 5));
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
    return c;
}

// c += A B with B[k][n] = M[k][n0 + n] (columns n >= ncols are zero)
template <int K>
__device__ __forceinline__ f32x16 mma_bcol(f32x16 c, const uint16_t *A, int lda, const uint16_t *M, int ldm, int n0,
                                           int ncols)
{
    int lane = threadIdx.x & 63;
    bool live = (lane & 31) < ncols;
    int n = n0 + (live ? (lane & 31) : 0);
#pragma unroll
    for (int kk = 0; kk < K; kk += 16) {
        bf16x8 av = ld8(A + (lane & 31) * lda + kk + 8 * (lane >> 5));
        bf16x8 bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) bv[q] = live ? (short)M[(kk + 8 * (lane >> 5) + q) * ldm + n] : (short)0;
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
    return c;
}

__device__ __forceinline__ f32x16 zero16()
{
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = 0.0f;
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

// padded row strides (elements)
constexpr int L16 = 24, L32 = 40, L64 = 72;

// activation tile (32 atoms) as a BF16 pair hi + lo
template <int LD>
struct Pair {
    uint16_t h[kTile * LD];
    uint16_t l[kTile * LD];
};

template <int LD>
__device__ __forceinline__ void put_pair(Pair<LD> &t, int row, int col, float v)
{
    uint16_t h, l;
    split_bf(v, h, l);
    t.h[row * LD + col] = h;
    t.l[row * LD + col] = l;
}

// A(hi, lo) Bt^T for the 32 columns of Bt: the two products of a split activation operand.
template <int K, int LD>
__device__ __forceinline__ f32x16 mma_split(const Pair<LD> &A, const uint16_t *Bt, int ldb)
{
    f32x16 c = mma<K>(zero16(), A.h, LD, Bt, ldb);
    return mma<K>(c, A.l, LD, Bt, ldb);
}

template <int K, int LD>
__device__ __forceinline__ f32x16 mma_split_bcol(const Pair<LD> &A, const uint16_t *M, int ldm, int n0, int ncols)
{
    f32x16 c = mma_bcol<K>(zero16(), A.h, LD, M, ldm, n0, ncols);
    return mma_bcol<K>(c, A.l, LD, M, ldm, n0, ncols);
}

// Weights in LDS: W1 [H][K] and W2 [H][H], BF16, padded rows.
struct WLds {
    uint16_t W1[kH * L16];
    uint16_t W2[kH * L64];
};

__device__ __forceinline__ void load_weights(WLds &w, const NNDev &p, int t, int nt)
{
    for (int q = t; q < kH * kK; q += nt) w.W1[(q / kK) * L16 + q % kK] = p.W1[q];
    for (int q = t; q < kH * kH; q += nt) w.W2[(q / kH) * L64 + q % kH] = p.W2[q];
}

// X = (G - m)/s of atoms a0 .. a0+31 (zero rows past N) into a split tile.
__device__ __forceinline__ void load_x(Pair<L16> &X, const NNDev &p, const float *G, int a0, int N, int lane)
{
    for (int q = lane; q < kTile * kK; q += 64) {
        int row = q / kK, k = q % kK, a = a0 + row;
        float x = a < N ? (G[(size_t)a * kK + k] - p.m[k]) / p.s[k] : 0.0f;
        put_pair(X, row, k, x);
    }
}

constexpr int kMlpWaves = 4;  // waves per workgroup of k_nn_mlp, sharing one copy of the weights

struct MlpLds {
    WLds w;
    Pair<L16> Xs[kMlpWaves];
    Pair<L64> Ts[kMlpWaves];
    float Es[kMlpWaves][kTile];
};

// Orders one wave's LDS writes before its later reads (every lane of the wave takes part).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-atom energies E_i and input gradients e_i = dE_i/dG_i for atoms [0, N), one wave per 32-atom tile; the
// kMlpWaves waves of a workgroup share the weights staged once in LDS and work on tiles of their own.
__global__ __launch_bounds__(64 * kMlpWaves) void k_nn_mlp(NNDev p, const float *__restrict__ G, int N,
                                                           float *__restrict__ Ei, float *__restrict__ e)
{
    __shared__ __align__(16) MlpLds sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int c32 = lane & 31;
    load_weights(sh.w, p, threadIdx.x, 64 * kMlpWaves);
    __syncthreads();
    struct {
        const WLds &w;
        Pair<L16> &X;
        Pair<L64> &T;
        float *E;
    } s = {sh.w, sh.Xs[wv], sh.Ts[wv], sh.Es[wv]};
    float b1[2], b2[2], w3[2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        b1[hf] = p.b1[32 * hf + c32];
        b2[hf] = p.b2[32 * hf + c32];
        w3[hf] = p.w3[32 * hf + c32];
    }
    float b3 = *p.b3;
    int ntiles = (N + kTile - 1) / kTile;
    for (int tile = blockIdx.x * kMlpWaves + wv; tile < ntiles; tile += gridDim.x * kMlpWaves) {
        int a0 = tile * kTile;
        wave_sync();
        load_x(s.X, p, G, a0, N, lane);
        wave_sync();
        // z1 = X W1^T + b1; h1 = sp(z1) -> T; a1 = sp'(z1)
        float a1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kK>(s.X, s.w.W1 + 32 * hf * L16, L16);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float z = c[r] + b1[hf];
                a1[hf][r] = sigmoid(z);
                put_pair(s.T, acc_row(r, lane), 32 * hf + c32, softplus(z));
            }
        }
        wave_sync();
        // z2 = H1 W2^T + b2; E_i = w3 . sp(z2) + b3; d2 = sp'(z2) w3
        float d2[2][16], erow[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) erow[r] = 0.0f;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kH>(s.T, s.w.W2 + 32 * hf * L64, L64);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float z = c[r] + b2[hf];
                erow[r] += w3[hf] * softplus(z);
                d2[hf][r] = sigmoid(z) * w3[hf];
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float v = erow[r];
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
            erow[r] = v;
        }
        if (c32 == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) s.E[acc_row(r, lane)] = erow[r];
        }
        wave_sync();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
#pragma unroll
            for (int r = 0; r < 16; ++r) put_pair(s.T, acc_row(r, lane), 32 * hf + c32, d2[hf][r]);
        wave_sync();
        if (lane < kTile && a0 + lane < N) Ei[a0 + lane] = s.E[lane] + b3;
        // d1 = a1 * (D2 W2)
        float d1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split_bcol<kH>(s.T, s.w.W2, L64, 32 * hf, 32);
#pragma unroll
            for (int r = 0; r < 16; ++r) d1[hf][r] = c[r] * a1[hf][r];
        }
        wave_sync();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
#pragma unroll
            for (int r = 0; r < 16; ++r) put_pair(s.T, acc_row(r, lane), 32 * hf + c32, d1[hf][r]);
        wave_sync();
        // e = (D1 W1) / s  (columns k < K of the product)
        f32x16 c = mma_split_bcol<kH>(s.T, s.w.W1, L16, 0, kK);
        if (c32 < kK) {
            float sk = p.s[c32];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int a = a0 + acc_row(r, lane);
                if (a < N) e[(size_t)a * kK + c32] = c[r] / sk;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// training pass

struct TrainLds {
    WLds w;
    Pair<L16> X;              // x, later xd (the tangent input)
    uint16_t Xt[32 * L32];    // x transposed [input k][atom], rows >= K zero
    uint16_t Xdt[32 * L32];   // xd transposed
    Pair<L64> A1;             // h1, later g_z2
    Pair<L64> A2;             // d2, later hd1
    uint16_t H1t[kH * L32];   // h1 transposed [unit][atom], later g_z1 transposed
    uint16_t D2t[kH * L32];   // d2 (the adjoint of z2 in the tangent's reverse pass) transposed
    uint16_t D1t[kH * L32];   // d1 (the adjoint of zd1) transposed
    uint16_t Hd1t[kH * L32];  // hd1 transposed
    uint16_t Gz2t[kH * L32];  // g_z2 transposed
};

__device__ __forceinline__ void put_t(uint16_t *t, int unit, int atom, float v)
{
    t[unit * L32 + atom] = f2bf(v);
}

// Weight gradient of the loss over atoms [0, N): the reverse pass of E_i with seed gE (one value per system of
// `seg` atoms) plus the reverse pass of the tangent w3 . hd2_i along xd_i = ebar_i / s.  One partial gradient
// (kNP floats) per wave.
__global__ __launch_bounds__(64) void k_nn_train(NNDev p, const float *__restrict__ G, int N, int seg,
                                                 const float *__restrict__ gE, const float *__restrict__ ebar,
                                                 float *__restrict__ partial)
{
    __shared__ __align__(16) TrainLds s;
    int lane = threadIdx.x;
    int c32 = lane & 31;
    load_weights(s.w, p, lane, 64);
    for (int q = lane; q < 32 * L32; q += 64) {
        s.Xt[q] = 0;
        s.Xdt[q] = 0;
    }
    float b1[2], b2[2], w3[2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        b1[hf] = p.b1[32 * hf + c32];
        b2[hf] = p.b2[32 * hf + c32];
        w3[hf] = p.w3[32 * hf + c32];
    }
    f32x16 gW2[2][2], gW1[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        gW1[a] = zero16();
        gW2[a][0] = zero16();
        gW2[a][1] = zero16();
    }
    float gb1[2] = {0.0f, 0.0f}, gb2[2] = {0.0f, 0.0f}, gw3[2] = {0.0f, 0.0f}, gb3 = 0.0f;
    int ntiles = (N + kTile - 1) / kTile;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int a0 = tile * kTile;
        __syncthreads();
        load_x(s.X, p, G, a0, N, lane);
        for (int q = lane; q < kTile * kK; q += 64) {
            int row = q / kK, k = q % kK, a = a0 + row;
            float x = a < N ? (G[(size_t)a * kK + k] - p.m[k]) / p.s[k] : 0.0f;
            s.Xt[k * L32 + row] = f2bf(x);
            float xd = a < N ? ebar[(size_t)a * kK + k] / p.s[k] : 0.0f;
            s.Xdt[k * L32 + row] = f2bf(xd);
        }
        float ge[16];  // dL/dE_i of the rows this lane holds
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int a = a0 + acc_row(r, lane);
            ge[r] = a < N ? gE[seg > 0 ? a / seg : 0] : 0.0f;
        }
        if (lane < kTile && a0 + lane < N) gb3 += gE[seg > 0 ? (a0 + lane) / seg : 0];
        __syncthreads();
        // forward: z1, h1 -> A1, H1t
        float z1[2][16], z2[2][16], g1[2][16], zd1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kK>(s.X, s.w.W1 + 32 * hf * L16, L16);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                z1[hf][r] = c[r] + b1[hf];
                float h = softplus(z1[hf][r]);
                put_pair(s.A1, acc_row(r, lane), 32 * hf + c32, h);
                put_t(s.H1t, 32 * hf + c32, acc_row(r, lane), h);
            }
        }
        __syncthreads();
        // z2; d2 = sp'(z2) w3 -> A2, D2t; the energy seed reaches w3 through h2
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kH>(s.A1, s.w.W2 + 32 * hf * L64, L64);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                z2[hf][r] = c[r] + b2[hf];
                float d = sigmoid(z2[hf][r]) * w3[hf];
                put_pair(s.A2, acc_row(r, lane), 32 * hf + c32, d);
                put_t(s.D2t, 32 * hf + c32, acc_row(r, lane), d);
                gw3[hf] += ge[r] * softplus(z2[hf][r]);
            }
        }
        __syncthreads();
        // g1 = D2 W2 (= dE/dh1); d1 = sp'(z1) g1 -> D1t
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split_bcol<kH>(s.A2, s.w.W2, L64, 32 * hf, 32);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                g1[hf][r] = c[r];
                put_t(s.D1t, 32 * hf + c32, acc_row(r, lane), sigmoid(z1[hf][r]) * c[r]);
            }
        }
        __syncthreads();
        // tangent input xd = ebar / s -> X
        for (int q = lane; q < kTile * kK; q += 64) {
            int row = q / kK, k = q % kK, a = a0 + row;
            put_pair(s.X, row, k, a < N ? ebar[(size_t)a * kK + k] / p.s[k] : 0.0f);
        }
        __syncthreads();
        // zd1 = Xd W1^T; hd1 = sp'(z1) zd1 -> A2, Hd1t
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kK>(s.X, s.w.W1 + 32 * hf * L16, L16);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                zd1[hf][r] = c[r];
                float hd = sigmoid(z1[hf][r]) * c[r];
                put_pair(s.A2, acc_row(r, lane), 32 * hf + c32, hd);
                put_t(s.Hd1t, 32 * hf + c32, acc_row(r, lane), hd);
            }
        }
        __syncthreads();
        // zd2 = Hd1 W2^T; hd2 = sp'(z2) zd2; g_z2 = gE w3 sp'(z2) + w3 sp''(z2) zd2 -> A1, Gz2t
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split<kH>(s.A2, s.w.W2 + 32 * hf * L64, L64);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float sg = sigmoid(z2[hf][r]);
                float zd2 = c[r];
                gw3[hf] += sg * zd2;
                float gz2 = w3[hf] * (ge[r] * sg + sg * (1.0f - sg) * zd2);
                gb2[hf] += gz2;
                put_pair(s.A1, acc_row(r, lane), 32 * hf + c32, gz2);
                put_t(s.Gz2t, 32 * hf + c32, acc_row(r, lane), gz2);
            }
        }
        __syncthreads();
        // dW2 += G_z2^T H1 + D2^T Hd1 (products over the tile's atoms)
#pragma unroll
        for (int mh = 0; mh < 2; ++mh)
#pragma unroll
            for (int nh = 0; nh < 2; ++nh) {
                gW2[mh][nh] = mma<kTile>(gW2[mh][nh], s.Gz2t + 32 * mh * L32, L32, s.H1t + 32 * nh * L32, L32);
                gW2[mh][nh] = mma<kTile>(gW2[mh][nh], s.D2t + 32 * mh * L32, L32, s.Hd1t + 32 * nh * L32, L32);
            }
        // g_h1 = G_z2 W2; g_z1 = g_h1 sp'(z1) + g1 sp''(z1) zd1
        float gz1[2][16];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x16 c = mma_split_bcol<kH>(s.A1, s.w.W2, L64, 32 * hf, 32);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float sg = sigmoid(z1[hf][r]);
                gz1[hf][r] = c[r] * sg + g1[hf][r] * sg * (1.0f - sg) * zd1[hf][r];
                gb1[hf] += gz1[hf][r];
            }
        }
        __syncthreads();
        // g_z1 transposed -> H1t (h1 is no longer needed)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
#pragma unroll
            for (int r = 0; r < 16; ++r) put_t(s.H1t, 32 * hf + c32, acc_row(r, lane), gz1[hf][r]);
        __syncthreads();
        // dW1 += G_z1^T X + D1^T Xd
#pragma unroll
        for (int mh = 0; mh < 2; ++mh) {
            gW1[mh] = mma<kTile>(gW1[mh], s.H1t + 32 * mh * L32, L32, s.Xt, L32);
            gW1[mh] = mma<kTile>(gW1[mh], s.D1t + 32 * mh * L32, L32, s.Xdt, L32);
        }
    }
    // the wave's partial gradient; bias sums combine the two lane halves of each column
    float *out = partial + (size_t)blockIdx.x * kNP;
#pragma unroll
    for (int mh = 0; mh < 2; ++mh) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int row = 32 * mh + acc_row(r, lane);
            if (c32 < kK) out[oW1 + row * kK + c32] = gW1[mh][r];
#pragma unroll
            for (int nh = 0; nh < 2; ++nh) out[oW2 + row * kH + 32 * nh + c32] = gW2[mh][nh][r];
        }
    }
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        float v1 = gb1[hf] + __shfl_xor(gb1[hf], 32);
        float v2 = gb2[hf] + __shfl_xor(gb2[hf], 32);
        float v3 = gw3[hf] + __shfl_xor(gw3[hf], 32);
        if (lane < 32) {
            out[ob1 + 32 * hf + lane] = v1;
            out[ob2 + 32 * hf + lane] = v2;
            out[ow3 + 32 * hf + lane] = v3;
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) gb3 += __shfl_xor(gb3, o);
    if (lane == 0) out[ob3] = gb3;
}

// grad[q] = sum over waves w of partial[w][q], in double and in a fixed order: a workgroup takes 64 parameters, its 16
// waves sum the partials w = g, g + 16, ... (g = the wave) and the 16 sums are added in order of g.
constexpr int kRedGroups = 16;
__global__ __launch_bounds__(64 * kRedGroups) void k_nn_grad_reduce(const float *__restrict__ partial, int nw,
                                                                    float *__restrict__ grad)
{
    __shared__ double part[kRedGroups][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int q = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (q < kNP)
        for (int w = g; w < nw; w += kRedGroups) acc += (double)partial[(size_t)w * kNP + q];
    part[g][lane] = acc;
    __syncthreads();
    if (g == 0 && q < kNP) {
        double t = 0.0;
#pragma unroll
        for (int h = 0; h < kRedGroups; ++h) t += part[h][lane];
        grad[q] = (float)t;
    }
}

// Per basis function k (one workgroup each) over the N descriptors G [N][K]: mean m[k] and population standard
// deviation s[k] (1 where it is below 1e-8), in double and in a fixed order, two passes.
__global__ __launch_bounds__(kBlock) void k_nn_desc_stats(const float *__restrict__ G, int N, float *m, float *sd)
{
    __shared__ double red[kBlock / 64];
    const int k = blockIdx.x;
    auto block_sum = [&](double v) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w];
        __syncthreads();
        return t;
    };
    double sum = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) sum += (double)G[(size_t)i * kK + k];
    const double mean = block_sum(sum) / (double)(N > 0 ? N : 1);
    double var = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
        const double d = (double)G[(size_t)i * kK + k] - mean;
        var += d * d;
    }
    const double sdev = sqrt(block_sum(var) / (double)(N > 0 ? N : 1));
    if (threadIdx.x == 0) {
        m[k] = (float)mean;
        sd[k] = sdev > 1e-8 ? (float)sdev : 1.0f;
    }
}

// One workgroup per system s of `seg` atoms: E_s (double, fixed order), gE[s] and the system's part of the
// loss; lam_i = 2 lam_F (F_i - F^_i)/(3N) for its atoms.
__global__ __launch_bounds__(kBlock) void k_nn_loss_sys(const float *__restrict__ Ei, const float *__restrict__ F,
                                                        const double *__restrict__ E_ref,
                                                        const float *__restrict__ F_ref, int N, int seg, int S,
                                                        float lam_F, float *__restrict__ gE, float *__restrict__ lam,
                                                        double *__restrict__ part)
{
    __shared__ double red[kBlock];
    int sys = blockIdx.x;
    int a0 = sys * seg;
    double e = 0.0, f2 = 0.0;
    double cf = 2.0 * (double)lam_F / (3.0 * (double)N);
    for (int a = a0 + threadIdx.x; a < a0 + seg; a += kBlock) {
        e += (double)Ei[a];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double r = (double)F[(size_t)a * 3 + q] - (double)F_ref[(size_t)a * 3 + q];
            f2 += r * r;
            lam[(size_t)a * 3 + q] = (float)(cf * r);
        }
    }
    e = block_sum(e, red);
    f2 = block_sum(f2, red);
    if (threadIdx.x == 0) {
        double rE = (e - E_ref[sys]) / (double)seg;
        gE[sys] = (float)(2.0 * rE / ((double)seg * (double)S));
        part[sys] = rE * rE / (double)S + (double)lam_F * f2 / (3.0 * (double)N);
    }
}

__global__ __launch_bounds__(kBlock) void k_nn_loss_final(const double *__restrict__ part, int S,
                                                          double *__restrict__ loss)
{
    __shared__ double red[kBlock];
    double v = 0.0;
    for (int q = threadIdx.x; q < S; q += kBlock) v += part[q];
    v = block_sum(v, red);
    if (threadIdx.x == 0) loss[0] = v;
}

// Adam (Kingma & Ba) on the FP32 master vector; W1 and W2 also written as BF16 (round to nearest even).
__global__ __launch_bounds__(kBlock) void k_nn_adam(float *__restrict__ th, float *__restrict__ m,
                                                    float *__restrict__ v, const float *__restrict__ g, int n,
                                                    float lr, float b1, float b2, float eps, float c1, float c2,
                                                    uint16_t *__restrict__ W1, uint16_t *__restrict__ W2)
{
    int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    float gq = g[q];
    float mq = b1 * m[q] + (1.0f - b1) * gq;
    float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    float t = th[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
    th[q] = t;
    if (q >= oW1 && q < oW1 + kH * kK) W1[q - oW1] = f2bf(t);
    if (q >= oW2 && q < oW2 + kH * kH) W2[q - oW2] = f2bf(t);
}

// BF16 copies of W1 and W2 from the master vector.
__global__ __launch_bounds__(kBlock) void k_nn_cast(const float *__restrict__ th, uint16_t *__restrict__ W1,
                                                    uint16_t *__restrict__ W2)
{
    int q = blockIdx.x * kBlock + threadIdx.x;
    if (q < kH * kK) W1[q] = f2bf(th[oW1 + q]);
    if (q < kH * kH) W2[q] = f2bf(th[oW2 + q]);
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// host

static bool make_nn(const md_nn_params *q, NNDev &p)
{
    if (!q || q->K != kK || q->H != kH || !q->W1 || !q->W2 || !q->b1 || !q->b2 || !q->w3 || !q->b3 || !q->m || !q->s)
        return false;
    if (!(q->r_c > 0.0f) || !(q->mu1 > q->mu0)) return false;
    p.mu0 = q->mu0;
    p.dmu = (q->mu1 - q->mu0) / (kK - 1);
    p.r_c = q->r_c;
    if (!(q->eta >= 0.0f) || !isfinite(q->eta)) return false;
    p.eta = q->eta > 0.0f ? q->eta : 1.0f / (2.0f * p.dmu * p.dmu);
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
    if (!md_list_covers(nl, q->r_c)) return MD_ERR_ARG;
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
    int blocks = (ntiles + kMlpWaves - 1) / kMlpWaves;
    int grid = blocks < 2048 ? blocks : 2048;
    hipLaunchKernelGGL(k_nn_mlp, dim3(grid), dim3(64 * kMlpWaves), 0, (hipStream_t)stream, p, G, N, Ei, e);
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

md_status nn_pair_adjoint(md_ctx *ctx, const md_box *box, const md_nn_params *q, const uint32_t *pos, int32_t N,
                          const md_nlist *nl, const float *lam, float *ebar, void *stream)
{
    DevBox b;
    NNDev p;
    md_status st = nn_checks(ctx, box, q, pos, N, nl, b, p);
    if (st != MD_OK) return st;
    if (!lam || !ebar) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    int W = nl->lanes, capW = nl->capacity / W;
    int grid = (int)(((int64_t)N * W + kBlock - 1) / kBlock);
    NN_LANES(W, hipLaunchKernelGGL((k_nn_adjoint<3, W>), dim3(grid), dim3(kBlock), 0, s, b, p, pos, N, nl->idx,
                                   nl->count, capW, lam, ebar));
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_loss(md_ctx *ctx, const float *Ei, const float *F, const double *E_ref, const float *F_ref, int32_t N,
                  int32_t segment, float lam_F, double *loss, float *gE, float *lam, void *stream)
{
    if (!ctx || !Ei || !F || !E_ref || !F_ref || !loss || !gE || !lam || N <= 0 || segment <= 0 ||
        N % segment != 0)
        return MD_ERR_ARG;
    int S = N / segment;
    if (S > 4 * md_partials_blocks()) return MD_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_nn_loss_sys, dim3(S), dim3(kBlock), 0, s, Ei, F, E_ref, F_ref, N, segment, S, lam_F, gE,
                       lam, ctx->partials);
    hipLaunchKernelGGL(k_nn_loss_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, S, loss);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_mlp_grad(md_ctx *ctx, const md_nn_params *q, const float *G, int32_t N, int32_t segment,
                      const float *gE, const float *ebar, float *grad, void *stream)
{
    NNDev p;
    if (!ctx || !make_nn(q, p) || !G || !gE || !ebar || !grad || N <= 0 || segment < 0 ||
        (segment > 0 && N % segment != 0))
        return MD_ERR_ARG;
    int ntiles = (N + kTile - 1) / kTile;
    int nw = ntiles < kTrainWaves ? ntiles : kTrainWaves;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_nn_train, dim3(nw), dim3(64), 0, s, p, G, N, segment, gE, ebar, ctx->nn_partial);
    hipLaunchKernelGGL(k_nn_grad_reduce, dim3((kNP + 63) / 64), dim3(64 * kRedGroups), 0, s, ctx->nn_partial, nw,
                       grad);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_adam(md_ctx *ctx, float *theta, float *m, float *v, const float *grad, int32_t n, int32_t step, float lr,
                  float beta1, float beta2, float eps, uint16_t *W1, uint16_t *W2, void *stream)
{
    if (!ctx || !theta || !m || !v || !grad || !W1 || !W2 || n != kNP || step < 1) return MD_ERR_ARG;
    float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_nn_adam, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream, theta, m, v,
                       grad, n, lr, beta1, beta2, eps, c1, c2, W1, W2);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_descriptor_stats(md_ctx *ctx, const float *G, int32_t N, float *mean, float *scale, void *stream)
{
    if (!ctx || !G || !mean || !scale || N < 1) return MD_ERR_ARG;
    hipLaunchKernelGGL(k_nn_desc_stats, dim3(kK), dim3(kBlock), 0, (hipStream_t)stream, G, N, mean, scale);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nn_cast_weights(md_ctx *ctx, const float *theta, uint16_t *W1, uint16_t *W2, void *stream)
{
    if (!ctx || !theta || !W1 || !W2) return MD_ERR_ARG;
    hipLaunchKernelGGL(k_nn_cast, dim3((kH * kH + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream, theta,
                       W1, W2);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

int32_t nn_param_count(void)
{
    return kNP;
}

}  // extern "C"
