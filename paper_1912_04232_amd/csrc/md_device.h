// Device-side building blocks shared by the gfx950 kernels: torus
// displacement, pair potentials, cell geometry, wave/block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace md {

constexpr int kBlock = 256;     // threads per workgroup for particle kernels
constexpr int kMaxSpecies = 8;

// Box as the kernels see it (Sec. 3.2.1).  A position is a uint32 fraction of
// the edge: x = u * s, s = L / 2^32.  The signed 32-bit wrap of u_i - u_j is
// the nearest-image displacement in units of s, exactly.
struct DevBox {
    float s[3];       // L_k / 2^32
    float inv_s[3];   // 2^32 / L_k
    double sd[3];     // L_k / 2^32 in double (exact)
    int nc[3];        // cells per dimension (1 = dimension scanned whole)
    int C;            // total cells
    int lo[3], hi[3]; // stencil offsets per dimension: [-1, 1] or [0, 0]
    float cw[3];      // cell width L_k / nc_k
    int iso;          // the same scale along every axis
};

// Per-pair-type coefficients (Sec. 3.3.2).  For LJ with r2i = 1/r^2 and
// q = r2i^3:  f/r = r2i q (a12 q - a6),  u = q (c12 q - c6) - ushift.
// For soft spheres: f/r = (eps/sig) t^(alpha-1) / r, u = eps/alpha t^alpha,
// t = 1 - r/sig.
struct DevPot {
    int kind;          // 0 LJ, 1 soft sphere, 2 Morse, 3 Buckingham
    int S;
    float rc2;         // LJ / Morse cutoff squared
    float alpha;
    int alpha_is_2;
    float mk;          // Morse: alpha log2(e)
    float a12[64], a6[64], c12[64], c6[64], ushift[64];  // LJ; Morse keeps 2 alpha eps in a12, eps in c12;
                                                         // Buckingham A/rho in a12, 6 C in a6, A in c12, C in c6
    float sig[64], inv_sig[64], eps_over_sig[64], eps_over_alpha[64];  // soft sphere
    double sigd[64];                                                    // sigma in double (overlap)
};

__device__ __forceinline__ float tdisp(uint32_t a, uint32_t b, float s)
{
    return (float)(int32_t)(a - b) * s;
}

__device__ __forceinline__ double tdisp_d(uint32_t a, uint32_t b, double s)
{
    return (double)(int32_t)(a - b) * s;
}

// Lennard-Jones: returns f/r (0 beyond the cutoff); u when WANT_U.
template <bool WANT_U>
__device__ __forceinline__ float lj_fs(float r2, float rc2, float a12, float a6, float c12, float c6, float ushift,
                                       float &u)
{
    float r2i = __builtin_amdgcn_rcpf(r2);
    float q = r2i * r2i * r2i;
    float fs = r2i * q * __builtin_fmaf(a12, q, -a6);
    bool in = r2 < rc2;
    if (WANT_U) u = in ? q * __builtin_fmaf(c12, q, -c6) - ushift : 0.0f;
    return in ? fs : 0.0f;
}

// Soft sphere with exponent alpha: returns f/r (0 for r >= sigma); u when WANT_U.
template <bool WANT_U>
__device__ __forceinline__ float ss_fs(float r2, float sig, float inv_sig, float eos, float eoa, float alpha,
                                       bool alpha2, float &u)
{
    float ri = __builtin_amdgcn_rsqf(r2);
    float r = r2 * ri;
    float t = __builtin_fmaf(-r, inv_sig, 1.0f);
    bool in = r < sig;
    float tp = alpha2 ? t : __builtin_exp2f((alpha - 1.0f) * __builtin_log2f(fmaxf(t, 1e-30f)));
    float fs = eos * tp * ri;
    if (WANT_U) u = in ? eoa * tp * t : 0.0f;
    return in ? fs : 0.0f;
}

// Morse, u = eps [(1 - x)^2 - 1] with x = exp(-alpha (r - r0)): returns f/r = 2 alpha eps x (x - 1) / r (0 beyond
// the cutoff); u = eps x (x - 2) - u(r_c) when WANT_U.
template <bool WANT_U>
__device__ __forceinline__ float morse_fs(float r2, float rc2, float r0, float mk, float eps, float two_ae,
                                          float ushift, float &u)
{
    float ri = __builtin_amdgcn_rsqf(r2);
    float r = r2 * ri;
    float x = __builtin_exp2f(mk * (r0 - r));
    float fs = two_ae * x * (x - 1.0f) * ri;
    bool in = r2 < rc2;
    if (WANT_U) u = in ? eps * x * (x - 2.0f) - ushift : 0.0f;
    return in ? fs : 0.0f;
}

// Buckingham, u = A exp(-r/rho) - C / r^6: returns f/r = (A/rho) exp(-r/rho) / r - 6 C / r^8 (0 beyond the cutoff);
// u - u(r_c) when WANT_U.  kr = log2(e) / rho, so exp(-r/rho) = exp2(-kr r).
template <bool WANT_U>
__device__ __forceinline__ float buck_fs(float r2, float rc2, float kr, float a_over_rho, float six_c, float a, float c,
                                         float ushift, float &u)
{
    float ri = __builtin_amdgcn_rsqf(r2);
    float r = r2 * ri;
    float x = __builtin_exp2f(-kr * r);
    float r2i = ri * ri;
    float r6i = r2i * r2i * r2i;
    float fs = a_over_rho * x * ri - six_c * r6i * r2i;
    bool in = r2 < rc2;
    if (WANT_U) u = in ? a * x - c * r6i - ushift : 0.0f;
    return in ? fs : 0.0f;
}

template <int KIND, bool MULTI, bool WANT_U>
__device__ __forceinline__ float pair_fs(const DevPot &p, int pt, float r2, float &u)
{
    if (KIND == 0) {
        int q = MULTI ? pt : 0;
        return lj_fs<WANT_U>(r2, p.rc2, p.a12[q], p.a6[q], p.c12[q], p.c6[q], p.ushift[q], u);
    } else if (KIND == 2) {
        int q = MULTI ? pt : 0;
        return morse_fs<WANT_U>(r2, p.rc2, p.sig[q], p.mk, p.c12[q], p.a12[q], p.ushift[q], u);
    } else if (KIND == 3) {
        int q = MULTI ? pt : 0;
        return buck_fs<WANT_U>(r2, p.rc2, p.inv_sig[q], p.a12[q], p.a6[q], p.c12[q], p.c6[q], p.ushift[q], u);
    } else {
        int q = MULTI ? pt : 0;
        return ss_fs<WANT_U>(r2, p.sig[q], p.inv_sig[q], p.eps_over_sig[q], p.eps_over_alpha[q], p.alpha,
                             p.alpha_is_2 != 0, u);
    }
}

// Soft sphere with the overlap t = 1 - r/sigma formed in double from the exact integer displacement
// (dd[k] = wrap32(u_ik - u_jk) * L_k/2^32): near contact t is a small difference of two numbers close to
// 1 and a float r would leave it with a relative error ~1e-7/t.  Returns f/r; u when WANT_U.
template <int D, bool MULTI, bool WANT_U>
__device__ __forceinline__ float ss_fs_precise(const DevPot &p, int pt, const double *dd, float &u)
{
    int q = MULTI ? pt : 0;
    double r2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) r2 = __builtin_fma(dd[k], dd[k], r2);
    double r = __builtin_sqrt(r2);
    double sig = p.sigd[q];
    bool in = r < sig;
    float t = (float)((sig - r) / sig);
    float tp = p.alpha_is_2 ? t : __builtin_exp2f((p.alpha - 1.0f) * __builtin_log2f(fmaxf(t, 1e-30f)));
    float fs = p.eps_over_sig[q] * tp / (float)r;
    if (WANT_U) u = in ? p.eps_over_alpha[q] * tp * t : 0.0f;
    return in ? fs : 0.0f;
}

// f/r (and u) of one pair from the torus coordinates ui, uj; d[] receives the float displacement.
template <int D, int KIND, bool MULTI, bool WANT_U>
__device__ __forceinline__ float pair_eval(const DevPot &p, int pt, const uint32_t *ui, const uint32_t *uj,
                                           const float *s, const double *sd, float *d, float &r2, float &u)
{
    r2 = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        d[k] = tdisp(ui[k], uj[k], s[k]);
        r2 = __builtin_fmaf(d[k], d[k], r2);
    }
    if (KIND != 1) return pair_fs<KIND, MULTI, WANT_U>(p, pt, r2, u);
    double dd[D];
#pragma unroll
    for (int k = 0; k < D; ++k) dd[k] = tdisp_d(ui[k], uj[k], sd[k]);
    return ss_fs_precise<D, MULTI, WANT_U>(p, pt, dd, u);
}

// Cell coordinate along one dimension: floor(u * nc / 2^32), exact in integers.
__device__ __forceinline__ int cell_coord(uint32_t u, int nc)
{
    return (int)(((uint64_t)u * (uint64_t)nc) >> 32);
}

template <int D>
__device__ __forceinline__ int cell_index(const uint32_t *ui, const DevBox &b)
{
    int c = cell_coord(ui[0], b.nc[0]) + b.nc[0] * cell_coord(ui[1], b.nc[1]);
    if constexpr (D == 3) c += b.nc[0] * b.nc[1] * cell_coord(ui[2], b.nc[2]);
    return c;
}

template <int D>
__device__ __forceinline__ void load_pos(const uint32_t *__restrict__ pos, int i, uint32_t *u)
{
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = pos[(size_t)i * D + k];
}

template <int D>
__device__ __forceinline__ void store_pos(uint32_t *__restrict__ pos, int i, const uint32_t *u)
{
#pragma unroll
    for (int k = 0; k < D; ++k) pos[(size_t)i * D + k] = u[k];
}

// Block-wide inclusive sum over kBlock threads (deterministic order).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds)
{
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) lds[t] = lds[t] + lds[t + off];
        __syncthreads();
    }
    T r = lds[0];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T *lds)
{
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) lds[t] = lds[t] > lds[t + off] ? lds[t] : lds[t + off];
        __syncthreads();
    }
    T r = lds[0];
    __syncthreads();
    return r;
}

// Exclusive scan of kBlock ints held one per thread (Hillis-Steele in LDS, no atomics).
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int &total)
{
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int a = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    int incl = lds[t];
    total = lds[kBlock - 1];
    __syncthreads();
    return incl - v;
}

}  // namespace md
