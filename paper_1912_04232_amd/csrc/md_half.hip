// Newton's-third-law variant of the list force pass, kept for comparison with the full list (Sec. 3.2.3 builds
// neighbor lists; each pair can be stored once and its force applied to both particles).
//
//   k_half_compact  keeps each pair of a full list (W interleaved sub-rows) in one of its two rows, in a one-lane
//                   layout hidx[t][i], hcount[i]: row i keeps j when (i < j) differs from (i + j odd), so a pair
//                   with i < j sits in row i when i + j is even and in row j when it is odd, and every row holds
//                   about half its neighbors whatever its index;
//   k_pair_half     one thread per particle walks its half row: F_i += f_ij in registers, F_j -= f_ij through
//                   float atomics in L2, then F_i is added atomically as well (other particles scatter into it).
//
// Every pair is evaluated once instead of twice, at the price of three atomics per pair and of a summation
// order that varies between runs (the last bits of the forces are not reproducible).  The full-list pass
// needs no atomics and is deterministic.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

template <int W>
__global__ __launch_bounds__(kBlock) void k_half_compact(const int32_t *__restrict__ idx,
                                                         const int32_t *__restrict__ count, int N, int capW,
                                                         int32_t *__restrict__ hidx, int32_t *__restrict__ hcount,
                                                         int hcap, int32_t *overflow)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    int m = 0;
#pragma unroll
    for (int l = 0; l < W; ++l) {
        int n = min(count[(size_t)i * W + l], capW);
        for (int t = 0; t < n; ++t) {
            int j = idx[((size_t)t * N + i) * W + l];
            if ((i < j) != (((i + j) & 1) != 0)) {
                if (m < hcap) hidx[(size_t)m * N + i] = j;
                ++m;
            }
        }
    }
    hcount[i] = m;
    if (m > hcap) overflow[0] = 1;
}

__global__ __launch_bounds__(kBlock) void k_zero_f(float *f, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBlock) f[q] = 0.0f;
}

template <int D, int KIND, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_pair_half(DevBox b, DevPot p, const uint32_t *__restrict__ pos,
                                                      const int32_t *__restrict__ species, int N,
                                                      const int32_t *__restrict__ hidx,
                                                      const int32_t *__restrict__ hcount, int hcap, float *force)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t ui[D];
    load_pos<D>(pos, i, ui);
    int si = MULTI ? species[i] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    int n = min(hcount[i], hcap);
    for (int t = 0; t < n; ++t) {
        int j = hidx[(size_t)t * N + i];
        uint32_t uj[D];
        load_pos<D>(pos, j, uj);
        float d[D], r2, u = 0.0f;
        int pt = MULTI ? si * p.S + species[j] : 0;
        float fs = pair_eval<D, KIND, MULTI, false>(p, pt, ui, uj, b.s, b.sd, d, r2, u);
        if (fs != 0.0f) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                F[q] = __builtin_fmaf(fs, d[q], F[q]);
                atomicAdd(&force[(size_t)j * D + q], -fs * d[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < D; ++q) atomicAdd(&force[(size_t)i * D + q], F[q]);
}

int nb(int64_t n)
{
    return (int)((n + kBlock - 1) / kBlock);
}

}  // namespace

extern "C" {

md_status nl_half(md_ctx *ctx, const md_nlist *nl, int32_t *hidx, int32_t *hcount, int32_t hcap, int32_t *overflow,
                  void *stream)
{
    if (!ctx || !nl || !nl->idx || !nl->count || !hidx || !hcount || !overflow || hcap < 1 || nl->N < 0 ||
        nl->segment != 0)
        return MD_ERR_ARG;
    int W = nl->lanes;
    if (W != 1 && W != 2 && W != 4 && W != 8) return MD_ERR_ARG;
    if ((int64_t)hcap * nl->N >= ((int64_t)1 << 31)) return MD_ERR_CAPACITY;
    if (nl->N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    int capW = nl->capacity / W;
    switch (W) {
    case 1: hipLaunchKernelGGL(k_half_compact<1>, dim3(nb(nl->N)), dim3(kBlock), 0, s, nl->idx, nl->count, nl->N, capW,
                               hidx, hcount, hcap, overflow); break;
    case 2: hipLaunchKernelGGL(k_half_compact<2>, dim3(nb(nl->N)), dim3(kBlock), 0, s, nl->idx, nl->count, nl->N, capW,
                               hidx, hcount, hcap, overflow); break;
    case 4: hipLaunchKernelGGL(k_half_compact<4>, dim3(nb(nl->N)), dim3(kBlock), 0, s, nl->idx, nl->count, nl->N, capW,
                               hidx, hcount, hcap, overflow); break;
    default: hipLaunchKernelGGL(k_half_compact<8>, dim3(nb(nl->N)), dim3(kBlock), 0, s, nl->idx, nl->count, nl->N,
                                capW, hidx, hcount, hcap, overflow); break;
    }
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status pair_force_half(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                          const int32_t *species, int32_t N, const int32_t *hidx, const int32_t *hcount, int32_t hcap,
                          float *force, void *stream)
{
    if (!ctx || !box || (box->dim != 2 && box->dim != 3) || !pos || !hidx || !hcount || !force || N < 0 || hcap < 1)
        return MD_ERR_ARG;
    DevPot p;
    if (!md_make_pot(pot, p)) return MD_ERR_ARG;
    bool multi = pot->n_species > 1;
    if (multi && !species) return MD_ERR_ARG;
    DevBox b{};
    for (int k = 0; k < box->dim; ++k) {
        float L = box->L[k];
        if (!(L > 0.0f) || !isfinite(L) || !(md_max_cutoff(pot) < 0.5f * L)) return MD_ERR_BOX;
        b.s[k] = L / 4294967296.0f;
        b.inv_s[k] = 4294967296.0f / L;
        b.sd[k] = (double)L / 4294967296.0;
    }
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    int64_t nf = (int64_t)N * box->dim;
    hipLaunchKernelGGL(k_zero_f, dim3(nb(nf) < 4096 ? nb(nf) : 4096), dim3(kBlock), 0, s, force, nf);
#define HALF(D_, K_, M_) \
    hipLaunchKernelGGL((k_pair_half<D_, K_, M_>), dim3(nb(N)), dim3(kBlock), 0, s, b, p, pos, species, N, hidx, hcount, \
                       hcap, force)
    const int K = pot->kind;
    if (box->dim == 3) {
        if (K == MD_LJ) { if (multi) HALF(3, 0, true); else HALF(3, 0, false); }
        else if (K == MD_MORSE) { if (multi) HALF(3, 2, true); else HALF(3, 2, false); }
        else if (K == MD_BUCKINGHAM) { if (multi) HALF(3, 3, true); else HALF(3, 3, false); }
        else { if (multi) HALF(3, 1, true); else HALF(3, 1, false); }
    } else {
        if (K == MD_LJ) { if (multi) HALF(2, 0, true); else HALF(2, 0, false); }
        else if (K == MD_MORSE) { if (multi) HALF(2, 2, true); else HALF(2, 2, false); }
        else if (K == MD_BUCKINGHAM) { if (multi) HALF(2, 3, true); else HALF(2, 3, false); }
        else { if (multi) HALF(2, 1, true); else HALF(2, 1, false); }
    }
#undef HALF
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
