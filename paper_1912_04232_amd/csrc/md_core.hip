// gfx950 kernels of the short-range MD path and the C ABI that launches them.
//
//   cell list      counting sort of particles by cell (Sec. 3.2.3): integer
//                  counts, an atomics-free exclusive scan in LDS, placement,
//                  then each cell's members ordered by index so every build
//                  is deterministic.
//   neighbor list  27 (3D) / 9 (2D) stencil cells per particle, float filter
//                  with a guard band, double recheck near r_list; ELL rows.
//   forces         one lane per particle i walks its ELL row; neighbor
//                  positions are gathered as packed uint32 torus coordinates
//                  whose integer difference is the nearest image (Sec. 3.2.1).
//   velocity Verlet / FIRE  one cooperative launch per step; the neighbor list
//                  is rebuilt inside that launch, behind grid barriers, when
//                  the previous step flagged a particle that moved more than
//                  skin/2 (Sec. 3.1), so no host round trip is needed.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <unordered_map>

#include "../../include/md.h"
#include "md_device.h"

namespace cg = cooperative_groups;
using namespace md;

// ------------------------------------------------------------------------------------------------
// argument blocks

struct CellScratch {
    int32_t *cell_of;
    int32_t *slot;
    int32_t *sorted_idx;
    uint32_t *pos_sorted;
    int32_t *cell_count;
    int32_t *cell_start;
};

struct NLView {
    int32_t N, cap;
    float rl2f_lo, rl2f_hi;  // float guard band around r_list^2
    double rl2;              // (double)r_list * (double)r_list
    float half_skin2;        // (skin/2)^2
    int32_t *idx;
    int32_t *count;
    uint32_t *pos_ref;
    int32_t *flags;
};

struct StepArgs {
    DevBox box;
    CellScratch cs;
    NLView nl;
    const uint32_t *pos_in;
    uint32_t *pos_out;
    float *vel;
    float *force;
    const int32_t *species;
    int32_t N;
    float dt;
    int32_t step;      // step index s >= 1
    int32_t rot_read, rot_set, rot_clear;
    int32_t mode;      // 1 = interior step (kick dt, drift), 2 = last step (kick dt/2, store F)
    int32_t force_rebuild;
};

// ------------------------------------------------------------------------------------------------
// cell list and neighbor list phases; (tid, nth) is a grid-stride range

__device__ void phase_zero_counts(const CellScratch &cs, int C, int tid, int nth)
{
    for (int c = tid; c < C; c += nth) cs.cell_count[c] = 0;
}

template <int D>
__device__ void phase_bin(const uint32_t *__restrict__ pos, int N, const DevBox &b, const CellScratch &cs, int tid,
                          int nth)
{
    for (int i = tid; i < N; i += nth) {
        uint32_t u[D];
        load_pos<D>(pos, i, u);
        int c = cell_index<D>(u, b);
        cs.cell_of[i] = c;
        cs.slot[i] = atomicAdd(&cs.cell_count[c], 1);  // integer counts: order-free result
    }
}

// Exclusive scan of cell_count into cell_start[0..C], run by one workgroup.
__device__ void phase_scan_block(const CellScratch &cs, int C)
{
    __shared__ int lds[kBlock];
    int t = threadIdx.x;
    int chunk = (C + kBlock - 1) / kBlock;
    int lo = min(C, t * chunk), hi = min(C, lo + chunk);
    int local = 0;
    for (int c = lo; c < hi; ++c) local += cs.cell_count[c];
    int total;
    int run = block_exclusive_scan(local, lds, total);
    for (int c = lo; c < hi; ++c) {
        cs.cell_start[c] = run;
        run += cs.cell_count[c];
    }
    if (t == 0) cs.cell_start[C] = total;
}

__device__ void phase_place(const CellScratch &cs, int N, int tid, int nth)
{
    for (int i = tid; i < N; i += nth) cs.sorted_idx[cs.cell_start[cs.cell_of[i]] + cs.slot[i]] = i;
}

// Order each cell's members by particle index and gather their positions in that order.
template <int D>
__device__ void phase_sort_cells(const uint32_t *__restrict__ pos, const CellScratch &cs, int C, int tid, int nth)
{
    for (int c = tid; c < C; c += nth) {
        int s = cs.cell_start[c], e = cs.cell_start[c + 1];
        for (int a = s + 1; a < e; ++a) {
            int key = cs.sorted_idx[a];
            int b = a - 1;
            while (b >= s && cs.sorted_idx[b] > key) {
                cs.sorted_idx[b + 1] = cs.sorted_idx[b];
                --b;
            }
            cs.sorted_idx[b + 1] = key;
        }
        for (int a = s; a < e; ++a) {
            uint32_t u[D];
            load_pos<D>(pos, cs.sorted_idx[a], u);
            store_pos<D>(cs.pos_sorted, a, u);
        }
    }
}

__device__ __forceinline__ int wrapc(int c, int n)
{
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

// One ELL row per particle.  Returns the largest row length this thread saw.
template <int D>
__device__ int phase_build(const uint32_t *__restrict__ pos, int N, const DevBox &b, const CellScratch &cs,
                           const NLView &nl, int tid, int nth)
{
    int mymax = 0;
    for (int i = tid; i < N; i += nth) {
        uint32_t ui[D];
        load_pos<D>(pos, i, ui);
        int cx = cell_coord(ui[0], b.nc[0]);
        int cy = cell_coord(ui[1], b.nc[1]);
        int cz = 0;
        if constexpr (D == 3) cz = cell_coord(ui[2], b.nc[2]);
        int n = 0;
        int zlo = D == 3 ? b.lo[2] : 0, zhi = D == 3 ? b.hi[2] : 0;
        for (int oz = zlo; oz <= zhi; ++oz) {
            int z = D == 3 ? wrapc(cz + oz, b.nc[2]) : 0;
            for (int oy = b.lo[1]; oy <= b.hi[1]; ++oy) {
                int y = wrapc(cy + oy, b.nc[1]);
                for (int ox = b.lo[0]; ox <= b.hi[0]; ++ox) {
                    int x = wrapc(cx + ox, b.nc[0]);
                    int cell = x + b.nc[0] * (y + b.nc[1] * z);
                    int s = cs.cell_start[cell], e = cs.cell_start[cell + 1];
                    for (int k = s; k < e; ++k) {
                        uint32_t uj[D];
                        load_pos<D>(cs.pos_sorted, k, uj);
                        float r2 = 0.0f;
#pragma unroll
                        for (int q = 0; q < D; ++q) {
                            float d = tdisp(ui[q], uj[q], b.s[q]);
                            r2 = __builtin_fmaf(d, d, r2);
                        }
                        bool acc;
                        if (r2 < nl.rl2f_lo) {
                            acc = true;
                        } else if (r2 > nl.rl2f_hi) {
                            acc = false;
                        } else {
                            // the defining double expression, no contraction
                            double r2d = 0.0;
#pragma unroll
                            for (int q = 0; q < D; ++q) {
                                double d = tdisp_d(ui[q], uj[q], b.sd[q]);
                                r2d = __dadd_rn(r2d, __dmul_rn(d, d));
                            }
                            acc = r2d < nl.rl2;
                        }
                        int j = cs.sorted_idx[k];
                        if (acc && j != i) {
                            if (n < nl.cap) nl.idx[(size_t)n * N + i] = j;
                            ++n;
                        }
                    }
                }
            }
        }
        nl.count[i] = n;
        if (n > nl.cap) nl.flags[MD_FLAG_OVERFLOW] = 1;
        mymax = max(mymax, n);
        store_pos<D>(nl.pos_ref, i, ui);
    }
    return mymax;
}

__device__ __forceinline__ int32_t load_flag(int32_t *flags, int w)
{
    return __hip_atomic_load(&flags[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Full rebuild inside a cooperative launch.  Every workgroup must call it.
template <int D>
__device__ void rebuild_coop(cg::grid_group &g, const uint32_t *pos, int N, const DevBox &b, const CellScratch &cs,
                             const NLView &nl, int tid, int nth)
{
    __shared__ int red[kBlock];
    phase_zero_counts(cs, b.C, tid, nth);
    g.sync();
    phase_bin<D>(pos, N, b, cs, tid, nth);
    g.sync();
    if (blockIdx.x == 0) phase_scan_block(cs, b.C);
    g.sync();
    phase_place(cs, N, tid, nth);
    g.sync();
    phase_sort_cells<D>(pos, cs, b.C, tid, nth);
    g.sync();
    int m = phase_build<D>(pos, N, b, cs, nl, tid, nth);
    m = block_max(m, red);
    if (threadIdx.x == 0) {
        atomicMax(&nl.flags[MD_FLAG_MAXCOUNT], m);
        if (blockIdx.x == 0) nl.flags[MD_FLAG_REBUILDS] += 1;
    }
    g.sync();
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_nl_build(DevBox b, CellScratch cs, NLView nl, const uint32_t *pos, int N)
{
    cg::grid_group g = cg::this_grid();
    int tid = blockIdx.x * kBlock + threadIdx.x, nth = gridDim.x * kBlock;
    rebuild_coop<D>(g, pos, N, b, cs, nl, tid, nth);
}

// ------------------------------------------------------------------------------------------------
// forces over the neighbor list / all pairs

template <int D, int KIND, bool MULTI, bool WANT_EW>
__global__ __launch_bounds__(kBlock) void k_pair_nl(DevBox b, DevPot p, const uint32_t *__restrict__ pos,
                                                     const int32_t *__restrict__ species, int N,
                                                     const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ count, int cap,
                                                     float *__restrict__ force,
                                                     double *__restrict__ energy, double *__restrict__ virial,
                                                     int32_t *flags)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t ui[D];
    load_pos<D>(pos, i, ui);
    int si = MULTI ? species[i] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    double e = 0.0, w = 0.0;
    int n = min(count[i], cap);  // an overflowed row holds only its first cap entries
    for (int k = 0; k < n; ++k) {
        int j = idx[(size_t)k * N + i];
        uint32_t uj[D];
        load_pos<D>(pos, j, uj);
        float d[D], r2 = 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            d[q] = tdisp(ui[q], uj[q], b.s[q]);
            r2 = __builtin_fmaf(d[q], d[q], r2);
        }
        int pt = MULTI ? si * p.S + species[j] : 0;
        float u = 0.0f;
        float fs = pair_fs<KIND, MULTI, WANT_EW>(p, pt, r2, u);
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
        if (WANT_EW) {
            e += (double)u;
            w += (double)(fs * r2);
        }
    }
    bool fin = true;
#pragma unroll
    for (int q = 0; q < D; ++q) fin = fin && isfinite(F[q]);
    if (!fin) flags[MD_FLAG_NONFINITE] = 1;
    if (force) {
#pragma unroll
        for (int q = 0; q < D; ++q) force[(size_t)i * D + q] = F[q];
    }
    if (WANT_EW) {
        if (energy) energy[i] = 0.5 * e;
        if (virial) virial[i] = 0.5 * w;
    }
}

// Dense O(N^2): each workgroup owns kBlock particles i and streams every j through LDS.
template <int D, int KIND, bool MULTI, bool WANT_EW>
__global__ __launch_bounds__(kBlock) void k_pair_dense(DevBox b, DevPot p, const uint32_t *__restrict__ pos,
                                                        const int32_t *__restrict__ species, int N,
                                                        float *__restrict__ force, double *__restrict__ energy,
                                                        double *__restrict__ virial, int32_t *flags)
{
    __shared__ uint32_t tile[kBlock * D];
    __shared__ int32_t tsp[kBlock];
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool live = i < N;
    uint32_t ui[D];
#pragma unroll
    for (int q = 0; q < D; ++q) ui[q] = live ? pos[(size_t)i * D + q] : 0u;
    int si = (MULTI && live) ? species[i] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    double e = 0.0, w = 0.0;
    for (int j0 = 0; j0 < N; j0 += kBlock) {
        int jl = j0 + threadIdx.x;
        if (jl < N) {
#pragma unroll
            for (int q = 0; q < D; ++q) tile[threadIdx.x * D + q] = pos[(size_t)jl * D + q];
            if (MULTI) tsp[threadIdx.x] = species[jl];
        }
        __syncthreads();
        int jn = min(kBlock, N - j0);
        if (live) {
            for (int jj = 0; jj < jn; ++jj) {
                if (j0 + jj == i) continue;
                float d[D], r2 = 0.0f;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    d[q] = tdisp(ui[q], tile[jj * D + q], b.s[q]);
                    r2 = __builtin_fmaf(d[q], d[q], r2);
                }
                int pt = MULTI ? si * p.S + tsp[jj] : 0;
                float u = 0.0f;
                float fs = pair_fs<KIND, MULTI, WANT_EW>(p, pt, r2, u);
#pragma unroll
                for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
                if (WANT_EW) {
                    e += (double)u;
                    w += (double)(fs * r2);
                }
            }
        }
        __syncthreads();
    }
    if (!live) return;
    bool fin = true;
#pragma unroll
    for (int q = 0; q < D; ++q) fin = fin && isfinite(F[q]);
    if (!fin) flags[MD_FLAG_NONFINITE] = 1;
    if (force) {
#pragma unroll
        for (int q = 0; q < D; ++q) force[(size_t)i * D + q] = F[q];
    }
    if (WANT_EW) {
        if (energy) energy[i] = 0.5 * e;
        if (virial) virial[i] = 0.5 * w;
    }
}

// ------------------------------------------------------------------------------------------------
// velocity Verlet

// Force on particle i from its ELL row (the hot loop of every step).
template <int D, int KIND, bool MULTI>
__device__ __forceinline__ void row_force(const DevBox &b, const DevPot &p, const uint32_t *__restrict__ pos,
                                          const int32_t *__restrict__ species, int N,
                                          const int32_t *__restrict__ idx, int n, int i, const uint32_t *ui, int si,
                                          float *F)
{
    int k = 0;
    for (; k + 4 <= n; k += 4) {
        int j[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) j[t] = idx[(size_t)(k + t) * N + i];
        uint32_t uj[4][D];
#pragma unroll
        for (int t = 0; t < 4; ++t) load_pos<D>(pos, j[t], uj[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float d[D], r2 = 0.0f;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                d[q] = tdisp(ui[q], uj[t][q], b.s[q]);
                r2 = __builtin_fmaf(d[q], d[q], r2);
            }
            int pt = MULTI ? si * p.S + species[j[t]] : 0;
            float u;
            float fs = pair_fs<KIND, MULTI, false>(p, pt, r2, u);
#pragma unroll
            for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
        }
    }
    for (; k < n; ++k) {
        int j = idx[(size_t)k * N + i];
        uint32_t uj[D];
        load_pos<D>(pos, j, uj);
        float d[D], r2 = 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            d[q] = tdisp(ui[q], uj[q], b.s[q]);
            r2 = __builtin_fmaf(d[q], d[q], r2);
        }
        int pt = MULTI ? si * p.S + species[j] : 0;
        float u;
        float fs = pair_fs<KIND, MULTI, false>(p, pt, r2, u);
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
    }
}

// Shift (Sec. 3.2.1) by a real displacement: add its nearest integer number of 2^-32 L units; wraps mod 2^32.
__device__ __forceinline__ uint32_t shift_coord(uint32_t u, float dx, float inv_s)
{
    return u + (uint32_t)__float2int_rn(dx * inv_s);
}

template <int D>
__device__ __forceinline__ bool moved_too_far(const uint32_t *un, const uint32_t *__restrict__ ref, int i,
                                              const DevBox &b, float half_skin2)
{
    float r2 = 0.0f;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        float d = tdisp(un[q], ref[(size_t)i * D + q], b.s[q]);
        r2 = __builtin_fmaf(d, d, r2);
    }
    return r2 > half_skin2;
}

// First half kick and drift: v += dt/2 F; r += dt v.  Flags a rebuild for step 1.
template <int D>
__global__ __launch_bounds__(kBlock) void k_verlet_begin(DevBox b, const uint32_t *__restrict__ pos_in,
                                                          uint32_t *__restrict__ pos_out, float *__restrict__ vel,
                                                          const float *__restrict__ force, const uint32_t *pos_ref,
                                                          int N, float dt, float half_skin2, int32_t *flags,
                                                          int rot_set)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t un[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        float v = __builtin_fmaf(0.5f * dt, force[(size_t)i * D + q], vel[(size_t)i * D + q]);
        vel[(size_t)i * D + q] = v;
        un[q] = shift_coord(pos_in[(size_t)i * D + q], dt * v, b.inv_s[q]);
        pos_out[(size_t)i * D + q] = un[q];
    }
    if (moved_too_far<D>(un, pos_ref, i, b, half_skin2)) flags[MD_FLAG_PENDING0 + rot_set] = 1;
}

// Block index remapped so that the workgroups an XCD receives (round-robin over 8 XCDs) own one
// contiguous range of particles: neighbor gathers then mostly hit that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    if ((nb & 7) != 0) return bid;
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

// One velocity-Verlet step s >= 1 on positions r(s): (rebuild if flagged), F(s),
// then v += dt F (interior: completes step s-1 and opens step s) and r(s+1) = r(s) + dt v,
// or v += dt/2 F and store F (last step).
template <int D, int KIND, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_verlet_step(StepArgs a, DevPot p)
{
    cg::grid_group g = cg::this_grid();
    int tid = blockIdx.x * kBlock + threadIdx.x, nth = gridDim.x * kBlock;
    int32_t *flags = a.nl.flags;
    if (flags[MD_FLAG_OVERFLOW]) return;  // written before this launch: same value in every workgroup
    if (a.force_rebuild || flags[MD_FLAG_PENDING0 + a.rot_read]) {
        rebuild_coop<D>(g, a.pos_in, a.N, a.box, a.cs, a.nl, tid, nth);
        if (load_flag(flags, MD_FLAG_OVERFLOW)) return;  // read after the barrier: same value everywhere
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flags[MD_FLAG_PENDING0 + a.rot_clear] = 0;
        flags[MD_FLAG_STEPS] = a.step;
    }
    int lb = xcd_block(blockIdx.x, gridDim.x);
    int per = (a.N + gridDim.x - 1) / gridDim.x;
    per = (per + kBlock - 1) / kBlock * kBlock;
    int i0 = lb * per, i1 = min(a.N, i0 + per);
    bool far = false, bad = false;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        uint32_t ui[D];
        load_pos<D>(a.pos_in, i, ui);
        int si = MULTI ? a.species[i] : 0;
        float F[D];
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = 0.0f;
        row_force<D, KIND, MULTI>(a.box, p, a.pos_in, a.species, a.N, a.nl.idx, min(a.nl.count[i], a.nl.cap), i, ui, si,
                                  F);
#pragma unroll
        for (int q = 0; q < D; ++q) bad = bad || !isfinite(F[q]);
        if (a.mode == 2) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                float v = __builtin_fmaf(0.5f * a.dt, F[q], a.vel[(size_t)i * D + q]);
                a.vel[(size_t)i * D + q] = v;
                a.force[(size_t)i * D + q] = F[q];
            }
        } else {
            uint32_t un[D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                float v = __builtin_fmaf(a.dt, F[q], a.vel[(size_t)i * D + q]);
                a.vel[(size_t)i * D + q] = v;
                un[q] = shift_coord(ui[q], a.dt * v, a.box.inv_s[q]);
            }
            store_pos<D>(a.pos_out, i, un);
            far = far || moved_too_far<D>(un, a.nl.pos_ref, i, a.box, a.nl.half_skin2);
        }
    }
    (void)tid;
    (void)nth;
    if (far) flags[MD_FLAG_PENDING0 + a.rot_set] = 1;
    if (bad) flags[MD_FLAG_NONFINITE] = 1;
}

// ------------------------------------------------------------------------------------------------
// FIRE

struct FireArgs {
    DevBox box;
    CellScratch cs;
    NLView nl;
    uint32_t *pos;
    float *vel;
    float *force;
    const int32_t *species;
    int32_t N;
    md_fire_state *st;
    double *partials;   // [4 * gridDim.x]
    double f_tol;
    float dt_max, f_inc, f_dec, alpha_start, f_alpha;
    int32_t n_min;
    int32_t init;       // 1: no drift/mix, forces only (fire_init)
};

template <int D, int KIND, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_fire_step(FireArgs a, DevPot p)
{
    cg::grid_group g = cg::this_grid();
    __shared__ double red[kBlock];
    int tid = blockIdx.x * kBlock + threadIdx.x, nth = gridDim.x * kBlock;
    int32_t *flags = a.nl.flags;
    md_fire_state *st = a.st;
    if (flags[MD_FLAG_OVERFLOW] || st->converged) return;  // values from before this launch
    int lb = xcd_block(blockIdx.x, gridDim.x);
    int per = (a.N + gridDim.x - 1) / gridDim.x;
    per = (per + kBlock - 1) / kBlock * kBlock;
    int i0 = lb * per, i1 = min(a.N, i0 + per);
    double dt = st->dt;
    if (!a.init) {
        // mixing decided by the previous step, then r += dt v + dt^2/2 F
        double mv = st->mix_v, mf = st->mix_f;
        bool far = false;
        for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
            uint32_t un[D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                float f = a.force[(size_t)i * D + q];
                float v = (float)(mv * (double)a.vel[(size_t)i * D + q] + mf * (double)f);
                a.vel[(size_t)i * D + q] = v;
                float dx = (float)(dt * (double)v + 0.5 * dt * dt * (double)f);
                un[q] = shift_coord(a.pos[(size_t)i * D + q], dx, a.box.inv_s[q]);
            }
            store_pos<D>(a.pos, i, un);
            far = far || moved_too_far<D>(un, a.nl.pos_ref, i, a.box, a.nl.half_skin2);
        }
        if (far) flags[MD_FLAG_PENDING0] = 1;
        g.sync();
        if (load_flag(flags, MD_FLAG_PENDING0)) {
            rebuild_coop<D>(g, a.pos, a.N, a.box, a.cs, a.nl, tid, nth);
            if (load_flag(flags, MD_FLAG_OVERFLOW)) return;
        }
    }
    // F' = F(r); v += dt/2 (F + F'); partial sums of F.v, v.v, F.F and max |F_i|^2
    double P = 0.0, vv = 0.0, ff = 0.0, fm = 0.0;
    bool bad = false;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        uint32_t ui[D];
        load_pos<D>(a.pos, i, ui);
        int si = MULTI ? a.species[i] : 0;
        float F[D];
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = 0.0f;
        row_force<D, KIND, MULTI>(a.box, p, a.pos, a.species, a.N, a.nl.idx, min(a.nl.count[i], a.nl.cap), i, ui, si,
                                  F);
        double fi2 = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            bad = bad || !isfinite(F[q]);
            float v = a.init ? 0.0f : (float)((double)a.vel[(size_t)i * D + q] +
                                              0.5 * dt * ((double)a.force[(size_t)i * D + q] + (double)F[q]));
            a.vel[(size_t)i * D + q] = v;
            a.force[(size_t)i * D + q] = F[q];
            P += (double)F[q] * (double)v;
            vv += (double)v * (double)v;
            fi2 += (double)F[q] * (double)F[q];
        }
        ff += fi2;
        fm = fmax(fm, fi2);
    }
    if (bad) flags[MD_FLAG_NONFINITE] = 1;
    P = block_sum(P, red);
    vv = block_sum(vv, red);
    ff = block_sum(ff, red);
    fm = block_max(fm, red);
    if (threadIdx.x == 0) {
        a.partials[4 * blockIdx.x + 0] = P;
        a.partials[4 * blockIdx.x + 1] = vv;
        a.partials[4 * blockIdx.x + 2] = ff;
        a.partials[4 * blockIdx.x + 3] = fm;
    }
    g.sync();
    if (blockIdx.x != 0) return;
    // workgroup 0: global sums in a fixed order, convergence test, FIRE rules
    double sP = 0.0, svv = 0.0, sff = 0.0, sfm = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
        sP += a.partials[4 * b + 0];
        svv += a.partials[4 * b + 1];
        sff += a.partials[4 * b + 2];
        sfm = fmax(sfm, a.partials[4 * b + 3]);
    }
    sP = block_sum(sP, red);
    svv = block_sum(svv, red);
    sff = block_sum(sff, red);
    sfm = block_max(sfm, red);
    if (threadIdx.x != 0) return;
    flags[MD_FLAG_PENDING0] = 0;
    st->fmax = sqrt(sfm);
    st->power = sP;
    if (!a.init) st->steps += 1;
    flags[MD_FLAG_STEPS] = (int32_t)st->steps;
    if (st->fmax < a.f_tol) {
        st->converged = 1;
        return;
    }
    if (a.init) {
        st->mix_v = 1.0;
        st->mix_f = 0.0;
        return;
    }
    double al = st->alpha;
    double fn = sqrt(sff), vn = sqrt(svv);
    if (sP > 0.0) {
        st->mix_v = 1.0 - al;
        st->mix_f = fn > 0.0 ? al * vn / fn : 0.0;
        st->n_pos += 1;
        if (st->n_pos > a.n_min) {
            st->dt = fmin(st->dt * (double)a.f_inc, (double)a.dt_max);
            st->alpha = al * (double)a.f_alpha;
        }
    } else {
        st->mix_v = 0.0;
        st->mix_f = 0.0;
        st->dt = st->dt * (double)a.f_dec;
        st->alpha = (double)a.alpha_start;
        st->n_pos = 0;
    }
}

// ------------------------------------------------------------------------------------------------
// small kernels: conversions, reductions, flags

__global__ void k_from_float(int n, int D, float L0, float L1, float L2, const float *x, uint32_t *u)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    int q = t % D;
    double L = q == 0 ? L0 : (q == 1 ? L1 : L2);
    long long v = llrint((double)x[t] * (4294967296.0 / L));
    u[t] = (uint32_t)(unsigned long long)v;
}

__global__ void k_to_float(int n, int D, double s0, double s1, double s2, const uint32_t *u, float *x)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    int q = t % D;
    double s = q == 0 ? s0 : (q == 1 ? s1 : s2);
    x[t] = (float)((double)u[t] * s);
}

__global__ void k_copy_u32(int n, const uint32_t *a, uint32_t *b)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) b[t] = a[t];
}

__global__ void k_fill_i32(int n, int32_t *a, int32_t v)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) a[t] = v;
}

__global__ void k_zero_pending(int32_t *flags)
{
    if (threadIdx.x < 3) flags[MD_FLAG_PENDING0 + threadIdx.x] = 0;
}

constexpr int kRedBlocks = 256;

__global__ __launch_bounds__(kBlock) void k_sum_partial(const double *x, int64_t n, double *partials)
{
    __shared__ double red[kBlock];
    int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kBlock) s += x[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_ke_partial(const float *v, int64_t n, double *partials)
{
    __shared__ double red[kBlock];
    int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kBlock) s += (double)v[q] * (double)v[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.5 * s;
}

__global__ __launch_bounds__(kBlock) void k_sum_final(const double *partials, int n, double *out)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += kBlock) s += partials[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

// ------------------------------------------------------------------------------------------------
// host side: context, argument checks, dispatch

struct md_ctx {
    int device = 0;
    int num_cu = 0;
    int32_t N_cap = 0, dim_cap = 0, C_cap = 0;
    uint32_t *pos_alt = nullptr;
    uint32_t *pos_sorted = nullptr;
    int32_t *cell_of = nullptr, *slot = nullptr, *sorted_idx = nullptr;
    int32_t *cell_count = nullptr, *cell_start = nullptr;
    double *partials = nullptr;  // 4 * kMaxCoopBlocks doubles
    int32_t *own_flags = nullptr;  // MD_NFLAGS words for calls made without a neighbor list
    std::unordered_map<const void *, int> coop_blocks;
};

static constexpr int kMaxCoopBlocks = 4096;

#define HIP_OK(x)                                    \
    do {                                             \
        if ((x) != hipSuccess) return MD_ERR_HIP;    \
    } while (0)

static bool make_box(const md_box *box, float r_list, DevBox &b)
{
    if (!box || (box->dim != 2 && box->dim != 3)) return false;
    memset(&b, 0, sizeof(b));
    b.C = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < box->dim) {
            float L = box->L[k];
            if (!(L > 0.0f) || !isfinite(L)) return false;
            b.s[k] = L / 4294967296.0f;
            b.inv_s[k] = 4294967296.0f / L;
            b.sd[k] = (double)L / 4294967296.0;
            int nc = 1;
            if (r_list > 0.0f) {
                double side = (double)r_list * (1.0 + 1e-6);
                double m = floor((double)L / side);
                nc = m >= 3.0 ? (int)fmin(m, 1 << 20) : 1;
            }
            b.nc[k] = nc;
            b.lo[k] = nc >= 3 ? -1 : 0;
            b.hi[k] = nc >= 3 ? 1 : 0;
            b.C *= nc;
        } else {
            b.nc[k] = 1;
        }
    }
    return true;
}

static bool make_pot(const md_potential *pot, DevPot &p)
{
    if (!pot || (pot->kind != MD_LJ && pot->kind != MD_SOFT_SPHERE)) return false;
    int S = pot->n_species;
    if (S < 1 || S > kMaxSpecies) return false;
    memset(&p, 0, sizeof(p));
    p.kind = pot->kind;
    p.S = S;
    p.alpha = pot->alpha;
    p.alpha_is_2 = pot->alpha == 2.0f;
    p.rc2 = pot->r_cut * pot->r_cut;
    if (pot->kind == MD_SOFT_SPHERE && !(pot->alpha >= 1.0f)) return false;
    if (pot->kind == MD_LJ && !(pot->r_cut > 0.0f)) return false;
    for (int a = 0; a < S; ++a)
        for (int c = 0; c < S; ++c) {
            int q = a * S + c;
            double s = pot->sigma[q], e = pot->epsilon[q];
            if (!(s > 0.0) || !isfinite(e)) return false;
            double s6 = s * s * s * s * s * s;
            p.a12[q] = (float)(48.0 * e * s6 * s6);
            p.a6[q] = (float)(24.0 * e * s6);
            p.c12[q] = (float)(4.0 * e * s6 * s6);
            p.c6[q] = (float)(4.0 * e * s6);
            double rc = pot->r_cut;
            double sc6 = pow(s / rc, 6.0);
            p.ushift[q] = pot->shift ? (float)(4.0 * e * (sc6 * sc6 - sc6)) : 0.0f;
            p.sig[q] = (float)s;
            p.inv_sig[q] = (float)(1.0 / s);
            p.eps_over_sig[q] = (float)(e / s);
            p.eps_over_alpha[q] = (float)(e / pot->alpha);
        }
    return true;
}

static float max_cutoff(const md_potential *pot)
{
    if (pot->kind == MD_LJ) return pot->r_cut;
    float m = 0.0f;
    for (int q = 0; q < pot->n_species * pot->n_species; ++q) m = fmaxf(m, pot->sigma[q]);
    return m;
}

static bool box_ok(const md_box *box, float r)
{
    for (int k = 0; k < box->dim; ++k)
        if (!(r < 0.5f * box->L[k])) return false;
    return true;
}

static NLView make_view(const md_nlist *nl)
{
    NLView v;
    v.N = nl->N;
    v.cap = nl->capacity;
    float rl2 = nl->r_list * nl->r_list;
    v.rl2f_lo = rl2 * (1.0f - 1e-5f);
    v.rl2f_hi = rl2 * (1.0f + 1e-5f);
    v.rl2 = (double)nl->r_list * (double)nl->r_list;
    float hs = 0.5f * nl->skin;
    v.half_skin2 = hs * hs;
    v.idx = nl->idx;
    v.count = nl->count;
    v.pos_ref = nl->pos_ref;
    v.flags = nl->flags;
    return v;
}

static CellScratch make_cs(md_ctx *ctx)
{
    CellScratch cs;
    cs.cell_of = ctx->cell_of;
    cs.slot = ctx->slot;
    cs.sorted_idx = ctx->sorted_idx;
    cs.pos_sorted = ctx->pos_sorted;
    cs.cell_count = ctx->cell_count;
    cs.cell_start = ctx->cell_start;
    return cs;
}

static int coop_grid(md_ctx *ctx, const void *kernel, int N)
{
    static std::mutex mu;
    int per_cu;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = ctx->coop_blocks.find(kernel);
        if (it == ctx->coop_blocks.end()) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
            ctx->coop_blocks[kernel] = nb;
            per_cu = nb;
        } else {
            per_cu = it->second;
        }
    }
    int maxb = per_cu * ctx->num_cu;
    if (maxb > kMaxCoopBlocks) maxb = kMaxCoopBlocks;
    int want = (N + kBlock - 1) / kBlock;
    if (want < 1) want = 1;
    int g = want < maxb ? want : maxb;
    if (g >= 8) g &= ~7;  // multiple of the XCD count so the remap is a permutation
    return g;
}

static md_status coop_launch(const void *kernel, int grid, void **args, hipStream_t s)
{
    hipError_t e = hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
    return e == hipSuccess ? MD_OK : MD_ERR_HIP;
}

static inline int nblk(int64_t n)
{
    return (int)((n + kBlock - 1) / kBlock);
}

// dispatch over (dim, kind, species) template instances
#define MD_DISPATCH(D_, KIND_, MULTI_, ...)                                  \
    do {                                                                     \
        if (D_ == 3) {                                                       \
            constexpr int D = 3;                                             \
            if (KIND_ == 0) {                                                \
                constexpr int KIND = 0;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }           \
                else { constexpr bool MULTI = false; __VA_ARGS__; }                 \
            } else {                                                         \
                constexpr int KIND = 1;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }           \
                else { constexpr bool MULTI = false; __VA_ARGS__; }                 \
            }                                                                \
        } else {                                                             \
            constexpr int D = 2;                                             \
            if (KIND_ == 0) {                                                \
                constexpr int KIND = 0;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }           \
                else { constexpr bool MULTI = false; __VA_ARGS__; }                 \
            } else {                                                         \
                constexpr int KIND = 1;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }           \
                else { constexpr bool MULTI = false; __VA_ARGS__; }                 \
            }                                                                \
        }                                                                    \
    } while (0)

static bool nl_ok(const md_nlist *nl, int N)
{
    return nl && nl->N == N && nl->capacity >= 1 && nl->idx && nl->count && nl->pos_ref && nl->flags &&
           nl->r_list > 0.0f && nl->skin >= 0.0f;
}

extern "C" {

const char *md_version(void)
{
    return "md-gfx950 0.1";
}

md_status md_ctx_create(int device, md_ctx **out)
{
    if (!out) return MD_ERR_ARG;
    *out = nullptr;
    HIP_OK(hipSetDevice(device));
    md_ctx *c = new md_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MD_ERR_HIP;
    }
    c->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&c->partials, sizeof(double) * 4 * kMaxCoopBlocks) != hipSuccess ||
        hipMalloc(&c->own_flags, sizeof(int32_t) * MD_NFLAGS) != hipSuccess ||
        hipMemset(c->own_flags, 0, sizeof(int32_t) * MD_NFLAGS) != hipSuccess) {
        (void)hipFree(c->partials);
        delete c;
        return MD_ERR_HIP;
    }
    *out = c;
    return MD_OK;
}

static void free_scratch(md_ctx *c)
{
    (void)hipFree(c->pos_alt);
    (void)hipFree(c->pos_sorted);
    (void)hipFree(c->cell_of);
    (void)hipFree(c->slot);
    (void)hipFree(c->sorted_idx);
    (void)hipFree(c->cell_count);
    (void)hipFree(c->cell_start);
    c->pos_alt = c->pos_sorted = nullptr;
    c->cell_of = c->slot = c->sorted_idx = c->cell_count = c->cell_start = nullptr;
}

md_status md_ctx_destroy(md_ctx *ctx)
{
    if (!ctx) return MD_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_scratch(ctx);
    (void)hipFree(ctx->partials);
    (void)hipFree(ctx->own_flags);
    delete ctx;
    return MD_OK;
}

md_status md_ctx_reserve(md_ctx *ctx, int32_t N, int32_t dim, int32_t max_cells)
{
    if (!ctx || N < 0 || (dim != 2 && dim != 3) || max_cells < 1) return MD_ERR_ARG;
    if (N <= ctx->N_cap && dim <= ctx->dim_cap && max_cells <= ctx->C_cap) return MD_OK;
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipDeviceSynchronize());
    int32_t n = N > ctx->N_cap ? N : ctx->N_cap;
    int32_t d = dim > ctx->dim_cap ? dim : ctx->dim_cap;
    int32_t C = max_cells > ctx->C_cap ? max_cells : ctx->C_cap;
    free_scratch(ctx);
    ctx->N_cap = ctx->dim_cap = ctx->C_cap = 0;
    size_t nn = (size_t)(n > 0 ? n : 1);
    HIP_OK(hipMalloc(&ctx->pos_alt, sizeof(uint32_t) * nn * d));
    HIP_OK(hipMalloc(&ctx->pos_sorted, sizeof(uint32_t) * nn * d));
    HIP_OK(hipMalloc(&ctx->cell_of, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->slot, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->sorted_idx, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->cell_count, sizeof(int32_t) * (size_t)C));
    HIP_OK(hipMalloc(&ctx->cell_start, sizeof(int32_t) * ((size_t)C + 1)));
    ctx->N_cap = n;
    ctx->dim_cap = d;
    ctx->C_cap = C;
    return MD_OK;
}

int32_t md_cell_count(const md_box *box, float r_list)
{
    DevBox b;
    if (!make_box(box, r_list, b)) return -1;
    return b.C;
}

md_status md_positions_from_float(const md_box *box, const float *x, uint32_t *pos, int32_t N, void *stream)
{
    DevBox b;
    if (!make_box(box, 0.0f, b) || !x || !pos || N < 0) return MD_ERR_ARG;
    int n = N * box->dim;
    if (n == 0) return MD_OK;
    hipLaunchKernelGGL(k_from_float, dim3(nblk(n)), dim3(kBlock), 0, (hipStream_t)stream, n, box->dim, box->L[0],
                       box->L[1], box->L[2], x, pos);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_positions_to_float(const md_box *box, const uint32_t *pos, float *x, int32_t N, void *stream)
{
    DevBox b;
    if (!make_box(box, 0.0f, b) || !x || !pos || N < 0) return MD_ERR_ARG;
    int n = N * box->dim;
    if (n == 0) return MD_OK;
    hipLaunchKernelGGL(k_to_float, dim3(nblk(n)), dim3(kBlock), 0, (hipStream_t)stream, n, box->dim, b.sd[0],
                       b.sd[1], b.sd[2], pos, x);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

static md_status check_common(md_ctx *ctx, const md_box *box, int32_t N)
{
    if (!ctx || !box || (box->dim != 2 && box->dim != 3) || N < 0) return MD_ERR_ARG;
    if (N > ctx->N_cap || box->dim > ctx->dim_cap) return MD_ERR_CAPACITY;
    return MD_OK;
}

static md_status launch_build(md_ctx *ctx, int dim, const DevBox &b, const uint32_t *pos, int32_t N, md_nlist *nl,
                              hipStream_t s)
{
    CellScratch cs = make_cs(ctx);
    NLView v = make_view(nl);
    void *args[] = {(void *)&b, (void *)&cs, (void *)&v, (void *)&pos, (void *)&N};
    const void *k = dim == 3 ? (const void *)k_nl_build<3> : (const void *)k_nl_build<2>;
    return coop_launch(k, coop_grid(ctx, k, N), args, s);
}

md_status nl_build(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, md_nlist *nl, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!pos || !nl_ok(nl, N)) return MD_ERR_ARG;
    if (!box_ok(box, nl->r_list)) return MD_ERR_BOX;
    DevBox b;
    if (!make_box(box, nl->r_list, b)) return MD_ERR_ARG;
    if (b.C > ctx->C_cap) return MD_ERR_CAPACITY;
    if (N == 0) return MD_OK;
    return launch_build(ctx, box->dim, b, pos, N, nl, (hipStream_t)stream);
}

md_status pair_energy_force(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                            const int32_t *species, int32_t N, const md_nlist *nl, float *force, double *energy,
                            double *virial, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    DevPot p;
    if (!pos || !make_pot(pot, p)) return MD_ERR_ARG;
    bool multi = pot->n_species > 1;
    if (multi && !species) return MD_ERR_ARG;
    if (nl && !nl_ok(nl, N)) return MD_ERR_ARG;
    if (nl && nl->r_list < max_cutoff(pot)) return MD_ERR_ARG;
    if (!box_ok(box, nl ? nl->r_list : max_cutoff(pot))) return MD_ERR_BOX;
    DevBox b;
    if (!make_box(box, 0.0f, b)) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    bool ew = energy || virial;
    // without a list the non-finite flag goes to the context's own flag words
    int32_t *flags = nl ? nl->flags : ctx->own_flags;
    int grid = nblk(N);
    if (nl) {
        if (ew) {
            MD_DISPATCH(box->dim, pot->kind, multi,
                        hipLaunchKernelGGL((k_pair_nl<D, KIND, MULTI, true>), dim3(grid), dim3(kBlock), 0, s, b, p,
                                           pos, species, N, nl->idx, nl->count, nl->capacity, force, energy, virial, flags));
        } else {
            MD_DISPATCH(box->dim, pot->kind, multi,
                        hipLaunchKernelGGL((k_pair_nl<D, KIND, MULTI, false>), dim3(grid), dim3(kBlock), 0, s, b, p,
                                           pos, species, N, nl->idx, nl->count, nl->capacity, force, energy, virial, flags));
        }
    } else {
        if (ew) {
            MD_DISPATCH(box->dim, pot->kind, multi,
                        hipLaunchKernelGGL((k_pair_dense<D, KIND, MULTI, true>), dim3(grid), dim3(kBlock), 0, s, b,
                                           p, pos, species, N, force, energy, virial, flags));
        } else {
            MD_DISPATCH(box->dim, pot->kind, multi,
                        hipLaunchKernelGGL((k_pair_dense<D, KIND, MULTI, false>), dim3(grid), dim3(kBlock), 0, s, b,
                                           p, pos, species, N, force, energy, virial, flags));
        }
    }
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status verlet_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                      float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt, int32_t n_steps,
                      void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    DevPot p;
    if (!pos || !vel || !force || !make_pot(pot, p) || !nl_ok(nl, N) || n_steps < 0 || !isfinite(dt))
        return MD_ERR_ARG;
    bool multi = pot->n_species > 1;
    if (multi && !species) return MD_ERR_ARG;
    if (nl->r_list < max_cutoff(pot)) return MD_ERR_ARG;
    if (!box_ok(box, nl->r_list)) return MD_ERR_BOX;
    DevBox b;
    if (!make_box(box, nl->r_list, b)) return MD_ERR_ARG;
    if (b.C > ctx->C_cap) return MD_ERR_CAPACITY;
    if (N == 0 || n_steps == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    NLView v = make_view(nl);
    hipLaunchKernelGGL(k_zero_pending, dim3(1), dim3(64), 0, s, nl->flags);
    uint32_t *buf[2] = {pos, ctx->pos_alt};
    if (box->dim == 3)
        hipLaunchKernelGGL(k_verlet_begin<3>, dim3(nblk(N)), dim3(kBlock), 0, s, b, buf[0], buf[1], vel, force,
                           nl->pos_ref, N, dt, v.half_skin2, nl->flags, 1);
    else
        hipLaunchKernelGGL(k_verlet_begin<2>, dim3(nblk(N)), dim3(kBlock), 0, s, b, buf[0], buf[1], vel, force,
                           nl->pos_ref, N, dt, v.half_skin2, nl->flags, 1);
    HIP_OK(hipGetLastError());
    StepArgs a;
    a.box = b;
    a.cs = make_cs(ctx);
    a.nl = v;
    a.vel = vel;
    a.force = force;
    a.species = species;
    a.N = N;
    a.dt = dt;
    a.force_rebuild = 0;
    const void *kern = nullptr;
    MD_DISPATCH(box->dim, pot->kind, multi, kern = (const void *)k_verlet_step<D, KIND, MULTI>);
    int grid = coop_grid(ctx, kern, N);
    void *args[] = {(void *)&a, (void *)&p};
    for (int32_t sidx = 1; sidx <= n_steps; ++sidx) {
        a.step = sidx;
        a.pos_in = buf[sidx & 1];
        a.pos_out = buf[(sidx + 1) & 1];
        a.rot_read = sidx % 3;
        a.rot_set = (sidx + 1) % 3;
        a.rot_clear = (sidx + 2) % 3;
        a.mode = sidx == n_steps ? 2 : 1;
        md_status r = coop_launch(kern, grid, args, s);
        if (r != MD_OK) return r;
    }
    if (n_steps & 1) {
        int n = N * box->dim;
        hipLaunchKernelGGL(k_copy_u32, dim3(nblk(n)), dim3(kBlock), 0, s, n, buf[1], buf[0]);
        HIP_OK(hipGetLastError());
    }
    return MD_OK;
}

static md_status fire_launch(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                             float *force, const int32_t *species, int32_t N, md_nlist *nl,
                             const md_fire_params *fp, md_fire_state *fst, int32_t n_steps, double f_tol, int init,
                             hipStream_t s)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    DevPot p;
    if (!pos || !vel || !force || !fst || !fp || !make_pot(pot, p) || !nl_ok(nl, N) || n_steps < 0)
        return MD_ERR_ARG;
    bool multi = pot->n_species > 1;
    if (multi && !species) return MD_ERR_ARG;
    if (nl->r_list < max_cutoff(pot)) return MD_ERR_ARG;
    if (!box_ok(box, nl->r_list)) return MD_ERR_BOX;
    DevBox b;
    if (!make_box(box, nl->r_list, b)) return MD_ERR_ARG;
    if (b.C > ctx->C_cap) return MD_ERR_CAPACITY;
    if (N == 0) return MD_OK;
    FireArgs a;
    a.box = b;
    a.cs = make_cs(ctx);
    a.nl = make_view(nl);
    a.pos = pos;
    a.vel = vel;
    a.force = force;
    a.species = species;
    a.N = N;
    a.st = fst;
    a.partials = ctx->partials;
    a.f_tol = f_tol;
    a.dt_max = fp->dt_max;
    a.f_inc = fp->f_inc;
    a.f_dec = fp->f_dec;
    a.alpha_start = fp->alpha_start;
    a.f_alpha = fp->f_alpha;
    a.n_min = fp->n_min;
    a.init = init;
    const void *kern = nullptr;
    MD_DISPATCH(box->dim, pot->kind, multi, kern = (const void *)k_fire_step<D, KIND, MULTI>);
    int grid = coop_grid(ctx, kern, N);
    void *args[] = {(void *)&a, (void *)&p};
    int n = init ? 1 : n_steps;
    for (int q = 0; q < n; ++q) {
        md_status r = coop_launch(kern, grid, args, s);
        if (r != MD_OK) return r;
    }
    return MD_OK;
}

__global__ void k_fire_state_init(md_fire_state *st, double dt, double alpha, int32_t *flags)
{
    st->dt = dt;
    st->alpha = alpha;
    st->fmax = 0.0;
    st->power = 0.0;
    st->mix_v = 1.0;
    st->mix_f = 0.0;
    st->steps = 0;
    st->n_pos = 0;
    st->converged = 0;
    flags[MD_FLAG_PENDING0] = 0;
}

md_status fire_init(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos, float *vel,
                    float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                    md_fire_state *st, double f_tol, void *stream)
{
    if (!st || !fp || !nl || !nl->flags) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    md_status r = check_common(ctx, box, N);
    if (r != MD_OK) return r;
    hipLaunchKernelGGL(k_fire_state_init, dim3(1), dim3(1), 0, s, st, (double)fp->dt_start, (double)fp->alpha_start,
                       nl->flags);
    HIP_OK(hipGetLastError());
    return fire_launch(ctx, box, pot, (uint32_t *)pos, vel, force, species, N, nl, fp, st, 1, f_tol, 1, s);
}

md_status fire_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                    float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                    md_fire_state *st, int32_t n_steps, double f_tol, void *stream)
{
    return fire_launch(ctx, box, pot, pos, vel, force, species, N, nl, fp, st, n_steps, f_tol, 0,
                       (hipStream_t)stream);
}

md_status md_sum(md_ctx *ctx, const double *x, int64_t n, double *out, void *stream)
{
    if (!ctx || !x || !out || n < 0) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sum_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, x, n, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_kinetic_energy(md_ctx *ctx, const float *vel, int32_t N, int32_t dim, double *out, void *stream)
{
    if (!ctx || !vel || !out || N < 0 || (dim != 2 && dim != 3)) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_ke_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, (int64_t)N * dim, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_flags_read(const md_nlist *nl, int32_t *out, void *stream)
{
    if (!nl || !nl->flags || !out) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(hipMemcpyAsync(out, nl->flags, sizeof(int32_t) * MD_NFLAGS, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return MD_OK;
}

md_status md_flags_clear(md_nlist *nl, void *stream)
{
    if (!nl || !nl->flags) return MD_ERR_ARG;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, (int)MD_NFLAGS, nl->flags, 0);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
