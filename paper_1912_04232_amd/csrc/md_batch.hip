// Batched replicas: many independent periodic 2D systems of uneven size in one launch, FIRE on
// each of them, and the parameter gradient of their energies.
//
// One workgroup of 512 threads owns one replica at a time and takes the next one from a work
// queue when it is done (an integer counter; every workgroup leaves when the queue is empty).
// The replica lives inside the workgroup: positions (uint32 torus coordinates), species and the
// cell list in LDS, velocities and forces in registers (thread t owns particles t, t + 512, ...).
// The cell list is rebuilt in LDS for every force evaluation (LDS counting sort, each cell's
// members ordered by index so sums are deterministic), so there is no skin and no neighbor-list
// bookkeeping; cells have edge >= the interaction range and 9 stencil cells are scanned.
//
//   k_fire_batched   FIRE (Bitzek et al. 2006, the minimizer of Sec. 3.3.1 and App. A) on every
//                    replica until max_i |F_i| < f_tol or max_steps; global sums in double.
//   k_param_grad     dU/dsigma_ab, dU/deps_ab and U at the given positions.  At a converged
//                    minimum this is dE*/dtheta by the envelope theorem, i.e. the derivative of
//                    the minimized energy that Sec. 4.2 obtains by differentiating the minimizer.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

constexpr int kRB = 512;          // threads per replica workgroup of the gradient kernel (FIRE: 512 or 1024)
constexpr int kMaxRepN = 4096;    // particles per replica (kMaxRepN / RB per thread)
constexpr int kMaxRepCells = 3072;
constexpr int kWaves = 1024 / 64;  // LDS slots for the largest workgroup's waves
constexpr int kMaxS = 8;          // species handled by the gradient kernel

struct RepGeom {
    float s[2], inv_s[2];
    double sd[2];
    int nc[2], lo[2], hi[2], C;
};

struct BatchArgs {
    int32_t B;
    const int32_t *offset;  // [B+1]
    const float *box;       // [B][2]
    uint32_t *pos;          // [total][2]
    const int32_t *species; // [total] or null
    int32_t *queue;         // work counter, zeroed before the launch
};

struct Lds {
    uint32_t pos[kMaxRepN * 2];
    int32_t start[kMaxRepCells + 1];  // counts, then exclusive starts
    int16_t sorted[kMaxRepN];
    int8_t spec[kMaxRepN];
    int32_t wtot[kWaves];
    double red[kWaves];
    double red4[4][kWaves];
    int32_t rep;
    DevPot pot;       // pair coefficients, indexed by pair type from LDS (not from kernel arguments)
    md_potential raw; // the caller's parameters, for the gradient kernel
};

__device__ __forceinline__ int wrap2(int c, int n)
{
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

__device__ __forceinline__ RepGeom rep_geom(float Lx, float Ly, float range)
{
    RepGeom g;
    float L[2] = {Lx, Ly};
    g.C = 1;
    for (int k = 0; k < 2; ++k) {
        g.s[k] = L[k] / 4294967296.0f;
        g.inv_s[k] = 4294967296.0f / L[k];
        g.sd[k] = (double)L[k] / 4294967296.0;
        int m = (int)floor((double)L[k] / ((double)range * (1.0 + 1e-6)));
        int nc = m >= 3 ? m : 1;
        g.nc[k] = nc;
        g.lo[k] = nc >= 3 ? -1 : 0;
        g.hi[k] = nc >= 3 ? 1 : 0;
        g.C *= nc;
    }
    return g;
}

__device__ __forceinline__ int rep_cell(const uint32_t *u, const RepGeom &g)
{
    return cell_coord(u[0], g.nc[0]) + g.nc[0] * cell_coord(u[1], g.nc[1]);
}

// Workgroup-wide sum / max of one double per thread; every thread gets the same value.
template <int RB>
__device__ __forceinline__ double wg_sum(double v, Lds &s)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < RB / 64; ++w) r += s.red[w];
    __syncthreads();
    return r;
}

template <int RB>
__device__ __forceinline__ double wg_max(double v, Lds &s)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < RB / 64; ++w) r = fmax(r, s.red[w]);
    __syncthreads();
    return r;
}

// Three sums and one maximum over the workgroup in a single exchange; each is combined in the order wg_sum and
// wg_max use (lanes by the xor tree, then the waves in order), so the results are theirs bit for bit.
template <int RB>
__device__ __forceinline__ void wg_sum3_max(double &a, double &b, double &c, double &m, Lds &s)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
        m = fmax(m, __shfl_xor(m, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s.red4[0][w] = a;
        s.red4[1][w] = b;
        s.red4[2][w] = c;
        s.red4[3][w] = m;
    }
    __syncthreads();
    double ra = 0.0, rb = 0.0, rc = 0.0, rm = 0.0;
    for (int q = 0; q < RB / 64; ++q) {
        ra += s.red4[0][q];
        rb += s.red4[1][q];
        rc += s.red4[2][q];
        rm = fmax(rm, s.red4[3][q]);
    }
    __syncthreads();
    a = ra;
    b = rb;
    c = rc;
    m = rm;
}

// Exclusive scan of one int per thread over the workgroup (shuffles + LDS, no atomics).
template <int RB>
__device__ __forceinline__ int wg_excl_scan(int v, Lds &s, int &total)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s.wtot[w] = incl;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int q = 0; q < RB / 64; ++q) {
        if (q < w) off += s.wtot[q];
        total += s.wtot[q];
    }
    __syncthreads();
    return off + incl - v;
}

// Cell list of the replica's LDS positions: counts (LDS integer atomics), exclusive scan,
// placement, then each cell's members ordered by index.
template <int RB>
__device__ void rep_cells(Lds &s, int n, const RepGeom &g)
{
    constexpr int PT = kMaxRepN / RB;
    int t = threadIdx.x;
    for (int c = t; c < g.C; c += RB) s.start[c] = 0;
    __syncthreads();
    int cell[PT], slot[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        int i = t + k * RB;
        cell[k] = 0;
        slot[k] = 0;
        if (i < n) {
            cell[k] = rep_cell(&s.pos[2 * i], g);
            slot[k] = atomicAdd(&s.start[cell[k]], 1);
        }
    }
    __syncthreads();
    int chunk = (g.C + RB - 1) / RB;
    int lo = min(g.C, t * chunk), hi = min(g.C, lo + chunk);
    int local = 0;
    for (int c = lo; c < hi; ++c) local += s.start[c];
    int total;
    int run = wg_excl_scan<RB>(local, s, total);
    for (int c = lo; c < hi; ++c) {
        int v = s.start[c];
        s.start[c] = run;
        run += v;
    }
    if (t == 0) s.start[g.C] = n;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        int i = t + k * RB;
        if (i < n) s.sorted[s.start[cell[k]] + slot[k]] = (int16_t)i;
    }
    __syncthreads();
    for (int c = t; c < g.C; c += RB) {
        int a0 = s.start[c], a1 = s.start[c + 1];
        for (int a = a0 + 1; a < a1; ++a) {
            int16_t key = s.sorted[a];
            int q = a - 1;
            while (q >= a0 && s.sorted[q] > key) {
                s.sorted[q + 1] = s.sorted[q];
                --q;
            }
            s.sorted[q + 1] = key;
        }
    }
    __syncthreads();
}

// Visit every neighbor j of particle i from the 9 stencil cells: f(j, ui, uj, pair type).
template <typename Fn>
__device__ __forceinline__ void rep_pairs(const Lds &s, const RepGeom &g, int i, int S, Fn &&f)
{
    uint32_t ui[2] = {s.pos[2 * i], s.pos[2 * i + 1]};
    int cx = cell_coord(ui[0], g.nc[0]), cy = cell_coord(ui[1], g.nc[1]);
    int si = s.spec[i];
    for (int oy = g.lo[1]; oy <= g.hi[1]; ++oy) {
        int y = wrap2(cy + oy, g.nc[1]);
        for (int ox = g.lo[0]; ox <= g.hi[0]; ++ox) {
            int c = wrap2(cx + ox, g.nc[0]) + g.nc[0] * y;
            for (int q = s.start[c]; q < s.start[c + 1]; ++q) {
                int j = s.sorted[q];
                if (j == i) continue;
                uint32_t uj[2] = {s.pos[2 * j], s.pos[2 * j + 1]};
                f(j, ui, uj, si * S + s.spec[j]);
            }
        }
    }
}

template <int KIND, int RB>
__device__ __forceinline__ void rep_forces(const Lds &s, const RepGeom &g, const DevPot &p, int n, float (*F)[2])
{
    constexpr int PT = kMaxRepN / RB;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        int i = threadIdx.x + k * RB;
        float fx = 0.0f, fy = 0.0f;
        if (i < n) {
            rep_pairs(s, g, i, p.S, [&](int, const uint32_t *ui, const uint32_t *uj, int pt) {
                float d[2], r2, u;
                float fs = pair_eval<2, KIND, true, false>(p, pt, ui, uj, g.s, g.sd, d, r2, u);
                fx = __builtin_fmaf(fs, d[0], fx);
                fy = __builtin_fmaf(fs, d[1], fy);
            });
        }
        F[k][0] = fx;
        F[k][1] = fy;
    }
}

template <int RB>
__device__ bool rep_load(Lds &s, const BatchArgs &a, int b, float range, int &n, int &off, RepGeom &g)
{
    off = a.offset[b];
    n = a.offset[b + 1] - off;
    g = rep_geom(a.box[2 * b], a.box[2 * b + 1], range);
    if (n < 0 || n > kMaxRepN || g.C > kMaxRepCells) return false;
    for (int i = threadIdx.x; i < n; i += RB) {
        s.pos[2 * i] = a.pos[2 * (size_t)(off + i)];
        s.pos[2 * i + 1] = a.pos[2 * (size_t)(off + i) + 1];
        s.spec[i] = a.species ? (int8_t)a.species[off + i] : (int8_t)0;
    }
    __syncthreads();
    return true;
}

__device__ __forceinline__ int next_replica(Lds &s, int32_t *queue)
{
    __syncthreads();
    if (threadIdx.x == 0) s.rep = atomicAdd(queue, 1);
    __syncthreads();
    return s.rep;
}

struct FireBatchParams {
    double *energy;
    double *fmax;
    int32_t *steps;
    int32_t *status;  // 1 converged, 0 not converged, -1 replica too large for a workgroup
    float dt_start, dt_max, f_inc, f_dec, alpha_start, f_alpha, range;
    int32_t n_min, max_steps;
    double f_tol;
};

template <int KIND, int RB>
__global__ __launch_bounds__(RB) void k_fire_batched(BatchArgs a, DevPot pin, FireBatchParams fp)
{
    constexpr int PT = kMaxRepN / RB;
    __shared__ Lds s;
    if (threadIdx.x == 0) s.pot = pin;
    __syncthreads();
    const DevPot &p = s.pot;
    for (int b = next_replica(s, a.queue); b < a.B; b = next_replica(s, a.queue)) {
        int n, off;
        RepGeom g;
        if (!rep_load<RB>(s, a, b, fp.range, n, off, g)) {
            if (threadIdx.x == 0) fp.status[b] = -1;
            continue;
        }
        float v[PT][2], F[PT][2], Fn[PT][2];
#pragma unroll
        for (int k = 0; k < PT; ++k) v[k][0] = v[k][1] = 0.0f;
        rep_cells<RB>(s, n, g);
        rep_forces<KIND, RB>(s, g, p, n, F);
        double fm = 0.0;
#pragma unroll
        for (int k = 0; k < PT; ++k)
            fm = fmax(fm, (double)F[k][0] * F[k][0] + (double)F[k][1] * F[k][1]);
        fm = wg_max<RB>(fm, s);
        double dt = fp.dt_start, alpha = fp.alpha_start, mix_v = 1.0, mix_f = 0.0;
        int n_pos = 0, steps = 0;
        bool conv = sqrt(fm) < fp.f_tol;
        while (!conv && steps < fp.max_steps) {
            // velocity mixing decided by the previous step, then r += dt v + dt^2/2 F
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                int i = threadIdx.x + k * RB;
                if (i < n) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        v[k][q] = (float)(mix_v * (double)v[k][q] + mix_f * (double)F[k][q]);
                        float dx = (float)(dt * (double)v[k][q] + 0.5 * dt * dt * (double)F[k][q]);
                        s.pos[2 * i + q] += (uint32_t)__float2int_rn(dx * g.inv_s[q]);
                    }
                }
            }
            __syncthreads();
            rep_cells<RB>(s, n, g);
            rep_forces<KIND, RB>(s, g, p, n, Fn);
            double P = 0.0, vv = 0.0, ff = 0.0;
            fm = 0.0;
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                int i = threadIdx.x + k * RB;
                if (i < n) {
                    double f2 = 0.0;
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        v[k][q] = (float)((double)v[k][q] + 0.5 * dt * ((double)F[k][q] + (double)Fn[k][q]));
                        F[k][q] = Fn[k][q];
                        P += (double)F[k][q] * (double)v[k][q];
                        vv += (double)v[k][q] * (double)v[k][q];
                        f2 += (double)F[k][q] * (double)F[k][q];
                    }
                    ff += f2;
                    fm = fmax(fm, f2);
                }
            }
            wg_sum3_max<RB>(P, vv, ff, fm, s);
            ++steps;
            if (sqrt(fm) < fp.f_tol) {
                conv = true;
                break;
            }
            if (P > 0.0) {
                double fn = sqrt(ff), vn = sqrt(vv);
                mix_v = 1.0 - alpha;
                mix_f = fn > 0.0 ? alpha * vn / fn : 0.0;
                if (++n_pos > fp.n_min) {
                    dt = fmin(dt * (double)fp.f_inc, (double)fp.dt_max);
                    alpha *= (double)fp.f_alpha;
                }
            } else {
                mix_v = 0.0;
                mix_f = 0.0;
                dt *= (double)fp.f_dec;
                alpha = (double)fp.alpha_start;
                n_pos = 0;
            }
        }
        // energy at the final positions, written back with them
        double e = 0.0;
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            int i = threadIdx.x + k * RB;
            if (i < n) {
                rep_pairs(s, g, i, p.S, [&](int, const uint32_t *ui, const uint32_t *uj, int pt) {
                    float d[2], r2, u = 0.0f;
                    pair_eval<2, KIND, true, true>(p, pt, ui, uj, g.s, g.sd, d, r2, u);
                    e += (double)u;
                });
            }
        }
        e = 0.5 * wg_sum<RB>(e, s);
        for (int i = threadIdx.x; i < n; i += RB) {
            a.pos[2 * (size_t)(off + i)] = s.pos[2 * i];
            a.pos[2 * (size_t)(off + i) + 1] = s.pos[2 * i + 1];
        }
        if (threadIdx.x == 0) {
            fp.energy[b] = e;
            fp.fmax[b] = sqrt(fm);
            fp.steps[b] = steps;
            fp.status[b] = conv ? 1 : 0;
        }
    }
}

// du/dsigma and du/deps of one pair at fixed r (KIND 0: LJ, 1: soft sphere), and u.
template <int KIND>
__device__ __forceinline__ void pair_dparam(const md_potential &pot, int pt, float r2, double rd, float &dus,
                                            float &due, float &u)
{
    double sigd = pot.sigma[pt];
    float sig = (float)sigd, eps = (float)pot.epsilon[pt];
    dus = due = u = 0.0f;
    if (KIND == 0) {
        if (!(r2 < pot.r_cut * pot.r_cut)) return;
        float q = sig * sig / r2;
        float s6 = q * q * q, s12 = s6 * s6;
        float uu = 4.0f * eps * (s12 - s6);
        float ds = 4.0f * eps * (12.0f * s12 - 6.0f * s6) / sig;
        if (pot.shift) {
            float qc = sig * sig / (pot.r_cut * pot.r_cut);
            float c6 = qc * qc * qc, c12 = c6 * c6;
            uu -= 4.0f * eps * (c12 - c6);
            ds -= 4.0f * eps * (12.0f * c12 - 6.0f * c6) / sig;
        }
        u = uu;
        dus = ds;
        due = uu / eps;
    } else {
        // overlap from the double distance (see ss_fs_precise)
        if (!(rd < sigd)) return;
        float r = (float)rd;
        float t = (float)((sigd - rd) / sigd);
        float a = pot.alpha;
        float tp = a == 2.0f ? t : powf(t, a - 1.0f);
        u = eps / a * tp * t;
        dus = eps * tp * r / (sig * sig);
        due = tp * t / a;
    }
}

struct GradParams {
    double *g_sigma;  // [B][S*S]
    double *g_eps;    // [B][S*S]
    double *energy;   // [B] or null
    int32_t *status;  // [B] or null: -1 replica too large
    float range;
};

template <int KIND>
__global__ __launch_bounds__(kRB) void k_param_grad(BatchArgs a, md_potential pin, GradParams gp)
{
    __shared__ Lds s;
    if (threadIdx.x == 0) s.raw = pin;
    __syncthreads();
    const md_potential &pot = s.raw;
    int S = pot.n_species;
    for (int b = next_replica(s, a.queue); b < a.B; b = next_replica(s, a.queue)) {
        int n, off;
        RepGeom g;
        if (!rep_load<kRB>(s, a, b, gp.range, n, off, g)) {
            if (threadIdx.x == 0 && gp.status) gp.status[b] = -1;
            continue;
        }
        rep_cells<kRB>(s, n, g);
        // one pass per pair type keeps the accumulators in two registers
        for (int q = 0; q < S * S; ++q) {
            double gs = 0.0, ge = 0.0, e = 0.0;
            for (int i = threadIdx.x; i < n; i += kRB) {
                rep_pairs(s, g, i, S, [&](int, const uint32_t *ui, const uint32_t *uj, int pt) {
                    if (pt != q) return;
                    double dx = tdisp_d(ui[0], uj[0], g.sd[0]), dy = tdisp_d(ui[1], uj[1], g.sd[1]);
                    double r2d = __builtin_fma(dx, dx, dy * dy);
                    float dus, due, u;
                    pair_dparam<KIND>(pot, pt, (float)r2d, __builtin_sqrt(r2d), dus, due, u);
                    gs += (double)dus;
                    ge += (double)due;
                    e += (double)u;
                });
            }
            gs = 0.5 * wg_sum<kRB>(gs, s);
            ge = 0.5 * wg_sum<kRB>(ge, s);
            e = 0.5 * wg_sum<kRB>(e, s);
            if (threadIdx.x == 0) {
                gp.g_sigma[(size_t)b * S * S + q] = gs;
                gp.g_eps[(size_t)b * S * S + q] = ge;
                if (gp.energy) gp.energy[b] = (q == 0 ? 0.0 : gp.energy[b]) + e;
            }
        }
        if (threadIdx.x == 0 && gp.status) gp.status[b] = 1;
    }
}

// Chain rule from the per-replica gradients to the requested parameters (one workgroup per replica):
//   MD_WRT_SIGMA / MD_WRT_EPSILON: the S*S ordered entries as they are;
//   MD_WRT_EPSILON_COMMON: sum over the entries (one epsilon shared by every pair);
//   MD_WRT_DIAMETER: dU/dd_s = 1/2 sum_c (G_sc + G_cs) (sigma_ab = (d_a + d_b)/2, App. A), plus with a box that
//   follows the packing fraction (L^2 proportional to sum_t n_t d_t^2 in 2D, positions fractional) the term
//   (n_s d_s / sum_t n_t d_t^2) dU/dln L, with dU/dln L given per replica or, for soft spheres (u a function of
//   r / sigma), equal to -sum_ab sigma_ab G_ab (minus the virial).
struct ChainArgs {
    int32_t B, S, wrt, box, m;     // m outputs per replica
    const int32_t *offset;         // [B+1]
    const int32_t *species;        // [total] or null
    const double *G;               // [B][S*S] dU/dsigma_ab or dU/deps_ab
    const double *rep_sigma;       // [B][S*S] or null (then sigma)
    double sigma[64];              // the potential's sigma matrix
    const double *dln;             // [B] dU/dln L, or null (minus the virial from G)
    double *out;                   // [B][m]
};

__global__ __launch_bounds__(256) void k_chain(ChainArgs a)
{
    __shared__ double red[4];
    __shared__ double cnt[kMaxS];
    const int b = blockIdx.x;
    const int S = a.S;
    const double *G = a.G + (size_t)b * S * S;
    double *out = a.out + (size_t)b * a.m;
    if (a.wrt == MD_WRT_SIGMA || a.wrt == MD_WRT_EPSILON) {
        for (int q = threadIdx.x; q < S * S; q += blockDim.x) out[q] = G[q];
        return;
    }
    if (a.wrt == MD_WRT_EPSILON_COMMON) {
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < S * S; ++q) t += G[q];
            out[0] = t;
        }
        return;
    }
    // species counts of the replica (needed for the packing box only)
    if (a.box == MD_BOX_PACKING) {
        const int lo = a.offset[b], hi = a.offset[b + 1];
        for (int sp = 0; sp < S; ++sp) {
            double c = 0.0;
            for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) c += (a.species ? a.species[i] : 0) == sp ? 1.0 : 0.0;
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
            __syncthreads();
            if (threadIdx.x == 0) cnt[sp] = red[0] + red[1] + red[2] + red[3];
            __syncthreads();
        }
    }
    if (threadIdx.x != 0) return;
    const double *sig = a.rep_sigma ? a.rep_sigma + (size_t)b * S * S : a.sigma;
    double dln = 0.0, nd2 = 0.0;
    if (a.box == MD_BOX_PACKING) {
        if (a.dln) {
            dln = a.dln[b];
        } else {
            for (int q = 0; q < S * S; ++q) dln -= sig[q] * G[q];
        }
        for (int t = 0; t < S; ++t) nd2 += cnt[t] * sig[t * S + t] * sig[t * S + t];
    }
    for (int sp = 0; sp < S; ++sp) {
        double g = 0.0;
        for (int c = 0; c < S; ++c) g += 0.5 * (G[sp * S + c] + G[c * S + sp]);
        if (a.box == MD_BOX_PACKING && nd2 > 0.0) g += cnt[sp] * sig[sp * S + sp] / nd2 * dln;
        out[sp] = g;
    }
}

// out[k] = sum_b w[b] per[b][k] for k < m, summed in a fixed order by one workgroup (a vector-Jacobian product).
__global__ __launch_bounds__(256) void k_weighted_sum(const double *per, const double *w, int B, int m, double *out)
{
    __shared__ double red[4];
    for (int k = 0; k < m; ++k) {
        double t = 0.0;
        for (int b = threadIdx.x; b < B; b += blockDim.x) t += w[b] * per[(size_t)b * m + k];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) out[k] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
}

__global__ void k_zero_queue(int32_t *q)
{
    if (threadIdx.x == 0) q[0] = 0;
}

md_status batch_check(md_ctx *ctx, const md_batch *bt, const md_potential *pot, DevPot &p)
{
    if (!ctx || !bt || !pot || bt->B < 0 || bt->dim != 2 || !bt->offset || !bt->box || !bt->pos) return MD_ERR_ARG;
    if (!md_make_pot(pot, p)) return MD_ERR_ARG;
    if (pot->kind != MD_LJ && pot->kind != MD_SOFT_SPHERE) return MD_ERR_ARG;  // the replica kernels know these two
    if (pot->n_species > 1 && !bt->species) return MD_ERR_ARG;
    if (bt->max_n > kMaxRepN || bt->max_cells > kMaxRepCells) return MD_ERR_CAPACITY;
    return MD_OK;
}

BatchArgs batch_args(md_ctx *ctx, const md_batch *bt)
{
    BatchArgs a;
    a.B = bt->B;
    a.offset = bt->offset;
    a.box = bt->box;
    a.pos = bt->pos;
    a.species = bt->species;
    a.queue = ctx->queue;
    return a;
}

int batch_grid(int B)
{
    return B < 512 ? (B > 0 ? B : 1) : 512;
}

}  // namespace

extern "C" {

md_status fire_batched(md_ctx *ctx, const md_batch *bt, const md_potential *pot, const md_fire_params *fp,
                       const md_batch_config *cfg, int32_t max_steps, double f_tol, double *energy, double *fmax,
                       int32_t *steps, int32_t *status, void *stream)
{
    DevPot p;
    md_status st = batch_check(ctx, bt, pot, p);
    if (st != MD_OK) return st;
    if (!fp || !energy || !fmax || !steps || !status || max_steps < 0) return MD_ERR_ARG;
    const int threads = cfg ? cfg->threads : 512;
    const float cell_factor = cfg ? cfg->cell_factor : 1.0f;
    if ((threads != 512 && threads != 1024) || !(cell_factor >= 1.0f && cell_factor <= 4.0f)) return MD_ERR_ARG;
    if (bt->B == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    BatchArgs a = batch_args(ctx, bt);
    FireBatchParams q;
    q.energy = energy;
    q.fmax = fmax;
    q.steps = steps;
    q.status = status;
    q.dt_start = fp->dt_start;
    q.dt_max = fp->dt_max;
    q.f_inc = fp->f_inc;
    q.f_dec = fp->f_dec;
    q.alpha_start = fp->alpha_start;
    q.f_alpha = fp->f_alpha;
    q.range = md_max_cutoff(pot) * cell_factor;  // cells of edge >= this; pairs still stop at the potential's range
    q.n_min = fp->n_min;
    q.max_steps = max_steps;
    q.f_tol = f_tol;
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, ctx->queue);
    if (pot->kind == MD_LJ) {
        if (threads == 1024) hipLaunchKernelGGL((k_fire_batched<0, 1024>), dim3(batch_grid(bt->B)), dim3(1024), 0, s, a, p, q);
        else hipLaunchKernelGGL((k_fire_batched<0, 512>), dim3(batch_grid(bt->B)), dim3(512), 0, s, a, p, q);
    } else {
        if (threads == 1024) hipLaunchKernelGGL((k_fire_batched<1, 1024>), dim3(batch_grid(bt->B)), dim3(1024), 0, s, a, p, q);
        else hipLaunchKernelGGL((k_fire_batched<1, 512>), dim3(batch_grid(bt->B)), dim3(512), 0, s, a, p, q);
    }
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status envelope_grad(md_ctx *ctx, const md_batch *bt, const md_potential *pot, double *g_sigma, double *g_eps,
                        double *energy, int32_t *status, void *stream)
{
    DevPot p;
    md_status st = batch_check(ctx, bt, pot, p);
    if (st != MD_OK) return st;
    if (!g_sigma || !g_eps || pot->n_species > kMaxS) return MD_ERR_ARG;
    if (bt->B == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    BatchArgs a = batch_args(ctx, bt);
    GradParams gp;
    gp.g_sigma = g_sigma;
    gp.g_eps = g_eps;
    gp.energy = energy;
    gp.status = status;
    gp.range = md_max_cutoff(pot);
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, ctx->queue);
    if (pot->kind == MD_LJ)
        hipLaunchKernelGGL(k_param_grad<0>, dim3(batch_grid(bt->B)), dim3(kRB), 0, s, a, *pot, gp);
    else
        hipLaunchKernelGGL(k_param_grad<1>, dim3(batch_grid(bt->B)), dim3(kRB), 0, s, a, *pot, gp);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}


// Outputs per replica for a derivative family.
static int wrt_width(int wrt, int S)
{
    return wrt == MD_WRT_SIGMA || wrt == MD_WRT_EPSILON ? S * S : (wrt == MD_WRT_DIAMETER ? S : 1);
}

// The chain-rule launches shared by envelope_grad_wrt and md_diameter_grad: per-replica results into `per`
// (scratch) or, without weights, straight into out.
static md_status launch_chain(const md_batch *bt, const md_potential *pot, int wrt, int box, const double *G,
                              const double *rep_sigma, const double *dln, const double *weights, double *per,
                              double *out, hipStream_t s)
{
    ChainArgs c{};
    c.B = bt->B;
    c.S = pot->n_species;
    c.wrt = wrt;
    c.box = box;
    c.m = wrt_width(wrt, c.S);
    c.offset = bt->offset;
    c.species = bt->species;
    c.G = G;
    c.rep_sigma = rep_sigma;
    for (int q = 0; q < 64; ++q) c.sigma[q] = pot->sigma[q];
    c.dln = dln;
    c.out = weights ? per : out;
    hipLaunchKernelGGL(k_chain, dim3(bt->B), dim3(256), 0, s, c);
    if (weights) hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(256), 0, s, per, weights, bt->B, c.m, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

// The diameter derivative needs sigma_ab = (d_a + d_b)/2 with d_s = sigma_ss.
static bool mixing_rule(const md_potential *pot)
{
    const int S = pot->n_species;
    for (int a = 0; a < S; ++a)
        for (int b = 0; b < S; ++b) {
            const double want = 0.5 * (pot->sigma[a * S + a] + pot->sigma[b * S + b]);
            if (fabs(pot->sigma[a * S + b] - want) > 1e-12 * fabs(want)) return false;
        }
    return true;
}

md_status envelope_grad_wrt(md_ctx *ctx, const md_batch *bt, const md_potential *pot, int32_t wrt, int32_t box,
                            const double *weights, double *grad, double *energy, int32_t *status, void *stream)
{
    DevPot p;
    md_status st = batch_check(ctx, bt, pot, p);
    if (st != MD_OK) return st;
    if (!grad || pot->n_species > kMaxS || wrt < MD_WRT_SIGMA || wrt > MD_WRT_EPSILON_COMMON) return MD_ERR_ARG;
    if (box != MD_BOX_FIXED && box != MD_BOX_PACKING) return MD_ERR_ARG;
    if (wrt == MD_WRT_DIAMETER && !mixing_rule(pot)) return MD_ERR_ARG;
    if (box == MD_BOX_PACKING && (wrt != MD_WRT_DIAMETER || pot->kind != MD_SOFT_SPHERE)) return MD_ERR_ARG;
    if (bt->B == 0) return MD_OK;
    const int S = pot->n_species, m = wrt_width(wrt, S);
    // scratch: dU/dsigma and dU/deps per replica, then the per-replica results when they are weighted
    if ((int64_t)bt->B * (2 * S * S + m) > (int64_t)4 * md_partials_blocks()) return MD_ERR_CAPACITY;
    double *gs = ctx->partials, *ge = gs + (size_t)bt->B * S * S, *per = ge + (size_t)bt->B * S * S;
    hipStream_t s = (hipStream_t)stream;
    st = envelope_grad(ctx, bt, pot, gs, ge, energy, status, stream);
    if (st != MD_OK) return st;
    const bool eps = wrt == MD_WRT_EPSILON || wrt == MD_WRT_EPSILON_COMMON;
    return launch_chain(bt, pot, wrt, box, eps ? ge : gs, nullptr, nullptr, weights, per, grad, s);
}

md_status md_diameter_grad(md_ctx *ctx, const md_batch *bt, const md_potential *pot, const double *sigma,
                           const double *g_sigma, const double *dln, int32_t box, const double *weights, double *out,
                           void *stream)
{
    if (!ctx || !bt || !pot || !g_sigma || !out || bt->B < 0 || pot->n_species < 1 || pot->n_species > kMaxS)
        return MD_ERR_ARG;
    if (box != MD_BOX_FIXED && box != MD_BOX_PACKING) return MD_ERR_ARG;
    if (bt->B > 0 && (!bt->offset || (pot->n_species > 1 && !bt->species))) return MD_ERR_ARG;
    if (!sigma && !mixing_rule(pot)) return MD_ERR_ARG;
    if (box == MD_BOX_PACKING && (bt->dim != 2 || (!dln && pot->kind != MD_SOFT_SPHERE))) return MD_ERR_ARG;
    if (bt->B == 0) return MD_OK;
    const int S = pot->n_species;
    if (weights && (int64_t)bt->B * S > (int64_t)4 * md_partials_blocks()) return MD_ERR_CAPACITY;
    return launch_chain(bt, pot, MD_WRT_DIAMETER, box, g_sigma, sigma, dln, weights, ctx->partials, out,
                        (hipStream_t)stream);
}

}  // extern "C"
