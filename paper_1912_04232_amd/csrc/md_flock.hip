// The flocking energy model of App. B on a neighbor list (Sec. 4.3: boids interact with their local
// neighborhood only, so a list scales the model to tens of thousands of agents), 2D.  W lanes per boid walk
// the W sub-rows of its list row and their sums are combined across the lanes (more waves in flight to hide the
// neighbor gathers than one thread per boid gives):
//
//   k_flock_heading N_i = (cos theta_i, sin theta_i), once per boid and step;
//   k_flock_terms   per boid i over its list row: avoidance dE/dR_i, alignment dE/dtheta_i, the obstacle terms,
//                   and cohesion: dR_i = mean over neighbors within R_coh of (R_j - R_i), its energy
//                   1/2 J (1 - hat(dR_i) . N_i)^2, the gradient g_i of that energy with respect to dR_i, the
//                   heading part, and the boid's own position part -g_i;
//   k_flock_gather  per boid k: adds g_i / n_i of every neighbor i within R_coh (dR_i moves with R_k);
//   k_pred_partial, k_pred_finish  (with predators) each predator's step on its own energy;
//   k_flock_move    forward Euler, R += dt (v N - dE/dR), theta -= dt dE/dtheta, and the rebuild trigger.
//
// With rho(r; Rc) = (1/alpha)(1 - r/Rc)^alpha the pair terms are J_avoid rho(r; R_avoid) and J_align rho(r;
// R_align)(1 - N_i . N_j)^2 (its position gradient stopped), and an obstacle o (center C, radius D) adds
// J_obs rho(|R_i - C|; D)(1 - N_i . hat(R_i - C))^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

constexpr int kWork = 8;  // floats per boid in the work array: dE/dR (2), dE/dtheta, pad, g / n (2), N (2)

struct FlockArgs {
    const uint32_t *pos;
    float *theta;
    int N, capW;
    const int32_t *idx, *count;
    float s[2], inv_s[2], L[2];
    md_flock_params fp;
    float inv_R_align, inv_R_avoid, inv_alpha;
    int ialpha;  // alpha when it is an integer in [1, 8] (powers by multiplication), else -1
    float *work;
    int P;                 // predators (0: none)
    uint32_t *ppos;        // [P][2]
    float *pth;            // [P]
    float J_flee, R_flee, J_chase, R_chase, v_pred;
};



// t^e for t in [0, 1]: repeated products when the exponent is a small integer (ie >= 0; t^0 = 1 even at t = 0),
// else exp2(e log2 t) for a non-integer e > 0 (ie < 0), which is 0 at t = 0
__device__ __forceinline__ float tpow(float t, int ie, float e)
{
    if (ie >= 0) {
        float p = 1.0f;
        for (int k = 0; k < ie; ++k) p *= t;
        return p;
    }
    return __builtin_exp2f(e * __builtin_log2f(t));
}

__device__ __forceinline__ float rho_t(const FlockArgs &a, float t)  // (1/alpha) t^alpha
{
    return tpow(t, a.ialpha, a.fp.alpha) * a.inv_alpha;
}

__device__ __forceinline__ float drho_t(const FlockArgs &a, float t, float inv_Rc)  // d rho / dr = -(1/Rc) t^(alpha-1)
{
    return -tpow(t, a.ialpha - 1, a.fp.alpha - 1.0f) * inv_Rc;
}

// J rho(|x|; D)(1 - N . hat x)^2 (the obstacle form; x = X - C) added to the gradients in X and in the angle.
__device__ __forceinline__ void facing_grad(const FlockArgs &a, float cx, float cy, float Nx, float Ny, float D,
                                            float J, float &gx, float &gy, float &gt)
{
    float ro = sqrtf(__builtin_fmaf(cx, cx, cy * cy));
    if (!(ro < D && ro > 0.0f)) return;
    float hx = cx / ro, hy = cy / ro;
    float am = __builtin_fmaf(Nx, hx, Ny * hy);
    float tt = 1.0f - ro / D;
    float w = tpow(tt, a.ialpha, a.fp.alpha) * a.inv_alpha;
    float dw = -tpow(tt, a.ialpha - 1, a.fp.alpha - 1.0f) / D;
    float om = 1.0f - am;
    gx += J * (dw * hx * om * om - 2.0f * w * om * (Nx - am * hx) / ro);
    gy += J * (dw * hy * om * om - 2.0f * w * om * (Ny - am * hy) / ro);
    gt += J * w * 2.0f * om * (Ny * hx - Nx * hy);      // -(N_perp . hat) with N_perp = (-sin, cos)
}

// Sum over the W lanes of one boid (adjacent lanes of a wave), a fixed tree: deterministic.
template <int W>
__device__ __forceinline__ float lane_sum(float v)
{
#pragma unroll
    for (int m = 1; m < W; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int W>
__device__ __forceinline__ int lane_sum_i(int v)
{
#pragma unroll
    for (int m = 1; m < W; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_flock_heading(FlockArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    float th = a.theta[i];
    a.work[(size_t)i * kWork + 6] = cosf(th);
    a.work[(size_t)i * kWork + 7] = sinf(th);
}

// W lanes per boid: lane l walks sub-row l of the list, the lane sums are combined, and lane 0 finishes.
template <int W>
__global__ __launch_bounds__(kBlock) void k_flock_terms(FlockArgs a)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int i = t / W, l = t % W;
    const bool live = i < a.N;
    const md_flock_params &p = a.fp;
    const int ic = live ? i : 0;
    uint32_t ui[2] = {a.pos[2 * (size_t)ic], a.pos[2 * (size_t)ic + 1]};
    const float2 Ni = *reinterpret_cast<const float2 *>(a.work + (size_t)ic * kWork + 6);
    float gx = 0.0f, gy = 0.0f, gt = 0.0f, Sx = 0.0f, Sy = 0.0f;
    int n = 0;
    const int len = live ? min(a.count[(size_t)i * W + l], a.capW) : 0;
    const float R2coh = p.R_coh * p.R_coh;
    for (int q = 0; q < len; ++q) {
        int j = a.idx[((size_t)q * a.N + i) * W + l];
        float dx = tdisp(ui[0], a.pos[2 * (size_t)j], a.s[0]);      // R_i - R_j
        float dy = tdisp(ui[1], a.pos[2 * (size_t)j + 1], a.s[1]);
        float r2 = __builtin_fmaf(dx, dx, dy * dy);
        float r = sqrtf(r2);
        if (r < p.R_avoid) {
            float c = p.J_avoid * drho_t(a, 1.0f - r * a.inv_R_avoid, a.inv_R_avoid) / r;
            gx = __builtin_fmaf(c, dx, gx);
            gy = __builtin_fmaf(c, dy, gy);
        }
        if (r < p.R_align) {
            const float2 Nj = *reinterpret_cast<const float2 *>(a.work + (size_t)j * kWork + 6);
            float cc = __builtin_fmaf(Ni.x, Nj.x, Ni.y * Nj.y);       // cos(theta_i - theta_j)
            float ss = __builtin_fmaf(Ni.y, Nj.x, -Ni.x * Nj.y);      // sin(theta_i - theta_j)
            gt += p.J_align * rho_t(a, 1.0f - r * a.inv_R_align) * 2.0f * (1.0f - cc) * ss;
        }
        if (r2 < R2coh) {
            Sx -= dx;
            Sy -= dy;
            ++n;
        }
    }
    // obstacles and predators, dealt round-robin to the boid's W lanes
    const float Nx = Ni.x, Ny = Ni.y;
    const float xi = (float)ui[0] * a.s[0], yi = (float)ui[1] * a.s[1];
    for (int o = l; o < p.n_obstacles; o += W) {
        float cx = xi - p.obstacles[o][0], cy = yi - p.obstacles[o][1];
        cx -= a.L[0] * rintf(cx / a.L[0]);
        cy -= a.L[1] * rintf(cy / a.L[1]);
        facing_grad(a, cx, cy, Nx, Ny, p.obstacles[o][2], p.J_obs, gx, gy, gt);
    }
    for (int q = l; q < a.P; q += W)  // fleeing: the obstacle form with the predator as the disk center
        facing_grad(a, tdisp(ui[0], a.ppos[2 * q], a.s[0]), tdisp(ui[1], a.ppos[2 * q + 1], a.s[1]), Nx, Ny,
                    a.R_flee, a.J_flee, gx, gy, gt);
    gx = lane_sum<W>(gx);
    gy = lane_sum<W>(gy);
    gt = lane_sum<W>(gt);
    Sx = lane_sum<W>(Sx);
    Sy = lane_sum<W>(Sy);
    n = lane_sum_i<W>(n);
    if (!live || l != 0) return;
    float Gx = 0.0f, Gy = 0.0f;
    if (n > 0) {
        float dRx = Sx / n, dRy = Sy / n;
        float dn = sqrtf(__builtin_fmaf(dRx, dRx, dRy * dRy));
        if (dn > 0.0f) {
            float hx = dRx / dn, hy = dRy / dn;
            float ci = __builtin_fmaf(hx, Nx, hy * Ny);
            float k = -p.J_coh * (1.0f - ci) / dn;
            float g0 = k * (Nx - ci * hx), g1 = k * (Ny - ci * hy);
            gt += -p.J_coh * (1.0f - ci) * (Nx * hy - Ny * hx);      // dh . N_perp
            gx -= g0;
            gy -= g1;
            Gx = g0 / n;
            Gy = g1 / n;
        }
    }
    float *w = a.work + (size_t)i * kWork;
    w[0] = gx;
    w[1] = gy;
    w[2] = gt;
    w[3] = 0.0f;
    w[4] = Gx;
    w[5] = Gy;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_flock_gather(FlockArgs a)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int k = t / W, l = t % W;
    const bool live = k < a.N;
    const float R2 = a.fp.R_coh * a.fp.R_coh;
    const int kc = live ? k : 0;
    uint32_t uk[2] = {a.pos[2 * (size_t)kc], a.pos[2 * (size_t)kc + 1]};
    float gx = 0.0f, gy = 0.0f;
    const int len = live ? min(a.count[(size_t)k * W + l], a.capW) : 0;
    for (int q = 0; q < len; ++q) {
        int i = a.idx[((size_t)q * a.N + k) * W + l];
        float dx = tdisp(uk[0], a.pos[2 * (size_t)i], a.s[0]);
        float dy = tdisp(uk[1], a.pos[2 * (size_t)i + 1], a.s[1]);
        if (__builtin_fmaf(dx, dx, dy * dy) < R2) {   // the same test as k_flock_terms, from the other end
            const float2 G = *reinterpret_cast<const float2 *>(a.work + (size_t)i * kWork + 4);
            gx += G.x;
            gy += G.y;
        }
    }
    gx = lane_sum<W>(gx);
    gy = lane_sum<W>(gy);
    if (!live || l != 0) return;
    a.work[(size_t)k * kWork + 0] += gx;
    a.work[(size_t)k * kWork + 1] += gy;
}

// Predators, in two launches.  k_pred_partial: workgroup (b, k) sums R_j - R_p and the count over the boids
// within R_chase of predator k among the b-th of B equal slices of the boids (a fixed LDS tree), into
// partials[(k B + b) 3 + 0..2] (double).  k_pred_finish: one wave per predator adds the B partials in a fixed
// xor tree (deterministic); its first lane forms the cohesion-form gradient (dR_p moves by -dR_p) and the
// obstacle terms, and takes the predator's forward-Euler step.  Both run after k_flock_terms has read the predators and before the boids move,
// so both sides step from the same state.
__global__ __launch_bounds__(kBlock) void k_pred_partial(FlockArgs a, double *partials, int B)
{
    __shared__ float sx[kBlock], sy[kBlock];
    __shared__ int sn[kBlock];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const uint32_t u0 = a.ppos[2 * k], u1 = a.ppos[2 * k + 1];
    const float R2 = a.R_chase * a.R_chase;
    const int chunk = (a.N + B - 1) / B;
    const int lo = b * chunk, hi = min(a.N, lo + chunk);
    float Sx = 0.0f, Sy = 0.0f;
    int n = 0;
    for (int j = lo + t; j < hi; j += kBlock) {
        float dx = tdisp(a.pos[2 * (size_t)j], u0, a.s[0]), dy = tdisp(a.pos[2 * (size_t)j + 1], u1, a.s[1]);
        if (__builtin_fmaf(dx, dx, dy * dy) < R2) {
            Sx += dx;
            Sy += dy;
            ++n;
        }
    }
    sx[t] = Sx;
    sy[t] = Sy;
    sn[t] = n;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) {
            sx[t] += sx[t + off];
            sy[t] += sy[t + off];
            sn[t] += sn[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *o = partials + ((size_t)k * B + b) * 3;
        o[0] = sx[0];
        o[1] = sy[0];
        o[2] = sn[0];
    }
}

__global__ __launch_bounds__(64) void k_pred_finish(FlockArgs a, const double *partials, int B)
{
    const int k = blockIdx.x, lane = threadIdx.x;  // one wave per predator, lane b holds partial b (B <= 64)
    double Sx = 0.0, Sy = 0.0, n = 0.0;
    if (lane < B) {
        const double *o = partials + ((size_t)k * B + lane) * 3;
        Sx = o[0];
        Sy = o[1];
        n = o[2];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {  // fixed xor tree: deterministic
        Sx += __shfl_xor(Sx, m, 64);
        Sy += __shfl_xor(Sy, m, 64);
        n += __shfl_xor(n, m, 64);
    }
    if (lane != 0) return;
    const uint32_t u0 = a.ppos[2 * k], u1 = a.ppos[2 * k + 1];
    const float th = a.pth[k], Nx = cosf(th), Ny = sinf(th);
    float gx = 0.0f, gy = 0.0f, gt = 0.0f;
    if (n > 0.0) {
        float dRx = (float)(Sx / n), dRy = (float)(Sy / n);
        float dn = sqrtf(__builtin_fmaf(dRx, dRx, dRy * dRy));
        if (dn > 0.0f) {
            float hx = dRx / dn, hy = dRy / dn;
            float ci = __builtin_fmaf(hx, Nx, hy * Ny);
            float kk = -a.J_chase * (1.0f - ci) / dn;
            gx -= kk * (Nx - ci * hx);
            gy -= kk * (Ny - ci * hy);
            gt += -a.J_chase * (1.0f - ci) * (Nx * hy - Ny * hx);
        }
    }
    const float xp = (float)u0 * a.s[0], yp = (float)u1 * a.s[1];
    for (int o = 0; o < a.fp.n_obstacles; ++o) {
        float cx = xp - a.fp.obstacles[o][0], cy = yp - a.fp.obstacles[o][1];
        cx -= a.L[0] * rintf(cx / a.L[0]);
        cy -= a.L[1] * rintf(cy / a.L[1]);
        facing_grad(a, cx, cy, Nx, Ny, a.fp.obstacles[o][2], a.fp.J_obs, gx, gy, gt);
    }
    const float dt = a.fp.dt;
    a.ppos[2 * k] = u0 + (uint32_t)__float2int_rn(dt * (a.v_pred * Nx - gx) * a.inv_s[0]);
    a.ppos[2 * k + 1] = u1 + (uint32_t)__float2int_rn(dt * (a.v_pred * Ny - gy) * a.inv_s[1]);
    a.pth[k] = th - dt * gt;
}

__global__ __launch_bounds__(kBlock) void k_flock_move(FlockArgs a, uint32_t *pos, const uint32_t *pos_ref,
                                                       float half_skin, int32_t *ctl)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < a.N) {
        const float *w = a.work + (size_t)i * kWork;
        float dt = a.fp.dt, v = a.fp.v;
        float dx = dt * (v * w[6] - w[0]), dy = dt * (v * w[7] - w[1]);
        uint32_t u0 = pos[2 * (size_t)i] + (uint32_t)__float2int_rn(dx * a.inv_s[0]);
        uint32_t u1 = pos[2 * (size_t)i + 1] + (uint32_t)__float2int_rn(dy * a.inv_s[1]);
        pos[2 * (size_t)i] = u0;
        pos[2 * (size_t)i + 1] = u1;
        a.theta[i] -= dt * w[2];
        float ex = tdisp(u0, pos_ref[2 * (size_t)i], a.s[0]), ey = tdisp(u1, pos_ref[2 * (size_t)i + 1], a.s[1]);
        far = __builtin_fmaf(ex, ex, ey * ey) > half_skin * half_skin;
    }
    uint64_t m = __ballot(far);  // one store per wave that has a far boid
    if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) ctl[kTrigWord] = 1;
}

int nblocks(int64_t n)
{
    return (int)((n + kBlock - 1) / kBlock);
}

}  // namespace

extern "C" {

md_status flock_step(md_ctx *ctx, const md_box *box, uint32_t *pos, float *theta, int32_t N, const md_nlist *nl,
                     const md_flock_params *fp, const md_flock_predators *pred, float *work, void *stream)
{
    if (!ctx || !box || box->dim != 2 || !nl || !fp || N < 0 || nl->N != N || nl->segment != 0 ||
        (N > 0 && (!pos || !theta || !work || !nl->idx || !nl->count || !nl->pos_ref)))
        return MD_ERR_ARG;
    if (fp->n_obstacles < 0 || fp->n_obstacles > 16 || !(fp->alpha >= 1.0f) || !(fp->R_align > 0.0f) ||
        !(fp->R_avoid > 0.0f) || !(fp->R_coh > 0.0f) || !isfinite(fp->dt))
        return MD_ERR_ARG;
    // between rebuilds a boid moves up to skin/2 from its reference position, so the list holds every pair within
    // r_list - skin; that must cover the longest interaction range
    float rmax = fmaxf(fp->R_align, fmaxf(fp->R_avoid, fp->R_coh));
    if (!md_list_covers(nl, rmax) || (int64_t)N * 8 >= ((int64_t)1 << 31)) return MD_ERR_ARG;
    int W = nl->lanes;
    if (W != 1 && W != 2 && W != 4 && W != 8) return MD_ERR_ARG;
    FlockArgs a{};
    for (int k = 0; k < 2; ++k) {
        float L = box->L[k];
        if (!(L > 0.0f) || !isfinite(L) || !(nl->r_list < 0.5f * L)) return MD_ERR_BOX;
        a.s[k] = L / 4294967296.0f;
        a.inv_s[k] = 4294967296.0f / L;
        a.L[k] = L;
    }
    if (pred && pred->P > 0) {
        if (pred->P > 4096 || !pred->pos || !pred->theta || !(pred->R_flee > 0.0f) || !(pred->R_chase > 0.0f) ||
            !isfinite(pred->J_flee) || !isfinite(pred->J_chase) || !isfinite(pred->v))
            return MD_ERR_ARG;
        if (!(pred->R_flee < 0.5f * fminf(a.L[0], a.L[1])) || !(pred->R_chase < 0.5f * fminf(a.L[0], a.L[1])))
            return MD_ERR_BOX;
        a.P = pred->P;
        a.ppos = pred->pos;
        a.pth = pred->theta;
        a.J_flee = pred->J_flee;
        a.R_flee = pred->R_flee;
        a.J_chase = pred->J_chase;
        a.R_chase = pred->R_chase;
        a.v_pred = pred->v;
    }
    a.pos = pos;
    a.theta = theta;
    a.N = N;
    a.capW = nl->capacity / W;
    a.idx = nl->idx;
    a.count = nl->count;
    a.fp = *fp;
    a.inv_R_align = 1.0f / fp->R_align;
    a.inv_R_avoid = 1.0f / fp->R_avoid;
    a.inv_alpha = 1.0f / fp->alpha;
    a.ialpha = (fp->alpha == floorf(fp->alpha) && fp->alpha <= 8.0f) ? (int)fp->alpha : -1;
    a.work = work;
    hipStream_t s = (hipStream_t)stream;
    const int g1 = nblocks(N), gW = nblocks((int64_t)N * W);
    // with no boids only the predators step: they still swim and feel the obstacles (their chase sums are empty)
    if (N > 0) {
    hipLaunchKernelGGL(k_flock_heading, dim3(g1), dim3(kBlock), 0, s, a);
    switch (W) {
    case 1:
        hipLaunchKernelGGL(k_flock_terms<1>, dim3(gW), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_flock_gather<1>, dim3(gW), dim3(kBlock), 0, s, a);
        break;
    case 2:
        hipLaunchKernelGGL(k_flock_terms<2>, dim3(gW), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_flock_gather<2>, dim3(gW), dim3(kBlock), 0, s, a);
        break;
    case 4:
        hipLaunchKernelGGL(k_flock_terms<4>, dim3(gW), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_flock_gather<4>, dim3(gW), dim3(kBlock), 0, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_flock_terms<8>, dim3(gW), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_flock_gather<8>, dim3(gW), dim3(kBlock), 0, s, a);
        break;
    }
    }
    if (a.P > 0) {
        // slices per predator: enough workgroups to fill the chip, within the context's partials buffer
        const int64_t cap = (int64_t)4 * md_partials_blocks() / (3 * (int64_t)a.P);
        const int B = (int)std::max<int64_t>(1, std::min<int64_t>({64, cap, (int64_t)(N + kBlock - 1) / kBlock}));
        hipLaunchKernelGGL(k_pred_partial, dim3(B, a.P), dim3(kBlock), 0, s, a, ctx->partials, B);
        hipLaunchKernelGGL(k_pred_finish, dim3(a.P), dim3(64), 0, s, a, (const double *)ctx->partials, B);
    }
    if (N > 0)
        hipLaunchKernelGGL(k_flock_move, dim3(g1), dim3(kBlock), 0, s, a, pos, nl->pos_ref, 0.5f * nl->skin, ctx->ctl);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
