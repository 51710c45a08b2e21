// The flocking energy model of App. B on a neighbor list (Sec. 4.3: boids interact with their local
// neighborhood only, so a list scales the model to tens of thousands of agents), 2D, one thread per boid:
//
//   k_flock_terms   per boid i over its list row: avoidance dE/dR_i, alignment dE/dtheta_i, the obstacle terms,
//                   and cohesion: dR_i = mean over neighbors within R_coh of (R_j - R_i), its energy
//                   1/2 J (1 - hat(dR_i) . N_i)^2, the gradient g_i of that energy with respect to dR_i, the
//                   heading part, and the boid's own position part -g_i;
//   k_flock_gather  per boid k: adds g_i / n_i of every neighbor i within R_coh (dR_i moves with R_k);
//   k_flock_move    forward Euler, R += dt (v N - dE/dR), theta -= dt dE/dtheta, and the rebuild trigger.
//
// With rho(r; Rc) = (1/alpha)(1 - r/Rc)^alpha the pair terms are J_avoid rho(r; R_avoid) and J_align rho(r;
// R_align)(1 - N_i . N_j)^2 (its position gradient stopped), and an obstacle o (center C, radius D) adds
// J_obs rho(|R_i - C|; D)(1 - N_i . hat(R_i - C))^2.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

constexpr int kWork = 6;  // floats per boid in the work array: dE/dR (2), dE/dtheta, g / n (2), pad

struct FlockArgs {
    const uint32_t *pos;
    float *theta;
    int N, W, capW;
    const int32_t *idx, *count;
    float s[2], inv_s[2], L[2];
    md_flock_params fp;
    float *work;
};

__device__ __forceinline__ float rho_t(float t, float a)  // (1/a) t^a, t in (0, 1]
{
    return __builtin_exp2f(a * __builtin_log2f(t)) / a;
}

__device__ __forceinline__ float drho_t(float t, float a, float Rc)  // d rho / dr = -(1/Rc) t^(a-1)
{
    return -__builtin_exp2f((a - 1.0f) * __builtin_log2f(t)) / Rc;
}

template <class Fn>
__device__ __forceinline__ void for_row(const FlockArgs &a, int i, Fn &&f)
{
    for (int l = 0; l < a.W; ++l) {
        int n = min(a.count[(size_t)i * a.W + l], a.capW);
        for (int t = 0; t < n; ++t) f(a.idx[((size_t)t * a.N + i) * a.W + l]);
    }
}

__global__ __launch_bounds__(kBlock) void k_flock_terms(FlockArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    const md_flock_params &p = a.fp;
    uint32_t ui[2] = {a.pos[2 * (size_t)i], a.pos[2 * (size_t)i + 1]};
    float th = a.theta[i];
    const float Nx = cosf(th), Ny = sinf(th);
    float gx = 0.0f, gy = 0.0f, gt = 0.0f, Sx = 0.0f, Sy = 0.0f;
    int n = 0;
    for_row(a, i, [&](int j) {
        float dx = tdisp(ui[0], a.pos[2 * (size_t)j], a.s[0]);      // R_i - R_j
        float dy = tdisp(ui[1], a.pos[2 * (size_t)j + 1], a.s[1]);
        float r2 = __builtin_fmaf(dx, dx, dy * dy);
        float r = sqrtf(r2);
        if (r < p.R_avoid) {
            float c = p.J_avoid * drho_t(1.0f - r / p.R_avoid, p.alpha, p.R_avoid) / r;
            gx = __builtin_fmaf(c, dx, gx);
            gy = __builtin_fmaf(c, dy, gy);
        }
        if (r < p.R_align) {
            float dth = th - a.theta[j];
            float cc = cosf(dth), ss = sinf(dth);
            gt += p.J_align * rho_t(1.0f - r / p.R_align, p.alpha) * 2.0f * (1.0f - cc) * ss;
        }
        if (r2 < p.R_coh * p.R_coh) {
            Sx -= dx;
            Sy -= dy;
            ++n;
        }
    });
    const float xi = (float)ui[0] * a.s[0], yi = (float)ui[1] * a.s[1];
    for (int o = 0; o < p.n_obstacles; ++o) {
        float cx = xi - p.obstacles[o][0], cy = yi - p.obstacles[o][1], D = p.obstacles[o][2];
        cx -= a.L[0] * rintf(cx / a.L[0]);
        cy -= a.L[1] * rintf(cy / a.L[1]);
        float ro = sqrtf(__builtin_fmaf(cx, cx, cy * cy));
        if (ro < D && ro > 0.0f) {
            float hx = cx / ro, hy = cy / ro;
            float am = __builtin_fmaf(Nx, hx, Ny * hy);
            float t = 1.0f - ro / D;
            float w = rho_t(t, p.alpha), dw = drho_t(t, p.alpha, D);
            float om = 1.0f - am;
            gx += p.J_obs * (dw * hx * om * om - 2.0f * w * om * (Nx - am * hx) / ro);
            gy += p.J_obs * (dw * hy * om * om - 2.0f * w * om * (Ny - am * hy) / ro);
            gt += p.J_obs * w * 2.0f * om * (Ny * hx - Nx * hy);      // -(N_perp . hat) with N_perp = (-sin, cos)
        }
    }
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
    w[3] = Gx;
    w[4] = Gy;
}

__global__ __launch_bounds__(kBlock) void k_flock_gather(FlockArgs a)
{
    int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.N) return;
    const float R2 = a.fp.R_coh * a.fp.R_coh;
    uint32_t uk[2] = {a.pos[2 * (size_t)k], a.pos[2 * (size_t)k + 1]};
    float gx = 0.0f, gy = 0.0f;
    for_row(a, k, [&](int i) {
        float dx = tdisp(uk[0], a.pos[2 * (size_t)i], a.s[0]);
        float dy = tdisp(uk[1], a.pos[2 * (size_t)i + 1], a.s[1]);
        if (__builtin_fmaf(dx, dx, dy * dy) < R2) {   // the same test as k_flock_terms, from the other end
            gx += a.work[(size_t)i * kWork + 3];
            gy += a.work[(size_t)i * kWork + 4];
        }
    });
    a.work[(size_t)k * kWork + 0] += gx;
    a.work[(size_t)k * kWork + 1] += gy;
}

__global__ __launch_bounds__(kBlock) void k_flock_move(FlockArgs a, uint32_t *pos, const uint32_t *pos_ref,
                                                       float half_skin, int32_t *ctl)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < a.N) {
        const float *w = a.work + (size_t)i * kWork;
        float th = a.theta[i];
        float dt = a.fp.dt, v = a.fp.v;
        float dx = dt * (v * cosf(th) - w[0]), dy = dt * (v * sinf(th) - w[1]);
        uint32_t u0 = pos[2 * (size_t)i] + (uint32_t)__float2int_rn(dx * a.inv_s[0]);
        uint32_t u1 = pos[2 * (size_t)i + 1] + (uint32_t)__float2int_rn(dy * a.inv_s[1]);
        pos[2 * (size_t)i] = u0;
        pos[2 * (size_t)i + 1] = u1;
        a.theta[i] = th - dt * w[2];
        float ex = tdisp(u0, pos_ref[2 * (size_t)i], a.s[0]), ey = tdisp(u1, pos_ref[2 * (size_t)i + 1], a.s[1]);
        far = __builtin_fmaf(ex, ex, ey * ey) > half_skin * half_skin;
    }
    uint64_t m = __ballot(far);  // one store per wave that has a far boid
    if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) ctl[kTrigWord] = 1;
}

int nblocks(int n)
{
    return (n + kBlock - 1) / kBlock;
}

}  // namespace

extern "C" {

md_status flock_step(md_ctx *ctx, const md_box *box, uint32_t *pos, float *theta, int32_t N, const md_nlist *nl,
                     const md_flock_params *fp, float *work, void *stream)
{
    if (!ctx || !box || box->dim != 2 || !pos || !theta || !nl || !fp || !work || N < 0 || nl->N != N ||
        nl->segment != 0 || !nl->idx || !nl->count || !nl->pos_ref)
        return MD_ERR_ARG;
    if (fp->n_obstacles < 0 || fp->n_obstacles > 16 || !(fp->alpha >= 1.0f) || !(fp->R_align > 0.0f) ||
        !(fp->R_avoid > 0.0f) || !(fp->R_coh > 0.0f) || !isfinite(fp->dt))
        return MD_ERR_ARG;
    float rmax = fmaxf(fp->R_align, fmaxf(fp->R_avoid, fp->R_coh));
    if (nl->r_list < rmax) return MD_ERR_ARG;
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
    if (N == 0) return MD_OK;
    a.pos = pos;
    a.theta = theta;
    a.N = N;
    a.W = W;
    a.capW = nl->capacity / W;
    a.idx = nl->idx;
    a.count = nl->count;
    a.fp = *fp;
    a.work = work;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_flock_terms, dim3(nblocks(N)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_flock_gather, dim3(nblocks(N)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_flock_move, dim3(nblocks(N)), dim3(kBlock), 0, s, a, pos, nl->pos_ref, 0.5f * nl->skin,
                       ctx->ctl);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
