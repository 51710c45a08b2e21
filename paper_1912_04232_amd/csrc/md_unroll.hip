// Reverse mode through a fixed number of FIRE steps for a batch of small 2D replicas: the derivative of
// the final energy that Sec. 4.2 obtains by differentiating through the minimizer (App. A runs FIRE for a
// fixed 300 steps on 128 disks and takes the gradient through the loop with respect to the diameter).
//
// One wavefront owns one replica (up to 256 particles, lane l holds particles l, l+64, ...); four
// replicas share a workgroup but never synchronize with each other.  Positions (uint32 torus
// coordinates, i.e. fractional coordinates R = u / 2^32) and the vector of the current pair pass live in
// the wave's LDS slice; every pair pass is a dense loop over all j (at ~128 particles each j is one
// broadcast LDS read, cheaper than keeping a cell list).
//
// Forward: K FIRE steps with the rules of fire_batched (velocity and force in real units, drift applied to
// R as (dt V + dt^2/2 F) / L, no convergence test), recording in a caller-owned HBM workspace, for every
// state k, the positions u_k and forces F_k, the pre-mixing velocity w_k of every step and the step's
// scalars (dt, alpha, |w|, |F'|, P > 0).  Reverse: the steps are transposed from k = K-1 down to 0 with
// cotangents Rb (of R), Vb (of V) and Fb (of the force of the state being processed):
//   mixing (P > 0):  c = (F_k+1 . Vb) / fn;  wb = (1 - a) Vb + a c w / vn;  Fb += a vn (Vb - c F_k+1 / fn) / fn
//   kick:            Fb += dt/2 wb
//   force at R_k+1:  Rb += L (dF/dx) Fb;  parameter cotangents += Fb . dF/dtheta     (one pair pass)
//   drift:           g_lnc -= Rb . (R_k+1 - R_k);  Vb = wb + dt Rb / L;  Fb = dt/2 wb + dt^2/2 Rb / L
// with (dF/dx z)_i = -sum_j [ (u'/r) z_ij + (u'' - u'/r)(rhat . z_ij) rhat ],  z_ij = z_i - z_j, and per
// ordered pair of species (a, c): dF/dsigma_ac . z += -1/2 du'/dsigma rhat . z_ij, dF/deps_ac . z +=
// -1/2 (u'/eps) rhat . z_ij, dF/dln c . z += -1/2 u'' r rhat . z_ij (box scaled at fixed R).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

namespace {

constexpr int kUW = 4;          // replicas (wavefronts) per workgroup
constexpr int kUMaxN = 256;     // particles per replica
constexpr int kUS = 4;          // species
constexpr int kRec = 5;         // doubles per step record: dt, alpha, |w|, |F'|, P > 0
constexpr int kAcc = 2 * kUS * kUS;
constexpr int kNb = 32;         // candidate partners per particle kept for one pair pass

struct UPot {
    int kind, S, alpha_is_2, shift;
    float alpha, rc2, rc, pad;
    float sig[kUS * kUS], eps[kUS * kUS], inv_eps[kUS * kUS];
    float ushift[kUS * kUS], ushift_s[kUS * kUS];  // LJ: u(r_c) and its sigma derivative when shifted
    double sigd[kUS * kUS];
};

struct UWave {
    UPot pot;  // the replica's pair table (sigma may differ per replica)
    uint32_t u[kUMaxN][2];
    float z[kUMaxN][2];
    int8_t sp[kUMaxN];
    uint8_t nb[kUMaxN][kNb];  // candidate partners of each particle in the current pass, ascending
    double acc[kAcc];         // sigma entries, then eps entries
};

struct ULds {
    UWave w[kUW];
};

struct UnrollArgs {
    int32_t B, K;
    const int32_t *offset;
    const float *box;
    uint32_t *pos;
    const int32_t *species;
    const double *rep_sigma;  // [B][S*S] or null
    uint8_t *ws;
    uint64_t ws_bytes, part_base;  // byte offset of the particle records inside ws
    double *energy, *g_sigma, *g_eps, *g_lnc;
    float *rbar0;
    uint8_t *mixed;
    int32_t *status;
    double dt_start, dt_max, f_inc, f_dec, alpha_start, f_alpha;
    int32_t n_min;
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterfly sum: IEEE addition is commutative, so every lane ends with the same bits.
__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct PairT {
    float dx, dy, r, u1, u2, u1s, u, us;
};

// Pair terms of one ordered pair: u' = du/dr, u'' and du'/dsigma always; u and du/dsigma when WANT_U.
// Soft spheres take the overlap 1 - r/sigma from the double distance, as the other force kernels do.
template <int KIND, bool WANT_U>
__device__ __forceinline__ bool pair_terms(const UPot &p, int pt, const uint32_t *ui, const uint32_t *uj,
                                           const float *s, const double *sd, PairT &o)
{
    int32_t ix = (int32_t)(ui[0] - uj[0]), iy = (int32_t)(ui[1] - uj[1]);
    float dx = (float)ix * s[0], dy = (float)iy * s[1];
    float r2 = __builtin_fmaf(dx, dx, dy * dy);
    if (KIND == 0) {
        if (!(r2 < p.rc2)) return false;
        float eps = p.eps[pt], sig = p.sig[pt];
        float r2i = 1.0f / r2;
        float q = sig * sig * r2i;
        q = q * q * q;
        float r = __builtin_sqrtf(r2), ri = 1.0f / r;
        o.dx = dx;
        o.dy = dy;
        o.r = r;
        o.u1 = -4.0f * eps * ri * (12.0f * q * q - 6.0f * q);
        o.u2 = 4.0f * eps * r2i * (156.0f * q * q - 42.0f * q);
        o.u1s = -4.0f * eps * ri / sig * (144.0f * q * q - 36.0f * q);
        if (WANT_U) {
            o.u = 4.0f * eps * (q * q - q) - p.ushift[pt];
            o.us = 4.0f * eps / sig * (12.0f * q * q - 6.0f * q) - p.ushift_s[pt];
        }
        return true;
    } else {
        float sig = p.sig[pt];
        if (!(r2 < sig * sig * 1.00001f)) return false;
        double dxd = (double)ix * sd[0], dyd = (double)iy * sd[1];
        double rd = __builtin_sqrt(__builtin_fma(dxd, dxd, dyd * dyd));
        double sigd = p.sigd[pt];
        if (!(rd < sigd)) return false;
        float t = (float)((sigd - rd) / sigd);
        float r = (float)rd, eps = p.eps[pt];
        float es = eps / sig, es2 = es / sig;
        float tp1, tp2;  // t^(alpha-1), t^(alpha-2)
        if (p.alpha_is_2) {
            tp1 = t;
            tp2 = 1.0f;
        } else {
            tp1 = __builtin_exp2f((p.alpha - 1.0f) * __builtin_log2f(t));
            tp2 = tp1 / t;
        }
        float am1 = p.alpha - 1.0f;
        o.dx = (float)dxd;
        o.dy = (float)dyd;
        o.r = r;
        o.u1 = -es * tp1;
        o.u2 = es2 * am1 * tp2;
        o.u1s = es2 * tp2 * (t - am1 * r / sig);
        if (WANT_U) {
            o.u = eps / p.alpha * tp1 * t;
            o.us = eps * tp1 * r / (sig * sig);
        }
        return true;
    }
}

template <int P>
struct Own {
    uint32_t u[P][2];
    int sp[P];
    bool on[P];
};

template <int P>
__device__ __forceinline__ void own_load(Own<P> &o, const UWave &W, int n, int lane)
{
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int i = lane + 64 * p;
        o.on[p] = i < n;
        int k = o.on[p] ? i : 0;
        o.u[p][0] = W.u[k][0];
        o.u[p][1] = W.u[k][1];
        o.sp[p] = W.sp[k];
    }
}

// The cheap first test of pair_terms (float distance against the cutoff, with the soft-sphere guard band).
template <int KIND>
__device__ __forceinline__ bool near_pair(const UPot &p, int pt, const uint32_t *ui, const uint32_t *uj,
                                          const float *s)
{
    float dx = (float)(int32_t)(ui[0] - uj[0]) * s[0], dy = (float)(int32_t)(ui[1] - uj[1]) * s[1];
    float r2 = __builtin_fmaf(dx, dx, dy * dy);
    if (KIND == 0) return r2 < p.rc2;
    float sig = p.sig[pt];
    return r2 < sig * sig * 1.00001f;
}

// Calls f(q, j, uj, sj) for every own particle q and every partner j != i_q that passes near_pair, in
// ascending j for each q (the order of a plain loop over j, so sums come out the same).  A cheap scan over all
// j writes each particle's candidates to its LDS row first; the expensive pair terms then run over the rows
// only.  A pass in which some particle has more than kNb candidates runs the plain loop instead.
template <int KIND, int P, class Fn>
__device__ __forceinline__ void wave_pairs(UWave &W, const Own<P> &o, int n, int lane, const float *s, Fn &&f)
{
    const UPot &p = W.pot;
    const int S = p.S;
    int cnt[P];
#pragma unroll
    for (int q = 0; q < P; ++q) cnt[q] = 0;
    for (int j = 0; j < n; ++j) {
        uint32_t uj[2] = {W.u[j][0], W.u[j][1]};
        int sj = W.sp[j];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (o.on[q] && j != lane + 64 * q && near_pair<KIND>(p, o.sp[q] * S + sj, o.u[q], uj, s)) {
                if (cnt[q] < kNb) W.nb[lane + 64 * q][cnt[q]] = (uint8_t)j;
                ++cnt[q];
            }
        }
    }
    bool over = false;
#pragma unroll
    for (int q = 0; q < P; ++q) over |= cnt[q] > kNb;
    if (__any(over)) {
        for (int j = 0; j < n; ++j) {
            uint32_t uj[2] = {W.u[j][0], W.u[j][1]};
            int sj = W.sp[j];
#pragma unroll
            for (int q = 0; q < P; ++q)
                if (o.on[q] && j != lane + 64 * q) f(q, j, uj, sj);
        }
        return;
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < P; ++q) {
        for (int m = 0; __any(m < cnt[q]); ++m) {
            if (m < cnt[q]) {
                int j = W.nb[lane + 64 * q][m];
                uint32_t uj[2] = {W.u[j][0], W.u[j][1]};
                f(q, j, uj, (int)W.sp[j]);
            }
        }
    }
}

// F_i for the wave's own particles at the positions in W.u.
template <int KIND, int P>
__device__ void wave_forces(UWave &W, const Own<P> &o, int n, int lane, const float *s, const double *sd,
                            float (&F)[P][2])
{
    const UPot &p = W.pot;
#pragma unroll
    for (int q = 0; q < P; ++q) F[q][0] = F[q][1] = 0.0f;
    const int S = p.S;
    wave_pairs<KIND, P>(W, o, n, lane, s, [&](int q, int, const uint32_t *uj, int sj) {
        PairT t;
        if (pair_terms<KIND, false>(p, o.sp[q] * S + sj, o.u[q], uj, s, sd, t)) {
            float c = -t.u1 / t.r;
            F[q][0] = __builtin_fmaf(c, t.dx, F[q][0]);
            F[q][1] = __builtin_fmaf(c, t.dy, F[q][1]);
        }
    });
}

// One reverse pair pass at the positions in W.u with the vector z = W.z: jv = (dF/dx) z for the own
// particles, and per own particle the parameter contractions by species of the partner (gs, ge) and the
// box-scale contraction gl.
template <int KIND, int P>
__device__ void wave_adjoint(UWave &W, const Own<P> &o, int n, int lane, const float *s, const double *sd,
                             float (&jv)[P][2], float (&gs)[P][kUS], float (&ge)[P][kUS], float &gl)
{
    const UPot &p = W.pot;
    float zi[P][2];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        int i = o.on[q] ? lane + 64 * q : 0;
        zi[q][0] = W.z[i][0];
        zi[q][1] = W.z[i][1];
        jv[q][0] = jv[q][1] = 0.0f;
#pragma unroll
        for (int c = 0; c < kUS; ++c) gs[q][c] = ge[q][c] = 0.0f;
    }
    gl = 0.0f;
    const int S = p.S;
    wave_pairs<KIND, P>(W, o, n, lane, s, [&](int q, int j, const uint32_t *uj, int sj) {
        PairT t;
        int pt = o.sp[q] * S + sj;
        if (pair_terms<KIND, false>(p, pt, o.u[q], uj, s, sd, t)) {
            float ri = 1.0f / t.r;
            float hx = t.dx * ri, hy = t.dy * ri;
            float z0 = zi[q][0] - W.z[j][0], z1 = zi[q][1] - W.z[j][1];
            float sh = __builtin_fmaf(hx, z0, hy * z1);   // rhat . z_ij
            float a = t.u1 * ri;
            float b = (t.u2 - a) * sh;
            jv[q][0] -= __builtin_fmaf(a, z0, b * hx);
            jv[q][1] -= __builtin_fmaf(a, z1, b * hy);
            float vs = -0.5f * t.u1s * sh;
            float ve = -0.5f * t.u1 * p.inv_eps[pt] * sh;
#pragma unroll
            for (int c = 0; c < kUS; ++c) {
                gs[q][c] += sj == c ? vs : 0.0f;
                ge[q][c] += sj == c ? ve : 0.0f;
            }
            gl = __builtin_fmaf(-0.5f * t.u2 * t.r, sh, gl);
        }
    });
}

// Energy and its own parameter derivatives at the positions in W.u (1/2 per ordered pair).
template <int KIND, int P>
__device__ void wave_energy(UWave &W, const Own<P> &o, int n, int lane, const float *s, const double *sd,
                            float &e, float (&gs)[P][kUS], float (&ge)[P][kUS], float &gl)
{
    const UPot &p = W.pot;
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
        for (int c = 0; c < kUS; ++c) gs[q][c] = ge[q][c] = 0.0f;
    e = gl = 0.0f;
    const int S = p.S;
    wave_pairs<KIND, P>(W, o, n, lane, s, [&](int q, int, const uint32_t *uj, int sj) {
        PairT t;
        int pt = o.sp[q] * S + sj;
        if (pair_terms<KIND, true>(p, pt, o.u[q], uj, s, sd, t)) {
            e += 0.5f * t.u;
#pragma unroll
            for (int c = 0; c < kUS; ++c) {
                gs[q][c] += sj == c ? 0.5f * t.us : 0.0f;
                ge[q][c] += sj == c ? 0.5f * t.u * p.inv_eps[pt] : 0.0f;
            }
            gl = __builtin_fmaf(0.5f * t.u1, t.r, gl);
        }
    });
}

// Adds the wave's per-lane parameter contractions into the replica's double accumulators (lane 0 writes).
template <int P>
__device__ __forceinline__ void fold(UWave &W, const Own<P> &o, int S, int lane, const float (&gs)[P][kUS],
                                     const float (&ge)[P][kUS])
{
    for (int a = 0; a < S; ++a)
        for (int c = 0; c < S; ++c) {
            double vs = 0.0, ve = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                bool m = o.on[q] && o.sp[q] == a;
                vs += m ? (double)gs[q][c] : 0.0;
                ve += m ? (double)ge[q][c] : 0.0;
            }
            vs = wsum(vs);
            ve = wsum(ve);
            if (lane == 0) {
                W.acc[a * S + c] += vs;
                W.acc[kUS * kUS + a * S + c] += ve;
            }
        }
}

template <int KIND, int P>
__global__ __launch_bounds__(64 * kUW) void k_fire_unrolled(UnrollArgs a, UPot pin)
{
    __shared__ ULds L;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = blockIdx.x * kUW + wv;
    if (b >= a.B) return;
    UWave &W = L.w[wv];
    if (lane == 0) W.pot = pin;
    wave_sync();
    const int S = pin.S;
    if (a.rep_sigma && lane < S * S) {
        double sg = a.rep_sigma[(size_t)b * S * S + lane];
        W.pot.sig[lane] = (float)sg;
        W.pot.sigd[lane] = sg;
        if (KIND == 0 && pin.shift) {
            double qc = sg / (double)pin.rc;
            qc = qc * qc * qc;
            qc = qc * qc;
            double ep = (double)pin.eps[lane];
            W.pot.ushift[lane] = (float)(4.0 * ep * (qc * qc - qc));
            W.pot.ushift_s[lane] = (float)(4.0 * ep / sg * (12.0 * qc * qc - 6.0 * qc));
        }
    }
    wave_sync();
    const UPot &pot = W.pot;
    const int off = a.offset[b], n = a.offset[b + 1] - off, K = a.K;
    if (n < 0 || n > 64 * P) {
        if (lane == 0 && a.status) a.status[b] = -1;
        return;
    }
    const uint64_t rec_bytes = (uint64_t)K * kRec * 8;
    const uint64_t part_off = a.part_base + 24ull * (uint64_t)(K + 1) * (uint64_t)off;
    if ((uint64_t)(b + 1) * rec_bytes > a.part_base || part_off + 24ull * (uint64_t)(K + 1) * n > a.ws_bytes) {
        if (lane == 0 && a.status) a.status[b] = -2;
        return;
    }
    double *rec = (double *)(a.ws + (uint64_t)b * rec_bytes);
    uint8_t *part = a.ws + part_off;
    const float Lb[2] = {a.box[2 * b], a.box[2 * b + 1]};
    const float s[2] = {Lb[0] * (1.0f / 4294967296.0f), Lb[1] * (1.0f / 4294967296.0f)};
    const double sd[2] = {(double)Lb[0] / 4294967296.0, (double)Lb[1] / 4294967296.0};
    const double inv_sd[2] = {4294967296.0 / (double)Lb[0], 4294967296.0 / (double)Lb[1]};
    // state k block: u [n][2] uint32, F [n][2] float, w [n][2] float
    auto blk = [&](int k) { return part + 24ull * (uint64_t)n * (uint64_t)k; };

#pragma unroll
    for (int q = 0; q < P; ++q) {
        int i = lane + 64 * q;
        if (i < n) {
            W.u[i][0] = a.pos[2 * (size_t)(off + i)];
            W.u[i][1] = a.pos[2 * (size_t)(off + i) + 1];
            W.sp[i] = a.species ? (int8_t)a.species[off + i] : (int8_t)0;
        }
    }
    if (lane < kAcc) W.acc[lane] = 0.0;
    wave_sync();
    Own<P> o;
    own_load(o, W, n, lane);

    auto store_state = [&](int k, const float (&F)[P][2]) {
        uint8_t *bk = blk(k);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            int i = lane + 64 * q;
            if (o.on[q]) {
                ((uint2 *)bk)[i] = make_uint2(o.u[q][0], o.u[q][1]);
                ((float2 *)(bk + 8ull * n))[i] = make_float2(F[q][0], F[q][1]);
            }
        }
    };

    // ---------------------------------------------------------------- forward
    float V[P][2], F[P][2];
#pragma unroll
    for (int q = 0; q < P; ++q) V[q][0] = V[q][1] = 0.0f;
    wave_forces<KIND, P>(W, o, n, lane, s, sd, F);
    store_state(0, F);
    double dt = a.dt_start, al = a.alpha_start;
    int n_pos = 0;
    for (int k = 0; k < K; ++k) {
        wave_sync();
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double dx = dt * (double)V[q][c] + 0.5 * dt * dt * (double)F[q][c];
                o.u[q][c] += (uint32_t)__double2int_rn(dx * inv_sd[c]);
            }
            int i = lane + 64 * q;
            if (o.on[q]) {
                W.u[i][0] = o.u[q][0];
                W.u[i][1] = o.u[q][1];
            }
        }
        wave_sync();
        float Fn[P][2], w[P][2];
        wave_forces<KIND, P>(W, o, n, lane, s, sd, Fn);
        double Pw = 0.0, vv = 0.0, ff = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                w[q][c] = (float)((double)V[q][c] + 0.5 * dt * ((double)F[q][c] + (double)Fn[q][c]));
                if (o.on[q]) {
                    Pw += (double)Fn[q][c] * (double)w[q][c];
                    vv += (double)w[q][c] * (double)w[q][c];
                    ff += (double)Fn[q][c] * (double)Fn[q][c];
                }
            }
        }
        Pw = wsum(Pw);
        vv = wsum(vv);
        ff = wsum(ff);
        const bool mix = Pw > 0.0;
        const double vn = sqrt(vv), fn = sqrt(ff);
        uint8_t *bw = blk(k);
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (o.on[q]) ((float2 *)(bw + 16ull * n))[lane + 64 * q] = make_float2(w[q][0], w[q][1]);
        store_state(k + 1, Fn);
        if (lane == 0) {
            double *r = rec + (size_t)k * kRec;
            r[0] = dt;
            r[1] = al;
            r[2] = vn;
            r[3] = fn;
            r[4] = mix ? 1.0 : 0.0;
            if (a.mixed) a.mixed[(size_t)b * K + k] = mix ? 1 : 0;
        }
        if (mix) {
            double cv = 1.0 - al, cf = al * vn / fn;
#pragma unroll
            for (int q = 0; q < P; ++q)
#pragma unroll
                for (int c = 0; c < 2; ++c) V[q][c] = (float)(cv * (double)w[q][c] + cf * (double)Fn[q][c]);
            if (++n_pos > a.n_min) {
                dt = fmin(dt * a.f_inc, a.dt_max);
                al *= a.f_alpha;
            }
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) V[q][0] = V[q][1] = 0.0f;
            dt *= a.f_dec;
            al = a.alpha_start;
            n_pos = 0;
        }
#pragma unroll
        for (int q = 0; q < P; ++q) F[q][0] = Fn[q][0], F[q][1] = Fn[q][1];
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        int i = lane + 64 * q;
        if (o.on[q]) {
            a.pos[2 * (size_t)(off + i)] = o.u[q][0];
            a.pos[2 * (size_t)(off + i) + 1] = o.u[q][1];
        }
    }

    // ---------------------------------------------------------------- reverse
    // every lane reads the step records lane 0 wrote
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    wave_sync();
    float gs[P][kUS], ge[P][kUS], gl_l, e_l;
    wave_energy<KIND, P>(W, o, n, lane, s, sd, e_l, gs, ge, gl_l);
    fold(W, o, S, lane, gs, ge);
    double E = wsum((double)e_l);
    double g_lnc = wsum((double)gl_l);
    float Rb[P][2], Vb[P][2], Fb[P][2];
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Rb[q][c] = -Lb[c] * F[q][c];
            Vb[q][c] = Fb[q][c] = 0.0f;
        }
    // data of step k: w_k, F_k+1 and u_k, loaded one step ahead
    float wn[P][2], Fnx[P][2];
    uint32_t un[P][2];
    auto load_step = [&](int k) {
        const uint8_t *bk = blk(k), *bk1 = blk(k + 1);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            int i = o.on[q] ? lane + 64 * q : 0;
            float2 w2 = ((const float2 *)(bk + 16ull * n))[i];
            float2 f2 = ((const float2 *)(bk1 + 8ull * n))[i];
            uint2 u2 = ((const uint2 *)bk)[i];
            wn[q][0] = w2.x;
            wn[q][1] = w2.y;
            Fnx[q][0] = f2.x;
            Fnx[q][1] = f2.y;
            un[q][0] = u2.x;
            un[q][1] = u2.y;
        }
    };
    if (K > 0 && n > 0) load_step(K - 1);
    for (int k = K - 1; k >= 0; --k) {
        const double *r = rec + (size_t)k * kRec;
        const double dt_k = r[0], a_k = r[1], vn = r[2], fn = r[3];
        const bool mix = r[4] != 0.0;
        float wk[P][2], Fk1[P][2];
        uint32_t uk[P][2];
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                wk[q][c] = wn[q][c];
                Fk1[q][c] = Fnx[q][c];
                uk[q][c] = un[q][c];
            }
        if (k > 0) load_step(k - 1);
        float wb[P][2];
        if (mix) {
            double cl = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q)
                if (o.on[q]) cl += (double)Fk1[q][0] * Vb[q][0] + (double)Fk1[q][1] * Vb[q][1];
            const double c = wsum(cl) / fn;
            const float c1 = (float)(1.0 - a_k), c2 = (float)(a_k * c / vn);
            const float c3 = (float)(a_k * vn / fn), c4 = (float)(c / fn);
#pragma unroll
            for (int q = 0; q < P; ++q)
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    wb[q][x] = __builtin_fmaf(c1, Vb[q][x], c2 * wk[q][x]);
                    Fb[q][x] = __builtin_fmaf(c3, Vb[q][x] - c4 * Fk1[q][x], Fb[q][x]);
                }
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) wb[q][0] = wb[q][1] = 0.0f;
        }
        const float hdt = (float)(0.5 * dt_k);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            Fb[q][0] = __builtin_fmaf(hdt, wb[q][0], Fb[q][0]);
            Fb[q][1] = __builtin_fmaf(hdt, wb[q][1], Fb[q][1]);
            if (o.on[q]) {
                W.z[lane + 64 * q][0] = Fb[q][0];
                W.z[lane + 64 * q][1] = Fb[q][1];
            }
        }
        wave_sync();
        float jv[P][2];
        wave_adjoint<KIND, P>(W, o, n, lane, s, sd, jv, gs, ge, gl_l);
        fold(W, o, S, lane, gs, ge);
        double gd = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                Rb[q][c] = __builtin_fmaf(Lb[c], jv[q][c], Rb[q][c]);
                if (o.on[q]) gd += (double)Rb[q][c] * (double)(int32_t)(o.u[q][c] - uk[q][c]);
            }
        }
        g_lnc += wsum((double)gl_l) - wsum(gd) * (1.0 / 4294967296.0);
        const float fdt = (float)dt_k, hdt2 = (float)(0.5 * dt_k * dt_k);
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float rl = Rb[q][c] / Lb[c];
                Vb[q][c] = __builtin_fmaf(fdt, rl, wb[q][c]);
                Fb[q][c] = __builtin_fmaf(hdt2, rl, hdt * wb[q][c]);
            }
        // the next pass is at state k
        wave_sync();
#pragma unroll
        for (int q = 0; q < P; ++q) {
            o.u[q][0] = uk[q][0];
            o.u[q][1] = uk[q][1];
            if (o.on[q]) {
                W.u[lane + 64 * q][0] = uk[q][0];
                W.u[lane + 64 * q][1] = uk[q][1];
            }
        }
    }
    // the force of R_0
#pragma unroll
    for (int q = 0; q < P; ++q)
        if (o.on[q]) {
            W.z[lane + 64 * q][0] = Fb[q][0];
            W.z[lane + 64 * q][1] = Fb[q][1];
        }
    wave_sync();
    {
        float jv[P][2];
        wave_adjoint<KIND, P>(W, o, n, lane, s, sd, jv, gs, ge, gl_l);
        fold(W, o, S, lane, gs, ge);
        g_lnc += wsum((double)gl_l);
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int c = 0; c < 2; ++c) Rb[q][c] = __builtin_fmaf(Lb[c], jv[q][c], Rb[q][c]);
    }
    wave_sync();
    if (a.rbar0) {
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (o.on[q]) {
                size_t g = (size_t)(off + lane + 64 * q);
                a.rbar0[2 * g] = Rb[q][0];
                a.rbar0[2 * g + 1] = Rb[q][1];
            }
    }
    if (lane < S * S) {
        a.g_sigma[(size_t)b * S * S + lane] = W.acc[lane];
        a.g_eps[(size_t)b * S * S + lane] = W.acc[kUS * kUS + lane];
    }
    if (lane == 0) {
        a.energy[b] = E;
        a.g_lnc[b] = g_lnc;
        if (a.status) a.status[b] = 1;
    }
}

bool make_upot(const md_potential *pot, UPot &u)
{
    if (!pot || (pot->kind != MD_LJ && pot->kind != MD_SOFT_SPHERE)) return false;
    int S = pot->n_species;
    if (S < 1 || S > kUS) return false;
    u = UPot{};
    u.kind = pot->kind;
    u.S = S;
    u.alpha = pot->alpha;
    u.alpha_is_2 = pot->alpha == 2.0f;
    if (pot->kind == MD_SOFT_SPHERE && !(pot->alpha >= 1.0f)) return false;
    if (pot->kind == MD_LJ && !(pot->r_cut > 0.0f)) return false;
    u.rc2 = pot->r_cut * pot->r_cut;
    u.rc = pot->r_cut;
    u.shift = pot->kind == MD_LJ && pot->shift;
    for (int q = 0; q < S * S; ++q) {
        double sg = pot->sigma[q], ep = pot->epsilon[q];
        int qt = (q % S) * S + q / S;
        if (!(sg > 0.0) || !(ep > 0.0) || sg != pot->sigma[qt] || ep != pot->epsilon[qt]) return false;
        u.sig[q] = (float)sg;
        u.sigd[q] = sg;
        u.eps[q] = (float)ep;
        u.inv_eps[q] = (float)(1.0 / ep);
        if (pot->kind == MD_LJ && pot->shift) {
            double qc = pow(sg / pot->r_cut, 6.0);
            u.ushift[q] = (float)(4.0 * ep * (qc * qc - qc));
            u.ushift_s[q] = (float)(4.0 * ep / sg * (12.0 * qc * qc - 6.0 * qc));
        }
    }
    return true;
}

uint64_t rec_region(int32_t B, int32_t K)
{
    uint64_t r = (uint64_t)B * (uint64_t)K * kRec * 8;
    return (r + 255) / 256 * 256;
}

}  // namespace

extern "C" {

uint64_t fire_unrolled_workspace_bytes(int32_t B, int64_t total_n, int32_t K)
{
    if (B < 0 || total_n < 0 || K < 0) return 0;
    return rec_region(B, K) + 24ull * (uint64_t)(K + 1) * (uint64_t)total_n;
}

md_status fire_unrolled_grad(md_ctx *ctx, const md_batch *bt, const md_potential *pot, const double *sigma,
                             const md_fire_params *fp, int32_t K, void *workspace, uint64_t workspace_bytes, double *energy, double *g_sigma,
                             double *g_eps, double *g_lnc, float *rbar0, uint8_t *mixed, int32_t *status,
                             void *stream)
{
    if (!ctx || !bt || !pot || !fp || bt->B < 0 || bt->dim != 2 || K < 0) return MD_ERR_ARG;
    if (bt->B > 0 && (!bt->offset || !bt->box || !bt->pos || !workspace || !energy || !g_sigma || !g_eps ||
                      !g_lnc))
        return MD_ERR_ARG;
    UPot up;
    if (!make_upot(pot, up)) return MD_ERR_ARG;
    if (pot->n_species > 1 && !bt->species) return MD_ERR_ARG;
    if (bt->max_n < 0 || bt->max_n > kUMaxN) return MD_ERR_CAPACITY;
    if (bt->B == 0) return MD_OK;
    if (workspace_bytes < rec_region(bt->B, K)) return MD_ERR_CAPACITY;
    HIP_OK(hipSetDevice(ctx->device));
    UnrollArgs a{};
    a.B = bt->B;
    a.K = K;
    a.offset = bt->offset;
    a.box = bt->box;
    a.pos = bt->pos;
    a.species = bt->species;
    a.rep_sigma = sigma;
    a.ws = (uint8_t *)workspace;
    a.ws_bytes = workspace_bytes;
    a.part_base = rec_region(bt->B, K);
    a.energy = energy;
    a.g_sigma = g_sigma;
    a.g_eps = g_eps;
    a.g_lnc = g_lnc;
    a.rbar0 = rbar0;
    a.mixed = mixed;
    a.status = status;
    a.dt_start = fp->dt_start;
    a.dt_max = fp->dt_max;
    a.f_inc = fp->f_inc;
    a.f_dec = fp->f_dec;
    a.alpha_start = fp->alpha_start;
    a.f_alpha = fp->f_alpha;
    a.n_min = fp->n_min;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((bt->B + kUW - 1) / kUW), block(64 * kUW);
    int P = bt->max_n <= 64 ? 1 : (bt->max_n <= 128 ? 2 : 4);
    if (pot->kind == MD_LJ) {
        if (P == 1) k_fire_unrolled<0, 1><<<grid, block, 0, st>>>(a, up);
        else if (P == 2) k_fire_unrolled<0, 2><<<grid, block, 0, st>>>(a, up);
        else k_fire_unrolled<0, 4><<<grid, block, 0, st>>>(a, up);
    } else {
        if (P == 1) k_fire_unrolled<1, 1><<<grid, block, 0, st>>>(a, up);
        else if (P == 2) k_fire_unrolled<1, 2><<<grid, block, 0, st>>>(a, up);
        else k_fire_unrolled<1, 4><<<grid, block, 0, st>>>(a, up);
    }
    HIP_OK(hipGetLastError());
    return MD_OK;
}

}  // extern "C"
