// gfx950 kernels of the short-range MD path and the C ABI that launches them.
//
//   lanes          every per-particle kernel gives a particle W lanes (W = nl->lanes, 1..8):
//                  the lanes split the particle's neighbor list (and, when building it,
//                  its stencil candidates) and meet again through __shfl_xor.  With one
//                  lane per particle a 256k-particle system is only ~4k waves, too few to
//                  hide gather latency on 256 CUs; W = 4 gives ~16k.
//   neighbor list  ELL with W interleaved sub-rows: entry t of lane l of particle i lives at
//                  idx[(t*N + i)*W + l], lane l's length at count[i*W + l].  A lane walks the
//                  stencil cells in a fixed order and takes every W-th candidate, so rows are
//                  deterministic.  A float filter with a guard band decides most pairs, the
//                  defining double expression the rest (Sec. 3.2.3).
//   cell list      fixed-capacity bins: bin c holds up to M (index, position) members.
//                  A standalone build fills them by a counting sort (integer counts, an
//                  atomics-free exclusive scan in LDS, placement, members ordered by index).
//                  Inside a Verlet run the bins are refreshed without atomics: one wave per
//                  cell gathers, from the previous bins of its stencil cells, the particles
//                  whose cell it now is (ballot compaction keeps the order deterministic).
//   forces         neighbor positions are uint32 torus coordinates whose integer difference
//                  is the nearest image exactly (Sec. 3.2.1).
//   velocity Verlet one regular launch per step.  A rebuild is pipelined over the next two
//                  step launches (bins, then rows of a second list generation) while forces
//                  keep using the current list; it starts when a particle's displacement plus
//                  twice its last step would exceed skin/2 (Sec. 3.1), and every step checks
//                  that the list it uses is still valid.  No grid barrier, no host round trip.
//   FIRE           per step: mix + drift, a counting-sort rebuild gated on the device (its
//                  launches return at once unless a particle moved more than skin/2), forces
//                  with per-workgroup double partial sums, and a one-workgroup reduction that
//                  applies the FIRE rules in a fixed order.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <type_traits>

#include "../../include/md.h"
#include "md_device.h"
#include "md_host.h"

using namespace md;

// ------------------------------------------------------------------------------------------------
// argument blocks

// Bin c holds cnt[c] <= M member records {u_x, u_y, u_z (0 in 2D), index} of 16 bytes at mem[(c*M + k)*4].
struct Bins {
    int32_t *cnt;   // [C]
    uint32_t *mem;  // [C][M][4]
};

// Member record `slot` (a 32-bit byte offset from the bin base; bins stay below 4 GiB).
__device__ __forceinline__ uint4 rec16(const uint32_t *mem, uint32_t slot)
{
    return *(const uint4 *)((const char *)mem + slot * 16u);
}

// Buffer resource over `bytes` bytes at `base` (raw addressing: loads at byte offsets at or past `bytes` return
// 0 and stores there are dropped, instead of touching memory).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <int D>
__device__ __forceinline__ void store_rec(uint32_t *mem, uint32_t slot, const uint32_t *u, int j)
{
    uint4 r;
    r.x = u[0];
    r.y = u[1];
    r.z = D == 3 ? u[D - 1] : 0u;
    r.w = (uint32_t)j;
    *(uint4 *)(mem + (size_t)slot * 4) = r;
}

struct ListGen {
    int32_t *idx;       // [cap/W][N][W]
    int32_t *count;     // [N][W]
    uint32_t *pos_ref;  // [N][D]
};

struct ListParams {
    int32_t N, cap, W, capW, M;
    int32_t seg;             // 0, or particles per independent system (cells of system s are s*C .. s*C + C-1)
    int32_t cells;           // cells of the list (C per system times the systems of a segmented list)
    int32_t pk;              // 1: candidates are tested on packed 16-bit coordinates (isotropic boxes)
    int32_t pk_lo, pk_hi;    // packed test: R16 < pk_lo is a neighbor, R16 >= pk_hi is not, else the double test
    float rl2f_lo, rl2f_hi;  // float guard band around r_list^2
    double rl2;              // (double)r_list * (double)r_list
    float half_skin;         // skin / 2
    uint32_t reach[3];       // skin / 2 with a margin, in torus units per axis (how far a particle can be from its record)
    float kappa;             // pipelined rebuild starts when disp + kappa * (last step + dt^2 |F|) > skin/2
};


// Running row lengths a building wave keeps in LDS: one per member of a bin (bins hold at most 252).
constexpr int kMaxPerCellPad = 256;
// Predicates of the lane-mask compare builtins (LLVM's numbering).
constexpr int kFCmpOLT = 4, kFCmpOLE = 5, kICmpNE = 33, kICmpSGE = 39, kICmpSLT = 40;

enum { M_IDLE = 0, M_BIN = 1, M_BUILD = 2 };
// Control words (device).  Verlet: ctl[2*slot] = mode and ctl[2*slot+1] = generation of step s at
// slot s % 3, written by workgroup 0 of step s-1; ctl[6 + slot] = rebuild request for step s, written
// by any workgroup of step s-1; ctl[kGenWord] = generation to use after the last step that ran.
// FIRE: ctl[kTrigWord] = rebuild needed before this step's forces.
// (kCtlWords and kTrigWord come from md_host.h)
constexpr int kGenWord = 9;

// Raise *addr to v.  Every workgroup calls this with its own maximum; atomics on one address from thousands
// of workgroups serialize (~0.1 us each), so only a workgroup that exceeds the value already there issues one.
__device__ __forceinline__ void raise_max(int32_t *addr, int v)
{
    if (v > __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(addr, v);
}

// Set *addr = 1 when any lane of the wave has cond (one store per wave instead of one per lane).
__device__ __forceinline__ void wave_flag(bool cond, int32_t *addr)
{
    uint64_t m = __ballot(cond);
    if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) *addr = 1;
}

__device__ __forceinline__ int wrapc(int c, int n)
{
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

// Block index remapped so that the workgroups one XCD receives (round-robin over 8 XCDs) own one
// contiguous range of particles: neighbor gathers then mostly hit that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    if ((nb & 7) != 0) return bid;
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

__device__ __forceinline__ bool gate_closed(const int32_t *gate)
{
    return gate != nullptr && *gate == 0;
}

// Stencil cell number t (0 .. nst-1) around cell (cx, cy, cz), in z-major, then y, then x order.
template <int D>
__device__ __forceinline__ int stencil_cell(const DevBox &b, int cx, int cy, int cz, int t)
{
    int n0 = b.hi[0] - b.lo[0] + 1, n1 = b.hi[1] - b.lo[1] + 1;
    int x = wrapc(cx + b.lo[0] + t % n0, b.nc[0]);
    int y = wrapc(cy + b.lo[1] + (t / n0) % n1, b.nc[1]);
    int z = 0;
    if constexpr (D == 3) z = wrapc(cz + b.lo[2] + t / (n0 * n1), b.nc[2]);
    return x + b.nc[0] * (y + b.nc[1] * z);
}

template <int D>
__device__ __forceinline__ int stencil_size(const DevBox &b)
{
    int n = (b.hi[0] - b.lo[0] + 1) * (b.hi[1] - b.lo[1] + 1);
    if constexpr (D == 3) n *= b.hi[2] - b.lo[2] + 1;
    return n;
}

// ------------------------------------------------------------------------------------------------
// counting sort into bins (deterministic); every kernel returns at once when its gate word is 0

template <int D>
__global__ void k_cs_count(const uint32_t *__restrict__ pos, int N, int seg, DevBox b, CountSort cs,
                           const int32_t *gate)
{
    if (gate_closed(gate)) return;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t u[D];
    load_pos<D>(pos, i, u);
    int c = cell_index<D>(u, b) + (seg > 0 ? (i / seg) * b.C : 0);
    cs.cell_of[i] = c;
    cs.slot[i] = atomicAdd(&cs.cell_count[c], 1);  // integer counts: the totals do not depend on order
}

constexpr int kScan = 1024;                 // threads of the one-workgroup scan
constexpr int kScanPer = 16;                // consecutive cells per thread and tile, held in registers
constexpr int kScanTile = kScan * kScanPer;  // cells per tile

// Counts of the kScanPer cells of thread t in the tile at base (zero past C): four 16-byte loads when the thread's
// cells are all below C.
__device__ __forceinline__ void scan_load(const int32_t *cnt, int base, int C, int t, int *v)
{
    const int c0 = base + t * kScanPer;
    if (c0 + kScanPer <= C) {
        const int4 *p = (const int4 *)(cnt + c0);
#pragma unroll
        for (int q = 0; q < kScanPer / 4; ++q) {
            const int4 x = p[q];
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) v[k] = c0 + k < C ? cnt[c0 + k] : 0;
    }
}

// Exclusive scan of cell_count into cell_start[0..C] by one workgroup (wave shuffles and LDS, no atomics); also the
// bin counts min(count, M), the cell-overflow flag and the largest occupancy.  It leaves the counts at zero for the
// next build.  Each thread holds kScanPer adjacent cells of a tile in registers and scans them, the workgroup scans
// the thread sums, and a carry joins the tiles; the next tile's counts are loaded while a tile is scanned.
__global__ __launch_bounds__(kScan) void k_cs_scan(CountSort cs, int C, Bins bins, int M, int32_t *flags,
                                                   int32_t *ok, const int32_t *gate)
{
    __shared__ int wsum[kScan / 64];
    __shared__ int wmax[kScan / 64];
    __shared__ int tile_total;
    if (gate_closed(gate)) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int carry = 0, mx = 0;
    int cur[kScanPer];
    scan_load(cs.cell_count, 0, C, t, cur);
    for (int base = 0; base < C; base += kScanTile) {
        int nxt[kScanPer];
        if (base + kScanTile < C) {
            scan_load(cs.cell_count, base + kScanTile, C, t, nxt);
        } else {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) nxt[k] = 0;
        }
        int local = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            local += cur[k];
            mx = max(mx, cur[k]);
        }
        int incl = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        if (w == 0) {
            const int x = lane < kScan / 64 ? wsum[lane] : 0;
            int xi = x;
#pragma unroll
            for (int o = 1; o < kScan / 64; o <<= 1) {
                const int v = __shfl_up(xi, o);
                if (lane >= o) xi += v;
            }
            if (lane < kScan / 64) wsum[lane] = xi - x;
            if (lane == kScan / 64 - 1) tile_total = xi;
        }
        __syncthreads();
        int run = carry + incl - local + wsum[w];
        const int c0 = base + t * kScanPer;
        int st[kScanPer], bc[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            st[k] = run;
            bc[k] = min(cur[k], M);
            run += cur[k];
        }
        if (c0 + kScanPer <= C) {
#pragma unroll
            for (int q = 0; q < kScanPer / 4; ++q) {
                ((int4 *)(cs.cell_start + c0))[q] = make_int4(st[4 * q], st[4 * q + 1], st[4 * q + 2], st[4 * q + 3]);
                ((int4 *)(cs.cell_count + c0))[q] = make_int4(0, 0, 0, 0);  // ready for the next build
                ((int4 *)(bins.cnt + c0))[q] = make_int4(bc[4 * q], bc[4 * q + 1], bc[4 * q + 2], bc[4 * q + 3]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) {
                if (c0 + k < C) {
                    cs.cell_start[c0 + k] = st[k];
                    cs.cell_count[c0 + k] = 0;
                    bins.cnt[c0 + k] = bc[k];
                }
            }
        }
        carry += tile_total;
        __syncthreads();  // the next tile overwrites wsum and tile_total
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) cur[k] = nxt[k];
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) mx = max(mx, __shfl_xor(mx, o));
    if (lane == 0) wmax[w] = mx;
    __syncthreads();
    if (w == 0) {
        int m2 = lane < kScan / 64 ? wmax[lane] : 0;
#pragma unroll
        for (int o = 1; o < kScan / 64; o <<= 1) m2 = max(m2, __shfl_xor(m2, o));
        if (lane == 0) {
            raise_max(&flags[MD_FLAG_MAXCELL], m2);
            if (m2 > M) flags[MD_FLAG_CELL_OVERFLOW] = 1;
            *ok = m2 <= M ? 1 : 0;  // the bins are complete (the rows may still overflow)
            cs.cell_start[C] = carry;
        }
    }
}

__global__ void k_cs_place(CountSort cs, int N, const int32_t *gate)
{
    if (gate_closed(gate)) return;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < N) cs.sorted_idx[cs.cell_start[cs.cell_of[i]] + cs.slot[i]] = i;
}

// Bin records in index order without sorting: particle i's rank in its cell is the number of members with a
// smaller index, which makes the bins (and so the rows built from them) deterministic.  A particle that does not
// fit its bin (the cell-overflow flag is raised) gets empty sub-rows, so no row length is left undefined.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cs_rank_fill(const uint32_t *__restrict__ pos, int N, CountSort cs,
                                                         Bins bins, int M, int32_t *count, int W, const int32_t *gate)
{
    if (gate_closed(gate)) return;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    int c = cs.cell_of[i];
    int s = cs.cell_start[c], e = cs.cell_start[c + 1];
    int rank = 0;
    for (int a = s; a < e; ++a) rank += cs.sorted_idx[a] < i ? 1 : 0;
    if (rank < M) {
        uint32_t u[D];
        load_pos<D>(pos, i, u);
        store_rec<D>(bins.mem, (uint32_t)(c * M + rank), u, i);
    } else {
        for (int l = 0; l < W; ++l) count[(size_t)i * W + l] = 0;
    }
}

// ------------------------------------------------------------------------------------------------
// neighbor rows (Sec. 3.2.3): one wave per cell
//
// A wave takes one cell c at a time.  The candidates of every particle of c are the same: the members of c's stencil
// cells, numbered in stencil order (x fastest, then y, then z) and then in bin order.  The wave holds up to
// kSlots x 64 of them in registers, one per lane and slot, and walks the particles of c one after the other, the
// particle's own record in scalar registers.  Per particle and slot the test is a few vector instructions whose
// comparison writes a lane mask directly; accepted candidates are numbered in sequence order by counting the mask
// bits of the lanes below (mbcnt) and dealt round-robin to the W interleaved sub-rows (neighbor n to sub-row n % W at
// position n / W), so rows are deterministic and the W lanes that later walk a row differ by at most one entry.
//
// Filter.  In a box with one scale along every axis the candidate test runs on the upper 16 bits of each torus
// coordinate, two coordinates packed per register: a packed 16-bit subtraction wraps modulo 2^16, which is the
// nearest image in units of u = L / 2^16, and a 16-bit dot product with 32-bit saturating accumulation gives
// R16 = sum d_k^2.  With e_k the exact displacement in units of u, |d_k - e_k| < 1 while |e_k| < 32767, so
// |R16 - R| < 2 sqrt(D R) + D for R = sum e_k^2.  ListParams.pk_lo / pk_hi bound that error around
// T = r_list^2 / u^2 (host, double): R16 < pk_lo means the pair is in the list, R16 >= pk_hi that it is not, and
// the rare candidates in between take the defining double expression.  Other boxes use single-precision
// displacements with a relative guard band of 1e-5 around r_list^2, again with the double expression in the band.

// Candidates a wave holds at once are NS x 64 (registers per lane: about 5 per slot).  The standalone build holds 8
// slots with the packed filter; the step kernel holds 4, which keeps it within the registers of its force loop.

__device__ __forceinline__ uint32_t pack_hi16(uint32_t a, uint32_t b)
{
    return (a >> 16) | (b & 0xffff0000u);
}

// R16 of a packed candidate (cxy, cz) against the particle's packed (pxy, pz): two wrapping 16-bit subtractions and
// two saturating 16-bit dot products.  cz / pz hold z in 3D and 0 in 2D, and the candidate's spare component (the
// upper half in 3D, the lower half in 2D) marks a lane past the last candidate.
__device__ __forceinline__ int r2_packed(uint32_t cxy, uint32_t cz, uint32_t pxy, uint32_t pz)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    typedef short i16x2 __attribute__((ext_vector_type(2)));
    const u16x2 dxy = __builtin_bit_cast(u16x2, cxy) - __builtin_bit_cast(u16x2, pxy);
    const u16x2 dz = __builtin_bit_cast(u16x2, cz) - __builtin_bit_cast(u16x2, pz);
    const int r2 = __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, dxy), __builtin_bit_cast(i16x2, dxy), 0, true);
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, dz), __builtin_bit_cast(i16x2, dz), r2, true);
}

// Sub-row length of lane l for a row of n entries dealt round-robin over W sub-rows.
template <int W>
__device__ __forceinline__ int sub_count(int n, int l)
{
    return (n + W - 1 - l) / W;
}

// Rows of every particle of cell gc (a global cell number: system gc / C of a segmented list, cell gc % C in it)
// from the bins, by the calling wave.  ncnt is the wave's LDS array of running row lengths (used when the stencil
// holds more candidates than the wave's slots).  Returns the longest row of the cell.
template <int D, int W, bool PK, int NS, bool SMALL_ROWS, bool SPARSE>
__device__ int build_cell(int gc, const DevBox &b, const Bins &bins, const ListParams &lp, int32_t *__restrict__ idx,
                          int32_t *__restrict__ count, int *ncnt)
{
    const int lane = threadIdx.x & 63;
    const int sys = gc / b.C, c = gc - sys * b.C, cbase = sys * b.C;
    const int cx = c % b.nc[0], cy = (c / b.nc[0]) % b.nc[1], cz = D == 3 ? c / (b.nc[0] * b.nc[1]) : 0;
    const int nst = stencil_size<D>(b);
    const int n0 = b.hi[0] - b.lo[0] + 1, n1 = b.hi[1] - b.lo[1] + 1;
    const int tc = -b.lo[0] + n0 * (-b.lo[1] + n1 * (D == 3 ? -b.lo[2] : 0));  // the cell itself in stencil order
    // candidate order: the cell's own members first, then the other stencil cells in stencil order, each in bin
    // order; entry u of the table is stencil cell tc for u = 0, else the (u-1)-th of the others
    int src = 0, m = 0;
    if (lane < nst) {
        const int t = lane == 0 ? tc : (lane - 1 < tc ? lane - 1 : lane);
        src = cbase + stencil_cell<D>(b, cx, cy, cz, t);
        m = bins.cnt[src];
    }
    int incl = m;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    const int excl = incl - m;
    const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, nst - 1));
    const int mc = __builtin_amdgcn_readfirstlane(m);  // members of the cell itself (entry 0, lane 0)
    if (mc == 0) return 0;
    const uint32_t M = (uint32_t)lp.M;
    const uint32_t row_bytes = (uint32_t)lp.N * W * 4u;  // bytes between positions t and t+1 of a sub-row
    // list entries through a range-checked buffer: an entry past the capacity (position >= capacity / W) lies past
    // the end of the array, and the store is dropped (N * capacity * 4 < 2^32, checked on the host)
    const __amdgpu_buffer_rsrc_t ridx = raw_rsrc(idx, (uint32_t)lp.N * (uint32_t)lp.cap * 4u);
    const bool iso = b.iso != 0;
    const float s2 = b.s[0] * b.s[0];
    const float flo = iso ? lp.rl2f_lo / s2 : lp.rl2f_lo, fhi = iso ? lp.rl2f_hi / s2 : lp.rl2f_hi;
    // record slot of candidate q (every lane runs it: a lane reads another lane's register through a shuffle only
    // while that lane is active); slot 0, always mapped, past the last candidate
    auto locate = [&](int q) -> uint32_t {
        int t = 0;
#pragma unroll
        for (int st = 16; st > 0; st >>= 1) {
            const int cand = t + st;
            const int e = __shfl(excl, cand < nst ? cand : nst - 1);
            if (cand < nst && e <= q) t = cand;
        }
        const int t_src = __shfl(src, t), t_ex = __shfl(excl, t);
        return q < total ? (uint32_t)t_src * M + (uint32_t)(q - t_ex) : 0u;
    };
    // packed test: a lane whose spare 16-bit component holds -32768 has R16 >= 2^30, above pk_hi for every
    // particle, so it never passes and never enters the uncertain band; it marks lanes past the last candidate
    constexpr uint32_t kMark = D == 3 ? 0x80000000u : 0x8000u;
    int longest = 0;
    for (int base = 0; base < total; base += NS * 64) {
        const bool last_batch = base + NS * 64 >= total;
        // slots that hold candidates (a sparse system fills one or two of them): the rest are neither loaded nor tested
        const int nslots = min(NS, (total - base + 63) >> 6);
        uint32_t ca[NS], cb[NS], cc[NS];
        int cj[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = base + s * 64 + lane;
            const uint4 r = !SPARSE || nslots == NS || s < nslots ? rec16(bins.mem, locate(q))
                                                                 : make_uint4(0u, 0u, 0u, 0u);
            const bool ok = q < total;
            cj[s] = ok ? (int)r.w : -1;
            if constexpr (PK) {
                ca[s] = pack_hi16(r.x, r.y);
                cb[s] = (D == 3 ? (r.z >> 16) : 0u) | (ok ? 0u : kMark);
                cc[s] = 0u;
            } else {
                ca[s] = r.x;
                cb[s] = r.y;
                cc[s] = r.z;
            }
            // at most four records in flight: the slots' registers, not the loads, set the register budget
            if (s % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
        uint4 rn = rec16(bins.mem, (uint32_t)gc * M);
        for (int p = 0; p < mc; ++p) {
            const uint4 ri = rn;
            rn = rec16(bins.mem, (uint32_t)gc * M + (uint32_t)min(p + 1, mc - 1));  // the next member's record
            const uint32_t ui[3] = {(uint32_t)__builtin_amdgcn_readfirstlane(ri.x),
                                    (uint32_t)__builtin_amdgcn_readfirstlane(ri.y),
                                    (uint32_t)__builtin_amdgcn_readfirstlane(ri.z)};
            const int i = __builtin_amdgcn_readfirstlane((int)ri.w);
            const uint32_t pxy = pack_hi16(ui[0], ui[1]), pz = D == 3 ? ui[2] >> 16 : 0u;
            const uint32_t iw4 = (uint32_t)i * W * 4u;
            int n = base > 0 ? __builtin_amdgcn_readfirstlane(ncnt[p]) : 0;
            // the particle itself is the one candidate with its own index.  The slots are tested in three passes so
            // that the filter of every slot is one straight run of independent instructions: the filter (lane masks
            // of every slot), then the double-precision recheck of the rare undecided candidates, then the stores in
            // sequence order.  FULL: every slot is tested, with no slot-count branches (a slot or lane past the last
            // candidate holds no accepted and no undecided candidate).  Otherwise (SPARSE builds with a partly used
            // batch) only the used slots are loaded and tested: the standalone build serves sparse systems (2D
            // packings, boids) with one or two of its eight slots in use, while the step kernel's dense cells fill
            // its four.
            auto test_slots = [&](auto full_tag) {
                constexpr bool FULL = decltype(full_tag)::value;
                uint64_t acc[NS], band[NS];
                uint64_t any_band = 0;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    acc[s] = band[s] = 0;
                    if (!FULL && s >= nslots) break;
                    // lane masks straight from the compares: acc = surely in the list, band = undecided by the filter
                    if constexpr (PK) {
                        const int r2 = r2_packed(ca[s], cb[s], pxy, pz);
                        const uint64_t lo = __builtin_amdgcn_sicmp(r2, lp.pk_lo, kICmpSLT);
                        const uint64_t hi = __builtin_amdgcn_sicmp(r2, lp.pk_hi, kICmpSLT);
                        const uint64_t other = __builtin_amdgcn_sicmp(cj[s], i, kICmpNE);
                        acc[s] = lo & other;
                        band[s] = hi & ~lo & other;
                    } else {
                        const uint32_t uj[3] = {ca[s], cb[s], cc[s]};
                        float r2 = 0.0f;
#pragma unroll
                        for (int z = 0; z < D; ++z) {
                            const float d = iso ? (float)(int32_t)(ui[z] - uj[z]) : tdisp(ui[z], uj[z], b.s[z]);
                            r2 = __builtin_fmaf(d, d, r2);
                        }
                        const uint64_t ok = __builtin_amdgcn_sicmp(cj[s], 0, kICmpSGE) &
                                            __builtin_amdgcn_sicmp(cj[s], i, kICmpNE);
                        const uint64_t lo = __builtin_amdgcn_fcmpf(r2, flo, kFCmpOLT) & ok;
                        const uint64_t hi = __builtin_amdgcn_fcmpf(r2, fhi, kFCmpOLE) & ok;
                        acc[s] = lo;
                        band[s] = hi & ~lo;
                    }
                    any_band |= band[s];
                }
                // candidates near r_list take the defining double expression (rare: the whole wave skips this)
                if (any_band != 0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        if (!FULL && s >= nslots) break;
                        if (band[s] == 0) continue;
                        const uint32_t slot = locate(base + s * 64 + lane);  // the full record (PK kept 16 bits)
                        bool take = false;
                        if (__builtin_amdgcn_inverse_ballot_w64(band[s])) {
                            uint32_t uj[3] = {ca[s], cb[s], cc[s]};
                            if constexpr (PK) {
                                const uint4 r = rec16(bins.mem, slot);
                                uj[0] = r.x;
                                uj[1] = r.y;
                                uj[2] = r.z;
                            }
                            double r2d = 0.0;
#pragma unroll
                            for (int z = 0; z < D; ++z) {
                                const double d = tdisp_d(ui[z], uj[z], b.sd[z]);
                                r2d = __dadd_rn(r2d, __dmul_rn(d, d));
                            }
                            take = r2d < lp.rl2;
                        }
                        acc[s] |= __builtin_amdgcn_ballot_w64(take);
                    }
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!FULL && s >= nslots) break;
                    if (__builtin_amdgcn_inverse_ballot_w64(acc[s])) {
                        // entry k = n + (accepted lanes below this one) goes to sub-row k % W at position k / W:
                        // (k / W) row_bytes + (k % W) 4 + 4 W i = (k / W) (row_bytes - 4 W) + 4 k + 4 W i
                        const uint32_t k = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(acc[s] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)acc[s], (uint32_t)n));
                        const uint32_t k4 = (k << 2) + iw4;
                        const uint32_t off = SMALL_ROWS ? __umul24(k / W, row_bytes - 4u * W) + k4
                                                        : k / W * (row_bytes - 4u * W) + k4;
                        __builtin_amdgcn_raw_buffer_store_b32(cj[s], ridx, off, 0, 0);
                    }
                    n += __popcll(acc[s]);
                }
            };
            if (!SPARSE || nslots == NS)
                test_slots(std::integral_constant<bool, true>());
            else
                test_slots(std::integral_constant<bool, false>());
            if (!last_batch) {
                if (lane == 0) ncnt[p] = n;
            } else {
                if (lane < W) count[(size_t)i * W + lane] = sub_count<W>(n, lane);
                longest = max(longest, n);
            }
        }
    }
    return longest;
}

// Cells of the list handed to the waves of a launch: wave w (blocks remapped so that one XCD's workgroups are one
// contiguous range) takes cells w, w + nwaves, ...  The longest row and the overflow flag go to flags.
template <int D, int W, bool PK, int NS, bool SPARSE>
__device__ __forceinline__ void build_rows_cells(const DevBox &b, const Bins &bins, const ListParams &lp,
                                                 int32_t *__restrict__ idx, int32_t *__restrict__ count,
                                                 int32_t *flags, int32_t *ok, int *ncnt_all, int *red)
{
    const int wave = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int nwaves = gridDim.x * (kBlock / 64);
    int *ncnt = ncnt_all + (threadIdx.x >> 6) * kMaxPerCellPad;
    int longest = 0;
    if ((uint64_t)lp.N * W * 4u < (1u << 24)) {  // row stride fits the 24-bit multiplier
        for (int gc = wave; gc < lp.cells; gc += nwaves)
            longest = max(longest, build_cell<D, W, PK, NS, true, SPARSE>(gc, b, bins, lp, idx, count, ncnt));
    } else {
        for (int gc = wave; gc < lp.cells; gc += nwaves)
            longest = max(longest, build_cell<D, W, PK, NS, false, SPARSE>(gc, b, bins, lp, idx, count, ncnt));
    }
    wave_flag(longest > lp.cap, &flags[MD_FLAG_OVERFLOW]);
    if (ok != nullptr && longest > lp.cap) *ok = 0;  // rare: only a wave with a row that did not fit stores
    longest = block_max(longest, red);
    if (threadIdx.x == 0) raise_max(&flags[MD_FLAG_MAXCOUNT], (longest + W - 1) / W * W);
}

// Standalone build: rows of every particle from the bins, and pos_ref = the positions they were built from.
template <int D, int W, bool PK>
__global__ __launch_bounds__(kBlock) void k_build_rows(const uint32_t *__restrict__ pos, DevBox b, Bins bins,
                                                       ListParams lp, ListGen g, int32_t *flags, int32_t *ok,
                                                       const int32_t *gate)
{
    __shared__ int ncnt[(kBlock / 64) * kMaxPerCellPad];
    __shared__ int red[kBlock];
    if (gate_closed(gate)) return;
    build_rows_cells<D, W, PK, PK ? 8 : 4, true>(b, bins, lp, g.idx, g.count, flags, ok, ncnt, red);
    for (int q = blockIdx.x * kBlock + threadIdx.x; q < lp.N * D; q += gridDim.x * kBlock) g.pos_ref[q] = pos[q];
    if (threadIdx.x == 0 && blockIdx.x == 0) flags[MD_FLAG_REBUILDS] += 1;
}

// ------------------------------------------------------------------------------------------------
// standalone build for sparsely filled cells: one particle per W lanes
//
// With a few particles per cell (a 2D packing or a flock, two to three per cell), a wave per cell holds one slot of
// candidates and walks two or three particles, so the cell's set-up and its chain of loads are the whole cost.
// Giving every particle its own W lanes keeps the machine full instead.

// Stencil table of particle i at reference position ui: the stencil cells that can hold a neighbor, in stencil
// order, packed as (cell << 8) | count at tab[e * ts].  A cell is left out when its slab distance from the particle
// (the distance to the faces it lies beyond) already exceeds r_list, or when it is empty.  Every lane of the
// particle computes the table; only lanes with `write` store it.  Returns the number of entries; `chunks` receives
// the number of 4-record chunks they hold.
template <int D>
__device__ __forceinline__ int stencil_table(int i, const uint32_t *ui, const DevBox &b, const Bins &bins,
                                             const ListParams &lp, uint32_t *tab, int ts, bool write, int &chunks)
{
    constexpr int NST = D == 3 ? 27 : 9;
    int cc[3][3];
    float lo2[3], hi2[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        cc[q][0] = cc[q][1] = cc[q][2] = 0;
        lo2[q] = hi2[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const uint64_t pr = (uint64_t)ui[q] * (uint64_t)b.nc[q];
        const int c = (int)(pr >> 32);
        const float f = (float)(uint32_t)pr * 2.3283064365386963e-10f;  // position within the cell, [0, 1)
        const float dl = f * b.cw[q], dh = (1.0f - f) * b.cw[q];
        lo2[q] = dl * dl;
        hi2[q] = dh * dh;
        cc[q][0] = wrapc(c - 1, b.nc[q]);
        cc[q][1] = c;
        cc[q][2] = wrapc(c + 1, b.nc[q]);
    }
    const int cbase = lp.seg > 0 ? (i / lp.seg) * b.C : 0;  // first cell of the particle's system
    // a cell whose slab distance exceeds r_list (with the float guard band above it) holds no neighbor
    const float cull2 = lp.rl2f_hi;
    int cell[NST], m[NST];
#pragma unroll
    for (int t = 0; t < NST; ++t) {
        const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = D == 3 ? t / 9 - 1 : 0;
        bool use = ox >= b.lo[0] && ox <= b.hi[0] && oy >= b.lo[1] && oy <= b.hi[1];
        if (D == 3) use = use && oz >= b.lo[2] && oz <= b.hi[2];
        const float g = (ox < 0 ? lo2[0] : ox > 0 ? hi2[0] : 0.0f) + (oy < 0 ? lo2[1] : oy > 0 ? hi2[1] : 0.0f) +
                        (oz < 0 ? lo2[2] : oz > 0 ? hi2[2] : 0.0f);
        use = use && g <= cull2;
        cell[t] = cbase + cc[0][ox + 1] + b.nc[0] * (cc[1][oy + 1] + b.nc[1] * cc[2][oz + 1]);
        m[t] = use ? bins.cnt[cell[t]] : 0;
    }
    int ne = 0;
    chunks = 0;
#pragma unroll
    for (int t = 0; t < NST; ++t) {
        if (m[t] > 0) {
            if (write) tab[ne * ts] = ((uint32_t)cell[t] << 8) | (uint32_t)m[t];
            ++ne;
            chunks += (m[t] + 3) >> 2;
        }
    }
    return ne;
}

// Inclusive prefix sum of x over the W lanes of a particle (W <= 8: the groups lie within DPP rows of 16 lanes),
// by DPP row shifts; tot = the group's sum.  Every lane of a group is active together.
template <int W>
__device__ __forceinline__ int group_scan(int x, int l, int &tot)
{
    int incl = x;
    if constexpr (W >= 2) {
        const int v = __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);  // row_shr:1
        incl += l >= 1 ? v : 0;
    }
    if constexpr (W >= 4) {
        const int v = __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);  // row_shr:2
        incl += l >= 2 ? v : 0;
    }
    if constexpr (W >= 8) {
        const int v = __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);  // row_shr:4
        incl += l >= 4 ? v : 0;
    }
    if constexpr (W == 1) tot = incl;
    else if constexpr (W == 2) tot = __builtin_amdgcn_update_dpp(0, incl, 0xF5, 0xf, 0xf, false);  // quad_perm 1,1,3,3
    else if constexpr (W == 4) tot = __builtin_amdgcn_update_dpp(0, incl, 0xFF, 0xf, 0xf, false);  // quad_perm 3,3,3,3
    else tot = __shfl(incl, W - 1, W);
    return incl;
}

// A lane's place in the stencil table's chunk sequence: entry e, chunk c within it, the entry's first slot cb and
// member count mc; `have` is false past the last chunk.
struct ChunkCursor {
    int e, c, mc;
    uint32_t cb;
    bool have;
};

// The four records of a chunk as separate registers.
struct Chunk4 {
    uint32_t x[4], y[4], z[4], j[4];
};

// The cursor's chunk, W chunks on (entries of the table are ts words apart).
template <int W>
__device__ __forceinline__ ChunkCursor chunk_next(ChunkCursor k, const uint32_t *tab, int ts, int ne, uint32_t M)
{
    k.c += W;
    if (k.have) {
        while (true) {
            const int nch = (k.mc + 3) >> 2;
            if (k.c < nch) break;
            k.c -= nch;
            ++k.e;
            if (k.e >= ne) {
                k.have = false;
                break;
            }
            const uint32_t en = tab[k.e * ts];
            k.mc = (int)(en & 255u);
            k.cb = (en >> 8) * M;
        }
    }
    return k;
}

// Loads the cursor's chunk (a cursor past the end reads slot 0, always mapped).
__device__ __forceinline__ void chunk_load(const ChunkCursor &k, const uint32_t *mem, Chunk4 &r)
{
    const uint4 *p = (const uint4 *)mem + (k.have ? k.cb + 4u * (uint32_t)k.c : 0u);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = p[q];
        r.x[q] = v.x;
        r.y[q] = v.y;
        r.z[q] = v.z;
        r.j[q] = v.w;
    }
}

// Row of particle i (Sec. 3.2.3) built by its W lanes from its stencil table.  The listed cells' records form one
// sequence of 4-record chunks; lane l tests chunks l, l + W, ..., loading its next chunk while it tests the current
// one.  Candidates are tested in float against a guard band around r_list^2; those inside the band take the double
// expression that defines the list.  Accepted neighbors are numbered in sequence order (a prefix sum over the W
// lanes after each round) and dealt round-robin to the interleaved sub-rows.  Returns the row length (the same in
// every lane of the particle; it may exceed the capacity, and only the first `cap` entries are stored).
template <int D, int W>
__device__ __forceinline__ int build_row(int i, int l, const uint32_t *ui, const DevBox &b, const Bins &bins,
                                         const ListParams &lp, int32_t *__restrict__ idx, const uint32_t *tab, int ts,
                                         int ne, int chunks)
{
    const uint32_t M = (uint32_t)lp.M;
    const uint32_t row_bytes = (uint32_t)lp.N * W * 4u;  // bytes between positions t and t+1 of a sub-row
    const bool iso = b.iso != 0;
    const float s2 = b.s[0] * b.s[0];
    const float lo = iso ? lp.rl2f_lo / s2 : lp.rl2f_lo, hi = iso ? lp.rl2f_hi / s2 : lp.rl2f_hi;
    ChunkCursor ka{0, l, 0, 0u, false};
    while (ka.e < ne) {
        const uint32_t en = tab[ka.e * ts];
        ka.mc = (int)(en & 255u);
        const int nch = (ka.mc + 3) >> 2;
        if (ka.c < nch) {
            ka.cb = (en >> 8) * M;
            ka.have = true;
            break;
        }
        ka.c -= nch;
        ++ka.e;
    }
    int n = 0;
    auto test = [&](const Chunk4 &r, const ChunkCursor &k) {
        int bits = 0, band = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t uj[3] = {r.x[q], r.y[q], r.z[q]};
            float r2 = 0.0f;
            if (iso) {
#pragma unroll
                for (int z = 0; z < D; ++z) {
                    const float d = (float)(int32_t)(ui[z] - uj[z]);
                    r2 = __builtin_fmaf(d, d, r2);
                }
            } else {
#pragma unroll
                for (int z = 0; z < D; ++z) {
                    const float d = tdisp(ui[z], uj[z], b.s[z]);
                    r2 = __builtin_fmaf(d, d, r2);
                }
            }
            bits |= r2 < lo ? 1 << q : 0;
            band |= r2 >= lo && r2 <= hi ? 1 << q : 0;
        }
        // candidates within the guard band (rare) take the defining double expression; the branch is taken by the
        // whole wave or not at all
        if (__ballot(band != 0) != 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (band & (1 << q)) {
                    const uint32_t uj[3] = {r.x[q], r.y[q], r.z[q]};
                    double r2d = 0.0;
#pragma unroll
                    for (int z = 0; z < D; ++z) {
                        const double d = tdisp_d(ui[z], uj[z], b.sd[z]);
                        r2d = __dadd_rn(r2d, __dmul_rn(d, d));
                    }
                    bits |= r2d < lp.rl2 ? 1 << q : 0;
                }
            }
        }
        // records of the chunk that are members (a cell's last chunk may be partial), other than i itself
        const int left = k.have ? k.mc - 4 * k.c : 0;
        bits &= left >= 4 ? 15 : (1 << max(left, 0)) - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) bits &= (int)r.j[q] != i ? 15 : ~(1 << q);
        const int a = __popc(bits);
        int tot;
        const int incl = group_scan<W>(a, l, tot);
        uint32_t slot = (uint32_t)(n + incl - a);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (bits & (1 << q)) {
                if (slot < (uint32_t)lp.cap) {
                    // byte offset of entry slot (below 4 GiB, checked on the host)
                    const uint32_t off = slot / W * row_bytes + ((uint32_t)i * W + slot % W) * 4u;
                    *(int32_t *)((char *)idx + off) = (int)r.j[q];
                }
                ++slot;
            }
        }
        n += tot;
    };
    const int iters = (chunks + W - 1) / W;  // the same in every lane of the particle
    Chunk4 A, B;
    chunk_load(ka, bins.mem, A);
    int it = 0;
    for (; it + 2 <= iters; it += 2) {
        const ChunkCursor kb = chunk_next<W>(ka, tab, ts, ne, M);
        chunk_load(kb, bins.mem, B);
        test(A, ka);
        ka = chunk_next<W>(kb, tab, ts, ne, M);
        chunk_load(ka, bins.mem, A);
        test(B, kb);
    }
    if (it < iters) test(A, ka);
    return n;
}

// Standalone build for sparse cells: rows of every particle from the bins, W lanes per particle, and pos_ref = the
// positions the rows were built from.
template <int D, int W>
__global__ __launch_bounds__(kBlock) void k_build_rows_pp(const uint32_t *__restrict__ pos, DevBox b, Bins bins,
                                                          ListParams lp, ListGen g, int32_t *flags, int32_t *ok,
                                                          const int32_t *gate)
{
    constexpr int TS = kBlock / W;
    __shared__ uint32_t tab[(D == 3 ? 27 : 9) * TS];
    __shared__ int red[kBlock];
    if (gate_closed(gate)) return;
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / W, l = gt % W;
    const bool live = i < lp.N;
    uint32_t ui[D];
    int ne = 0, chunks = 0, n = 0;
    if (live) {
        load_pos<D>(pos, i, ui);
        ne = stencil_table<D>(i, ui, b, bins, lp, tab + threadIdx.x / W, TS, l == 0, chunks);
    }
    __syncthreads();
    if (live) {
        n = build_row<D, W>(i, l, ui, b, bins, lp, g.idx, tab + threadIdx.x / W, TS, ne, chunks);
        g.count[(size_t)i * W + l] = sub_count<W>(n, l);
        if (l == 0) store_pos<D>(g.pos_ref, i, ui);
    }
    wave_flag(n > lp.cap, &flags[MD_FLAG_OVERFLOW]);
    if (ok != nullptr && n > lp.cap) *ok = 0;  // rare: only a particle whose row did not fit stores
    n = block_max(n, red);
    if (threadIdx.x == 0) {
        raise_max(&flags[MD_FLAG_MAXCOUNT], (n + W - 1) / W * W);
        if (blockIdx.x == 0) flags[MD_FLAG_REBUILDS] += 1;
    }
}

// ------------------------------------------------------------------------------------------------
// in-run bin refresh (no atomics): one wave per cell

// Gather, from the previous bins of cell c's stencil, the members whose cell at the current positions `pos` is c.
// The stencil's candidates are numbered in stencil order, then previous bin order, and handed out 64 at a time to the
// wave's lanes.  A previous member's record holds its position at the last build, and no particle is farther than
// skin/2 from it (a step that finds one farther raises the stale flag, and the run stops), so along each axis it can
// now be only in the cells of its recorded coordinate -+ reach (ListParams.reach: skin/2 with a margin, in torus
// units).  Candidates that cannot be in c are dropped from their records alone; the rest are queued in LDS in
// sequence order and tested against their current positions in one pass of independent loads (ballot compaction
// keeps the order).  q is the wave's LDS queue of kMaxPerCellPad entries.
template <int D>
__device__ int bin_gather(const uint32_t *__restrict__ pos, const DevBox &b, const ListParams &lp, const Bins &prev,
                          const Bins &next, int32_t *flags, int wave, int nwaves, int *queue)
{
    const int lane = threadIdx.x & 63;
    const int nst = stencil_size<D>(b);
    const uint32_t M = (uint32_t)lp.M;
    int mymax = 0;
    for (int c = wave; c < b.C; c += nwaves) {
        const int cc[3] = {c % b.nc[0], (c / b.nc[0]) % b.nc[1], D == 3 ? c / (b.nc[0] * b.nc[1]) : 0};
        int src = 0, m = 0;
        if (lane < nst) {
            src = stencil_cell<D>(b, cc[0], cc[1], cc[2], lane);
            m = prev.cnt[src];
        }
        int incl = m;
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        const int excl = incl - m;
        const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, nst - 1));
        int cnt = 0, queued = 0;
        // members of the queue: tested at their current positions and written in queue order
        auto flush = [&]() {
            for (int base = 0; base < queued; base += 64) {
                const int e = base + lane;
                bool take = false;
                int j = 0;
                uint32_t u[D];
                if (e < queued) {
                    j = queue[e];
                    load_pos<D>(pos, j, u);
                    take = cell_index<D>(u, b) == c;
                }
                const uint64_t mask = __ballot(take);
                const int slot = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                if (take && slot < (int)M) store_rec<D>(next.mem, (uint32_t)(c * (int)M + slot), u, j);
                cnt += __popcll(mask);
            }
            queued = 0;
        };
        // four batches of 64 candidates at a time: their record loads are issued together
        for (int base = 0; base < total; base += 4 * 64) {
            uint4 r[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int q = base + h * 64 + lane;
                // stencil cell holding candidate q: the largest t with excl_t <= q
                int t = 0;
#pragma unroll
                for (int st = 16; st > 0; st >>= 1) {
                    const int cand = t + st;
                    const int e = __shfl(excl, cand < nst ? cand : nst - 1);
                    if (cand < nst && e <= q) t = cand;
                }
                // the shuffles run in every lane: a lane reads another lane's register only while that lane is active
                const int t_src = __shfl(src, t), t_ex = __shfl(excl, t);
                r[h] = rec16(prev.mem, q < total ? (uint32_t)t_src * M + (uint32_t)(q - t_ex) : 0u);
            }
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int q = base + h * 64 + lane;
                bool may = q < total;
                const uint32_t w[3] = {r[h].x, r[h].y, r[h].z};
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int lo = cell_coord(w[k] - lp.reach[k], b.nc[k]);
                    const int hi = cell_coord(w[k] + lp.reach[k], b.nc[k]);
                    may = may && (lo == cc[k] || hi == cc[k]);
                }
                const uint64_t mask = __ballot(may);
                if (may) queue[queued + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))] =
                    (int)r[h].w;
                queued += __popcll(mask);
                if (queued > kMaxPerCellPad - 64) flush();
            }
        }
        flush();
        if (lane == 0) {
            next.cnt[c] = min(cnt, (int)M);
            if (cnt > (int)M) flags[MD_FLAG_CELL_OVERFLOW] = 1;  // one store per overflowing cell
        }
        mymax = max(mymax, cnt);
    }
    return mymax;
}

// ------------------------------------------------------------------------------------------------
// forces

// Byte-offset loads from a uniform base: the offsets are 32-bit (the host keeps every array below 4 GiB),
// so the address is one scalar base plus one vector register.
template <typename T>
__device__ __forceinline__ T ld_off(const void *base, uint32_t off)
{
    return *(const T *)((const char *)base + off);
}

// Position of particle j through a range-checked buffer load: an index read from past the end of a row (a stale
// or never written entry) cannot fault.  j < 2^24 for real entries (checked on the host).
template <int D>
__device__ __forceinline__ void ld_pos(const __amdgpu_buffer_rsrc_t &rp, int j, uint32_t *u)
{
    const uint32_t off = __umul24((uint32_t)j & 0xffffffu, (uint32_t)(4 * D));
    if constexpr (D == 3) {
        auto v = __builtin_amdgcn_raw_buffer_load_b96(rp, off, 0, 0);
        u[0] = v[0];
        u[1] = v[1];
        u[2] = v[2];
    } else {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(rp, off, 0, 0);
        u[0] = v[0];
        u[1] = v[1];
    }
}

// Species of particle j through a range-checked buffer load (0 for an index past the array).
__device__ __forceinline__ int ld_species(const __amdgpu_buffer_rsrc_t &rs, int j)
{
    return __builtin_amdgcn_raw_buffer_load_b32(rs, ((uint32_t)j & 0xffffffu) << 2, 0, 0);
}

// Four pairs of one lane: positions pc of neighbors jc against ui; `live` masks slots past the row's end.  With
// ISO (LJ in a box with one scale s along every axis) the displacement stays in integer units: r^2 is their
// squared sum times s^2, and the caller multiplies the summed force by s once.
template <int D, int KIND, bool MULTI, bool MASK, bool ISO>
__device__ __forceinline__ void quad_force(const DevBox &b, const DevPot &p, int si, const uint32_t *ui,
                                           const int *sc, const uint32_t (*pc)[D], int t0, int n, float s2, float *F)
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float d[D], r2, u, fs;
        int pt = MULTI ? si * p.S + sc[a] : 0;
        if constexpr (ISO) {
            float r2u = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                d[k] = (float)(int32_t)(ui[k] - pc[a][k]);
                r2u = __builtin_fmaf(d[k], d[k], r2u);
            }
            r2 = r2u * s2;
            fs = pair_fs<KIND, MULTI, false>(p, pt, r2, u);
        } else {
            fs = pair_eval<D, KIND, MULTI, false>(p, pt, ui, pc[a], b.s, b.sd, d, r2, u);
        }
        if (MASK) fs = t0 + a < n ? fs : 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
    }
}

// Lane l's sub-row of particle i: entries go in groups of four, two groups per iteration with the register sets
// alternating; the indices two groups ahead and the neighbor positions one group ahead are loaded while a group
// is evaluated.  An entry's address is a scalar row base (the same in every lane, clamped to the list's last row)
// plus the lane's own offset, so the loads carry no per-lane address arithmetic.  Rows are clamped to tlast, the
// last entry any lane of the wave needs, so prefetches past it re-read cached lines; entries past a lane's own
// row end may hold anything, their positions come through the range-checked load and their slots are masked.
template <int D, int KIND, bool MULTI, int W, bool ISO>
__device__ __forceinline__ void lane_force_rows(const DevBox &b, const DevPot &p, const __amdgpu_buffer_rsrc_t &rp,
                                                const __amdgpu_buffer_rsrc_t &rs, int N, int tlast,
                                                const int32_t *__restrict__ idx, int n, int i, int l,
                                                const uint32_t *ui, int si, float *F)
{
    const uint32_t step = (uint32_t)N * W * 4u;  // bytes between consecutive entries of a sub-row
    const uint32_t off = ((uint32_t)i * W + (uint32_t)l) * 4u;
    const float s2 = b.s[0] * b.s[0];
    // the row's byte offset goes in the load's scalar offset; the lane's offset is the only vector operand
    const __amdgpu_buffer_rsrc_t ri = raw_rsrc(idx, (uint32_t)(tlast + 1) * step);
    auto ldj = [&](int t) -> int {
        return __builtin_amdgcn_raw_buffer_load_b32(ri, off, (uint32_t)min(t, tlast) * step, 0);
    };
    int jA[4], jB[4];
    uint32_t pA[4][D], pB[4][D];
    int sA[4] = {0, 0, 0, 0}, sB[4] = {0, 0, 0, 0};  // species, loaded with the positions (two or more species)
    // a neighbor's position and species; a slot past the row's end comes through the range-checked loads
    auto ld_nb = [&](int j, uint32_t *pj, int &sj) {
        ld_pos<D>(rp, j, pj);
        if constexpr (MULTI) sj = ld_species(rs, j);
    };
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        jA[a] = ldj(a);
        jB[a] = ldj(4 + a);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) ld_nb(jA[a], pA[a], sA[a]);
    int t = 0;
    // full pairs of groups: A holds group t/4 (positions loaded), B the next group's indices
    for (; t + 8 <= n; t += 8) {
        int jC[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) ld_nb(jB[a], pB[a], sB[a]);
#pragma unroll
        for (int a = 0; a < 4; ++a) jC[a] = ldj(t + 8 + a);
        asm volatile("" ::: "memory");  // keep the loads above ahead of the arithmetic below
        quad_force<D, KIND, MULTI, false, ISO>(b, p, si, ui, sA, pA, t, n, s2, F);
#pragma unroll
        for (int a = 0; a < 4; ++a) ld_nb(jC[a], pA[a], sA[a]);
#pragma unroll
        for (int a = 0; a < 4; ++a) jA[a] = ldj(t + 12 + a);
        asm volatile("" ::: "memory");
        quad_force<D, KIND, MULTI, false, ISO>(b, p, si, ui, sB, pB, t + 4, n, s2, F);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            int x = jA[a];
            jA[a] = jC[a];
            jB[a] = x;
        }
    }
    // at most two groups remain: A (positions loaded) and B (indices loaded)
    if (t < n) {
#pragma unroll
        for (int a = 0; a < 4; ++a) ld_nb(jB[a], pB[a], sB[a]);
        quad_force<D, KIND, MULTI, true, ISO>(b, p, si, ui, sA, pA, t, n, s2, F);
        if (t + 4 < n) quad_force<D, KIND, MULTI, true, ISO>(b, p, si, ui, sB, pB, t + 4, n, s2, F);
    }
    if constexpr (ISO) {
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] *= b.s[0];
    }
}

// Force from lane l's sub-row of particle i (the hot loop), then summed over the W lanes.
template <int D, int KIND, bool MULTI, int W>
__device__ __forceinline__ void lane_force(const DevBox &b, const DevPot &p, const uint32_t *__restrict__ pos,
                                           const int32_t *__restrict__ species, int N, int capW,
                                           const int32_t *__restrict__ idx, int n, int i, int l, const uint32_t *ui,
                                           int si, float *F)
{
    const __amdgpu_buffer_rsrc_t rp = raw_rsrc(pos, (uint32_t)N * 4u * D);
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(species, MULTI ? (uint32_t)N * 4u : 0u);
    // last entry of the longest sub-row in the wave (every lane of the wave calls this), never past the list
    int nw = n;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nw = max(nw, __shfl_xor(nw, o));
    // (scalar instructions on purpose: the compiler otherwise keeps tlast in a vector register and turns every
    // entry load below into 64-bit vector address arithmetic)
    int tlast;
    asm volatile("s_min_i32 %0, %1, %2\n\ts_add_i32 %0, %0, -1"
                 : "=s"(tlast)
                 : "s"(__builtin_amdgcn_readfirstlane(nw)), "s"(__builtin_amdgcn_readfirstlane(capW))
                 : "scc");
    if (n > 0) {
        if (KIND == 0 && b.iso)
            lane_force_rows<D, KIND, MULTI, W, KIND == 0>(b, p, rp, rs, N, tlast, idx, n, i, l, ui, si, F);
        else
            lane_force_rows<D, KIND, MULTI, W, false>(b, p, rp, rs, N, tlast, idx, n, i, l, ui, si, F);
    }
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] += __shfl_xor(F[q], o);
    }
}

// Forces (and optionally e_i, w_i) over a list: one thread per particle walks all W sub-rows.
template <int D, int KIND, bool MULTI, bool WANT_EW>
__global__ __launch_bounds__(kBlock) void k_pair_nl(DevBox b, DevPot p, const uint32_t *__restrict__ pos,
                                                     const int32_t *__restrict__ species, int N,
                                                     const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ count, int W, int capW,
                                                     float *__restrict__ force, double *__restrict__ energy,
                                                     double *__restrict__ virial, int32_t *flags)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < N) {
        uint32_t ui[D];
        load_pos<D>(pos, i, ui);
        int si = MULTI ? species[i] : 0;
        float F[D];
#pragma unroll
        for (int q = 0; q < D; ++q) F[q] = 0.0f;
        double e = 0.0, w = 0.0;
        for (int l = 0; l < W; ++l) {
            int n = min(count[(size_t)i * W + l], capW);  // an overflowed sub-row holds its first capW entries
            for (int t = 0; t < n; ++t) {
                int j = idx[((size_t)t * N + i) * W + l];
                uint32_t uj[D];
                load_pos<D>(pos, j, uj);
                float d[D], r2, u = 0.0f;
                int pt = MULTI ? si * p.S + species[j] : 0;
                float fs = pair_eval<D, KIND, MULTI, WANT_EW>(p, pt, ui, uj, b.s, b.sd, d, r2, u);
#pragma unroll
                for (int q = 0; q < D; ++q) F[q] = __builtin_fmaf(fs, d[q], F[q]);
                if (WANT_EW) {
                    e += (double)u;
                    w += (double)(fs * r2);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < D; ++q) bad = bad || !isfinite(F[q]);
        if (force) {
#pragma unroll
            for (int q = 0; q < D; ++q) force[(size_t)i * D + q] = F[q];
        }
        if (WANT_EW) {
            if (energy) energy[i] = 0.5 * e;
            if (virial) virial[i] = 0.5 * w;
        }
    }
    wave_flag(bad, &flags[MD_FLAG_NONFINITE]);
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
                float d[D], r2, u = 0.0f;
                int pt = MULTI ? si * p.S + tsp[jj] : 0;
                float fs = pair_eval<D, KIND, MULTI, WANT_EW>(p, pt, ui, &tile[jj * D], b.s, b.sd, d, r2, u);
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
    bool bad = false;
    if (live) {
#pragma unroll
        for (int q = 0; q < D; ++q) bad = bad || !isfinite(F[q]);
        if (force) {
#pragma unroll
            for (int q = 0; q < D; ++q) force[(size_t)i * D + q] = F[q];
        }
        if (WANT_EW) {
            if (energy) energy[i] = 0.5 * e;
            if (virial) virial[i] = 0.5 * w;
        }
    }
    wave_flag(bad, &flags[MD_FLAG_NONFINITE]);
}

// ------------------------------------------------------------------------------------------------
// velocity Verlet

// Shift (Sec. 3.2.1) by a real displacement: add its nearest whole number of 2^-32 L units (wraps mod 2^32).
// Value q of up to three by selects (no dynamic indexing, no address taken).
template <int D, typename T>
__device__ __forceinline__ T pick(int q, T v0, T v1, T v2)
{
    if constexpr (D == 3) return q == 0 ? v0 : (q == 1 ? v1 : v2);
    else return q == 0 ? v0 : v1;
}

__device__ __forceinline__ uint32_t shift_coord(uint32_t u, float dx, float inv_s)
{
    return u + (uint32_t)__float2int_rn(dx * inv_s);
}

template <int D>
__device__ __forceinline__ float disp2(const uint32_t *a, const uint32_t *__restrict__ ref, int i, const DevBox &b)
{
    float r2 = 0.0f;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        float d = tdisp(a[q], ref[(size_t)i * D + q], b.s[q]);
        r2 = __builtin_fmaf(d, d, r2);
    }
    return r2;
}

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): the counter c is replaced by the output block.
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(m0, c[0]), lo0 = m0 * c[0];
        uint64_t hi1 = __umul64hi(m1, c[2]), lo1 = m1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += w0;
        k1 += w1;
    }
}

// Four standard normals of particle i at step s: the top 24 bits of each Philox word plus half a unit give a
// uniform in (0, 1), exact in float; Box-Muller turns (u0, u1) and (u2, u3) into normals.
__device__ __forceinline__ void normals4(uint64_t i, uint64_t s, uint64_t seed, float z[4])
{
    uint64_t c[4] = {i, s, 0, 0};
    philox4x64(c, seed, 0);
    float u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = ((float)(uint32_t)(c[q] >> 40) + 0.5f) * (1.0f / 16777216.0f);
    float r0 = sqrtf(-2.0f * logf(u[0])), r1 = sqrtf(-2.0f * logf(u[2]));
    float s0, c0, s1, c1;
    sincospif(2.0f * u[1], &s0, &c0);
    sincospif(2.0f * u[3], &s1, &c1);
    z[0] = r0 * c0;
    z[1] = r0 * s0;
    z[2] = r1 * c1;
    z[3] = r1 * s1;
}

struct StepArgs {
    DevBox box;
    ListParams lp;
    ListGen gen[2];
    Bins bins[2];
    int32_t *flags;
    int32_t *ctl;
    const uint32_t *pos_in;
    uint32_t *pos_out;
    float *vel;
    float *force;
    const int32_t *species;
    float dt;
    int32_t step;  // s >= 1
    int32_t last;  // 1: kick dt/2, store F, no drift
    // Langevin (BAOAB) instead of velocity Verlet when langevin != 0: the drift of a step becomes x += dt/2 v,
    // v = c1 v + c2 xi, x += dt/2 v, with xi the normals of particle i at noise step noise_step[0] + s
    int32_t langevin;
    float c1, c2;
    uint64_t seed;
    const uint64_t *noise_step;
};

// The BAOAB update of one coordinate after the force F of this step: the closing half kick of the last step and
// the opening half kick of this one (two roundings, as the kick and the BAOA launches of the composed step do), the
// friction and noise, and the displacement dt/2 (v_b + v').  Returns the new velocity; dx receives the displacement.
__device__ __forceinline__ float baoab_coord(float v, float F, float dt, float c1, float c2, float z, float &dx)
{
    const float vh = __builtin_fmaf(0.5f * dt, F, v);
    const float vb = __builtin_fmaf(0.5f * dt, F, vh);
    const float vo = __builtin_fmaf(c1, vb, c2 * z);
    dx = 0.5f * dt * (vb + vo);
    return vo;
}

// Control state of step s: {mode, gen} from the previous step's workgroup 0, upgraded to BIN when a
// rebuild was requested.  Workgroup 0 publishes step s+1's words and clears the request slot of s+2.
__device__ __forceinline__ void step_control(int32_t *ctl, int32_t *flags, int s, int &mode, int &gen)
{
    int r = s % 3;
    mode = ctl[2 * r];
    gen = ctl[2 * r + 1];
    if (mode == M_IDLE && ctl[6 + r]) mode = M_BIN;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int nm = mode == M_BIN ? M_BUILD : M_IDLE;
        int ng = mode == M_BUILD ? gen ^ 1 : gen;
        ctl[2 * ((s + 1) % 3)] = nm;
        ctl[2 * ((s + 1) % 3) + 1] = ng;
        ctl[6 + (s + 2) % 3] = 0;
        ctl[kGenWord] = ng;
        flags[MD_FLAG_STEPS] = s;
        if (mode == M_BUILD) flags[MD_FLAG_REBUILDS] += 1;
    }
}

__device__ __forceinline__ bool frozen(const int32_t *flags)
{
    return flags[MD_FLAG_OVERFLOW] | flags[MD_FLAG_CELL_OVERFLOW] | flags[MD_FLAG_STALE];
}

// The rebuild work a step does for the list generation not in use: gather the bins and reference positions of
// the other generation from the positions of this step (BIN), or build its rows from those bins, one wave per cell
// (BUILD).  One XCD's workgroups take one contiguous range of cells in both, so the build finds the bins in its L2.
template <int D, int W>
__device__ __forceinline__ void list_phase(int mode, int gen, const DevBox &box, const ListParams &lp,
                                           const Bins *bins, const ListGen *gens, const uint32_t *pos,
                                           int32_t *flags, int *red, int *ncnt)
{
    if (mode == M_BIN) {
        int wave = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (int)(threadIdx.x >> 6);
        int nwaves = (gridDim.x * kBlock) >> 6;
        int *queue = ncnt + (threadIdx.x >> 6) * kMaxPerCellPad;
        int occ = bin_gather<D>(pos, box, lp, bins[gen], bins[gen ^ 1], flags, wave, nwaves, queue);
        occ = block_max(occ, red);
        if (threadIdx.x == 0) raise_max(&flags[MD_FLAG_MAXCELL], occ);
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < lp.N; i += gridDim.x * kBlock) {
            uint32_t ui[D];
            load_pos<D>(pos, i, ui);
            store_pos<D>(gens[gen ^ 1].pos_ref, i, ui);
        }
    } else if (mode == M_BUILD) {
        const ListGen &g1 = gens[gen ^ 1];
        if (lp.pk)
            build_rows_cells<D, W, true, 4, false>(box, bins[gen ^ 1], lp, g1.idx, g1.count, flags, nullptr, ncnt, red);
        else
            build_rows_cells<D, W, false, 4, false>(box, bins[gen ^ 1], lp, g1.idx, g1.count, flags, nullptr, ncnt, red);
    }
}

// First half kick and drift of a verlet_step call: v += dt/2 F; r(1) = r(0) + dt v; rebuild request for step 1.
template <int D>
__global__ __launch_bounds__(kBlock) void k_verlet_begin(StepArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool req = false;
    if (i < a.lp.N) {
        uint32_t ui[D], un[D];
        float step2 = 0.0f, f2 = 0.0f;
        load_pos<D>(a.pos_in, i, ui);
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (a.langevin) normals4((uint64_t)i, a.noise_step[0], a.seed, z);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            float f = a.force[(size_t)i * D + q];
            float v = __builtin_fmaf(0.5f * a.dt, f, a.vel[(size_t)i * D + q]);
            float dx = a.dt * v;
            if (a.langevin) {
                const float vo = __builtin_fmaf(a.c1, v, a.c2 * z[q]);
                dx = 0.5f * a.dt * (v + vo);
                v = vo;
            }
            a.vel[(size_t)i * D + q] = v;
            un[q] = shift_coord(ui[q], dx, a.box.inv_s[q]);
            step2 = __builtin_fmaf(dx, dx, step2);
            f2 = __builtin_fmaf(f, f, f2);
        }
        store_pos<D>(a.pos_out, i, un);
        float d = sqrtf(disp2<D>(un, a.gen[0].pos_ref, i, a.box));
        float ahead = sqrtf(step2) + a.dt * a.dt * sqrtf(f2);
        req = d + a.lp.kappa * ahead > a.lp.half_skin;
    }
    wave_flag(req, &a.ctl[6 + 1]);
}

// One velocity-Verlet step s >= 1 on r(s): rebuild work if one is in progress, F(s) over the current
// list by W lanes per particle, then v += dt F and r(s+1) = r(s) + dt v (interior step) or
// v += dt/2 F and F stored (last step).
template <int D, int KIND, bool MULTI, int W>
__global__ __launch_bounds__(kBlock) void k_md_step(StepArgs a, DevPot p)
{
    __shared__ int red[kBlock];
    __shared__ int ncnt[(kBlock / 64) * kMaxPerCellPad];
    if (frozen(a.flags)) return;
    int mode, gen;
    step_control(a.ctl, a.flags, a.step, mode, gen);
    const ListParams &lp = a.lp;
    list_phase<D, W>(mode, gen, a.box, lp, a.bins, a.gen, a.pos_in, a.flags, red, ncnt);
    const ListGen &g = a.gen[gen];
    int gt = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    int i = gt / W, l = gt % W;
    bool live = i < lp.N;
    int ii = live ? i : lp.N - 1;  // dead lanes shadow the last particle so the lane reduction stays uniform
    uint32_t ui[D];
    load_pos<D>(a.pos_in, ii, ui);
    bool stale = live && l == 0 && disp2<D>(ui, g.pos_ref, ii, a.box) > lp.half_skin * lp.half_skin;
    wave_flag(stale, &a.flags[MD_FLAG_STALE]);
    int si = MULTI ? a.species[ii] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    int n = live ? min(g.count[(size_t)ii * W + l], lp.capW) : 0;
    lane_force<D, KIND, MULTI, W>(a.box, p, a.pos_in, a.species, lp.N, lp.capW, g.idx, n, ii, l, ui, si, F);
    bool bad = false;
#pragma unroll
    for (int q = 0; q < D; ++q) bad = bad || !isfinite(F[q]);
    wave_flag(live && bad, &a.flags[MD_FLAG_NONFINITE]);
    // The rebuild lookahead measures r(s+1) against the reference positions of the list step s+1 will use: the
    // current one, or after a build step the new one, so that a new rebuild can start right after a switch.
    const uint32_t *ref_next = mode == M_BUILD ? a.gen[gen ^ 1].pos_ref : g.pos_ref;
    if constexpr (W >= D) {
        // every lane of the particle holds the summed force: lane q < D updates coordinate q
        if (!live) return;
        const int q = l < D ? l : 0;
        const float Fq = pick<D>(q, F[0], F[1], F[D - 1]);
        const float sq = pick<D>(q, a.box.s[0], a.box.s[1], a.box.s[2]);
        const float isq = pick<D>(q, a.box.inv_s[0], a.box.inv_s[1], a.box.inv_s[2]);
        const uint32_t uq = pick<D>(q, ui[0], ui[1], ui[D - 1]);
        const size_t at = (size_t)i * D + q;
        float dq2 = 0.0f, st2 = 0.0f, f2q = 0.0f;
        if (l < D) {
            if (a.last) {
                a.vel[at] = __builtin_fmaf(0.5f * a.dt, Fq, a.vel[at]);
                a.force[at] = Fq;
            } else {
                float v, dx;
                if (a.langevin) {
                    float z[4];
                    normals4((uint64_t)i, a.noise_step[0] + (uint64_t)a.step, a.seed, z);
                    v = baoab_coord(a.vel[at], Fq, a.dt, a.c1, a.c2, pick<D>(q, z[0], z[1], z[2]), dx);
                } else {
                    v = __builtin_fmaf(a.dt, Fq, a.vel[at]);
                    dx = a.dt * v;
                }
                a.vel[at] = v;
                const uint32_t un = shift_coord(uq, dx, isq);
                a.pos_out[at] = un;
                const float d = tdisp(un, ref_next[at], sq);
                dq2 = d * d;
                st2 = dx * dx;
                f2q = Fq * Fq;
            }
        }
        if (a.last || mode == M_BIN) return;
        // |r(s+1) - r_ref|^2, |step|^2 and |F|^2 summed over the particle's lanes
#pragma unroll
        for (int o = 1; o < W; o <<= 1) {
            dq2 += __shfl_xor(dq2, o, W);
            st2 += __shfl_xor(st2, o, W);
            f2q += __shfl_xor(f2q, o, W);
        }
        if (l == 0) {
            float ahead = sqrtf(st2) + a.dt * a.dt * sqrtf(f2q);
            if (sqrtf(dq2) + lp.kappa * ahead > lp.half_skin) a.ctl[6 + (a.step + 1) % 3] = 1;
        }
        return;
    }
    if (!live || l != 0) return;
    if (a.last) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            a.vel[(size_t)i * D + q] = __builtin_fmaf(0.5f * a.dt, F[q], a.vel[(size_t)i * D + q]);
            a.force[(size_t)i * D + q] = F[q];
        }
        return;
    }
    uint32_t un[D];
    float step2 = 0.0f, f2 = 0.0f;
    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (a.langevin) normals4((uint64_t)i, a.noise_step[0] + (uint64_t)a.step, a.seed, z);
#pragma unroll
    for (int q = 0; q < D; ++q) {
        float v, dx;
        if (a.langevin) {
            v = baoab_coord(a.vel[(size_t)i * D + q], F[q], a.dt, a.c1, a.c2, z[q], dx);
        } else {
            v = __builtin_fmaf(a.dt, F[q], a.vel[(size_t)i * D + q]);
            dx = a.dt * v;
        }
        a.vel[(size_t)i * D + q] = v;
        un[q] = shift_coord(ui[q], dx, a.box.inv_s[q]);
        step2 = __builtin_fmaf(dx, dx, step2);
        f2 = __builtin_fmaf(F[q], F[q], f2);
    }
    store_pos<D>(a.pos_out, i, un);
    if (mode != M_BIN) {
        float d = sqrtf(disp2<D>(un, ref_next, i, a.box));
        float ahead = sqrtf(step2) + a.dt * a.dt * sqrtf(f2);
        if (d + lp.kappa * ahead > lp.half_skin) a.ctl[6 + (a.step + 1) % 3] = 1;
    }
}

__global__ void k_ctl_init(int32_t *ctl)
{
    int t = threadIdx.x;
    if (t < kCtlWords && t != kListOkWord) ctl[t] = 0;
}

// After a run: if the list in use is the second generation, copy it into the caller's list.
template <int D>
__global__ __launch_bounds__(kBlock) void k_list_finalize(const int32_t *ctl, ListGen dst, ListGen src, ListParams lp)
{
    if (ctl[kGenWord] == 0) return;
    int gt = blockIdx.x * kBlock + threadIdx.x;
    int i = gt / lp.W, l = gt % lp.W;
    if (i >= lp.N) return;
    int n = src.count[(size_t)i * lp.W + l];
    dst.count[(size_t)i * lp.W + l] = n;
    n = min(n, lp.capW);
    for (int t = 0; t < n; ++t) {
        size_t q = ((size_t)t * lp.N + i) * lp.W + l;
        dst.idx[q] = src.idx[q];
    }
    if (l == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) dst.pos_ref[(size_t)i * D + q] = src.pos_ref[(size_t)i * D + q];
    }
}

// After a run: if the list in use is the second generation, its bins become generation 0 (the bins of the list
// now in the caller's arrays), and the list is marked unusable by the next call when the run ended frozen.
__global__ __launch_bounds__(kBlock) void k_bins_finalize(int32_t *ctl, const int32_t *flags, Bins dst, Bins src,
                                                          int C, int M)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && frozen(flags)) ctl[kListOkWord] = 0;
    if (ctl[kGenWord] == 0) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // record slot q = c * M + k
    if (q >= (int64_t)C * M) return;
    const int c = (int)(q / M), k = (int)(q - (int64_t)c * M);
    const int n = src.cnt[c];
    if (k == 0) dst.cnt[c] = n;
    if (k < n) *(uint4 *)(dst.mem + (size_t)q * 4) = *(const uint4 *)(src.mem + (size_t)q * 4);
}

// Start of a verlet_step that may keep the caller's list: raises ctl[kTrigWord] (the gate of a full rebuild) unless
// the list is complete and every particle is within skin/2 of its reference position by a margin of three steps
// of dt |v| + dt^2 |F| (the longest a rebuild requested by the first step can take to replace it).
template <int D>
__global__ __launch_bounds__(kBlock) void k_verlet_check(const uint32_t *__restrict__ pos,
                                                         const float *__restrict__ vel, const float *__restrict__ force,
                                                         const uint32_t *__restrict__ pos_ref, DevBox b, int N,
                                                         float dt, float half_skin, int32_t *ctl)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < N) {
        uint32_t ui[D];
        load_pos<D>(pos, i, ui);
        float v2 = 0.0f, f2 = 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const float v = vel[(size_t)i * D + q], f = force[(size_t)i * D + q];
            v2 = __builtin_fmaf(v, v, v2);
            f2 = __builtin_fmaf(f, f, f2);
        }
        const float ahead = dt * sqrtf(v2) + dt * dt * sqrtf(f2);
        far = !(sqrtf(disp2<D>(ui, pos_ref, i, b)) + 3.0f * ahead <= half_skin);  // NaN counts as far
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && ctl[kListOkWord] == 0) ctl[kTrigWord] = 1;
    wave_flag(far, &ctl[kTrigWord]);
}

// ------------------------------------------------------------------------------------------------
// FIRE

struct FireArgs {
    DevBox box;
    ListParams lp;
    ListGen list;    // the caller's list (the first force evaluation of fire_init)
    ListGen gen[2];  // list generations of the step pipeline: the caller's and the context's
    Bins bins[2];
    int32_t *flags;
    int32_t *ctl;
    uint32_t *pos;
    float *vel;
    float *force;
    const int32_t *species;
    const md_fire_state *st_in;  // the state a launch starts from
    md_fire_state *st_out;       // where the state after the rules goes (workgroup 0)
    double *partials;            // [4 * nparts]: F.v, v.v, F.F and max |F_i|^2 of each force workgroup
    int32_t nparts;
    int32_t apply;  // mixing launch: 1 = apply the rules to the partials first; 0 = st_in is the state of the step
    int32_t step;   // step of the call, >= 1
    int32_t sync;   // 1: a full rebuild gated on ctl[kTrigWord] runs between the two launches of a step
    int32_t pp;     // 1: sparse cells; the pipeline's rows are built one particle per W lanes
    float kappa;    // rebuild lookahead of the pipeline, in steps of the current displacement
    double f_tol;
    float dt_max, f_inc, f_dec, alpha_start, f_alpha;
    int32_t n_min;
};

// Three sums and a maximum over the workgroup: lanes by an xor tree, then the four waves in order.  Every thread
// gets the results, and every workgroup that reduces the same values gets them bit for bit.
__device__ __forceinline__ void block_sum3_max(double &x, double &y, double &z, double &m, double (*red4)[kBlock / 64])
{
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o);
        y += __shfl_xor(y, o);
        z += __shfl_xor(z, o);
        m = fmax(m, __shfl_xor(m, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red4[0][w] = x;
        red4[1][w] = y;
        red4[2][w] = z;
        red4[3][w] = m;
    }
    __syncthreads();
    x = y = z = m = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
        x += red4[0][q];
        y += red4[1][q];
        z += red4[2][q];
        m = fmax(m, red4[3][q]);
    }
    __syncthreads();
}

// The global P = F.v, |v|^2, |F|^2 and max |F_i|^2 of a step from its force workgroups' partials, in a fixed order:
// thread t adds partials t, t + kBlock, ... from zero, then the workgroup's threads are combined.  fire_part_first
// loads the first of them (issued early by the mixing launch), fire_totals the rest and the combination.
__device__ __forceinline__ void fire_part_first(const double *part, int n, double &P, double &vv, double &ff,
                                                double &fm)
{
    P = vv = ff = fm = 0.0;
    const int b = threadIdx.x;
    if (b < n) {
        const double4 q = *(const double4 *)(part + 4 * b);
        P += q.x;
        vv += q.y;
        ff += q.z;
        fm = fmax(fm, q.w);
    }
}

__device__ __forceinline__ void fire_totals(const double *part, int n, double &P, double &vv, double &ff, double &fm,
                                            double (*red4)[kBlock / 64])
{
    for (int b = threadIdx.x + kBlock; b < n; b += kBlock) {
        const double4 q = *(const double4 *)(part + 4 * b);
        P += q.x;
        vv += q.y;
        ff += q.z;
        fm = fmax(fm, q.w);
    }
    block_sum3_max(P, vv, ff, fm, red4);
}

// The FIRE rules after the forces of a step (Sec. 3.3.1, after Bitzek et al. 2006): stop once max |F_i| < f_tol;
// otherwise decide the velocity mixing of the next drift and that step's dt and alpha from the sign of P.
__device__ __forceinline__ void fire_rules(md_fire_state &s, double P, double vv, double ff, double fm,
                                           const FireArgs &a, int init)
{
    s.fmax = sqrt(fm);
    s.power = P;
    if (!init) s.steps += 1;
    if (s.fmax < a.f_tol) {
        s.converged = 1;
        return;
    }
    if (init) {
        s.mix_v = 1.0;
        s.mix_f = 0.0;
        return;
    }
    const double al = s.alpha, fn = sqrt(ff), vn = sqrt(vv);
    if (P > 0.0) {
        s.mix_v = 1.0 - al;
        s.mix_f = fn > 0.0 ? al * vn / fn : 0.0;
        s.n_pos += 1;
        if (s.n_pos > a.n_min) {
            s.dt = fmin(s.dt * (double)a.f_inc, (double)a.dt_max);
            s.alpha = al * (double)a.f_alpha;
        }
    } else {
        s.mix_v = 0.0;
        s.mix_f = 0.0;
        s.dt = s.dt * (double)a.f_dec;
        s.alpha = (double)a.alpha_start;
        s.n_pos = 0;
    }
}

// The particle a FIRE force-launch thread works on (W lanes per particle) and that particle's own state, loaded
// before the launch's first decision so that these loads and the control words' are waited on together.
template <int D, int W>
struct FireOwn {
    int i, l, ii;
    bool live;
    uint32_t u[D];
    float v[D], f[D];
    __device__ __forceinline__ void load(const FireArgs &a)
    {
        const int gt = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
        i = gt / W;
        l = gt % W;
        live = i < a.lp.N;
        ii = live ? i : a.lp.N - 1;  // dead lanes shadow the last particle so the lane reduction stays uniform
        load_pos<D>(a.pos, ii, u);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            v[q] = a.vel[(size_t)ii * D + q];
            f[q] = a.force[(size_t)ii * D + q];
        }
    }
};

// F' = F(r) over the list by W lanes per particle; v += dt/2 (F + F') (v = 0 for the first evaluation); workgroup
// partials of F.v, v.v, F.F and max |F_i|^2 in double.
template <int D, int KIND, bool MULTI, int W>
__device__ __forceinline__ void fire_force_pass(const FireArgs &a, const DevPot &p, const ListGen &g,
                                                const FireOwn<D, W> &o, double dt, int init,
                                                double (*red4)[kBlock / 64])
{
    const ListParams &lp = a.lp;
    const int i = o.i, l = o.l, ii = o.ii;
    const bool live = o.live;
    bool stale = live && l == 0 && disp2<D>(o.u, g.pos_ref, ii, a.box) > lp.half_skin * lp.half_skin;
    wave_flag(stale, &a.flags[MD_FLAG_STALE]);
    int si = MULTI ? a.species[ii] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    int n = live ? min(g.count[(size_t)ii * W + l], lp.capW) : 0;
    lane_force<D, KIND, MULTI, W>(a.box, p, a.pos, a.species, lp.N, lp.capW, g.idx, n, ii, l, o.u, si, F);
    double P = 0.0, vv = 0.0, ff = 0.0;
    bool bad = false;
    if (live && l == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            bad = bad || !isfinite(F[q]);
            float v = init ? 0.0f : (float)((double)o.v[q] + 0.5 * dt * ((double)o.f[q] + (double)F[q]));
            a.vel[(size_t)i * D + q] = v;
            a.force[(size_t)i * D + q] = F[q];
            P += (double)F[q] * (double)v;
            vv += (double)v * (double)v;
            ff += (double)F[q] * (double)F[q];
        }
    }
    wave_flag(bad, &a.flags[MD_FLAG_NONFINITE]);
    double fm = ff;
    block_sum3_max(P, vv, ff, fm, red4);
    if (threadIdx.x == 0) {
        a.partials[4 * blockIdx.x + 0] = P;
        a.partials[4 * blockIdx.x + 1] = vv;
        a.partials[4 * blockIdx.x + 2] = ff;
        a.partials[4 * blockIdx.x + 3] = fm;
    }
}

// The first force evaluation of fire_init, over the caller's list.
template <int D, int KIND, bool MULTI, int W>
__global__ __launch_bounds__(kBlock) void k_fire_force(FireArgs a, DevPot p)
{
    __shared__ double red4[4][kBlock / 64];
    if (frozen(a.flags)) return;
    FireOwn<D, W> o;
    o.load(a);
    fire_force_pass<D, KIND, MULTI, W>(a, p, a.list, o, a.st_in->dt, 1, red4);
}

// One FIRE step's force launch.  Pipelined: the list pipeline's rebuild work when a rebuild is under way (bins one
// step, rows the next, as in the Verlet step kernel), then the forces over the list in use.  Synchronous: the
// gated rebuild before this launch has brought the caller's list up to date; clear its trigger, then the forces.
// The flags, the state, the step's control words and the particle's own state are loaded first and waited on
// together (a chain of dependent loads is what a launch of a small system spends its time on).
// The pipeline's rows for sparse cells: the rows of generation gen1 from its bins, one particle per W lanes (the
// particles' reference positions are those the bins were gathered at).
template <int D, int W>
__device__ __forceinline__ void fire_build_pp(const FireArgs &a, int gen1, int *red, uint32_t *tab)
{
    constexpr int TS = kBlock / W;
    const ListParams &lp = a.lp;
    const ListGen &g1 = a.gen[gen1];
    const Bins &bn = a.bins[gen1];
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / W, l = gt % W;
    const bool live = i < lp.N;
    uint32_t ur[D];
    int ne = 0, chunks = 0, n = 0;
    if (live) {
        load_pos<D>(g1.pos_ref, i, ur);
        ne = stencil_table<D>(i, ur, a.box, bn, lp, tab + threadIdx.x / W, TS, l == 0, chunks);
    }
    __syncthreads();
    if (live) {
        n = build_row<D, W>(i, l, ur, a.box, bn, lp, g1.idx, tab + threadIdx.x / W, TS, ne, chunks);
        g1.count[(size_t)i * W + l] = sub_count<W>(n, l);
    }
    wave_flag(n > lp.cap, &a.flags[MD_FLAG_OVERFLOW]);
    n = block_max(n, red);
    if (threadIdx.x == 0) raise_max(&a.flags[MD_FLAG_MAXCOUNT], (n + W - 1) / W * W);
}

template <int D, int KIND, bool MULTI, int W>
__global__ __launch_bounds__(kBlock) void k_fire_step(FireArgs a, DevPot p)
{
    __shared__ int red[kBlock];
    __shared__ int ncnt[(kBlock / 64) * kMaxPerCellPad];
    __shared__ double red4[4][kBlock / 64];
    __shared__ uint32_t tab[(D == 3 ? 27 : 9) * (kBlock / W)];
    const int r = a.step % 3;
    const int32_t halt = a.flags[MD_FLAG_OVERFLOW] | a.flags[MD_FLAG_CELL_OVERFLOW] | a.flags[MD_FLAG_STALE] |
                         a.st_in->converged;
    const double dt = a.st_in->dt;
    const int32_t c_mode = a.ctl[2 * r], c_gen = a.ctl[2 * r + 1], c_req = a.ctl[6 + r];
    FireOwn<D, W> o;
    o.load(a);
    asm volatile("" ::"v"(c_mode), "v"(c_gen), "v"(c_req), "v"(dt), "v"(o.u[0]), "v"(o.v[0]), "v"(o.f[0]));
    if (halt) return;
    int gen = 0;
    if (a.sync) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[kTrigWord] = 0;
    } else {
        // the step's mode and list generation; workgroup 0 publishes the next step's and clears the request slot
        // of the step after it
        int mode = c_mode;
        gen = c_gen;
        if (mode == M_IDLE && c_req) mode = M_BIN;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int ng = mode == M_BUILD ? gen ^ 1 : gen;
            a.ctl[2 * ((a.step + 1) % 3)] = mode == M_BIN ? M_BUILD : M_IDLE;
            a.ctl[2 * ((a.step + 1) % 3) + 1] = ng;
            a.ctl[6 + (a.step + 2) % 3] = 0;
            a.ctl[kGenWord] = ng;
            if (mode == M_BUILD) a.flags[MD_FLAG_REBUILDS] += 1;
        }
        if (mode == M_BUILD && a.pp)
            fire_build_pp<D, W>(a, gen ^ 1, red, tab);
        else
            list_phase<D, W>(mode, gen, a.box, a.lp, a.bins, a.gen, a.pos, a.flags, red, ncnt);
    }
    fire_force_pass<D, KIND, MULTI, W>(a, p, a.gen[gen], o, dt, 0, red4);
}

// One FIRE step's mixing launch.  Each workgroup sums the previous step's partials (the same values in every
// workgroup) and applies the rules to st_in; workgroup 0 stores the resulting state in st_out, which the force
// launch of this step reads.  Then v = mix_v v + mix_f F and r += dt v + dt^2/2 F.  Pipelined, a rebuild is
// requested for this step when a particle is within kappa steps of the current displacement of skin/2 from the
// reference positions of the list this step uses; synchronous, the gated rebuild is triggered when a particle is
// farther than skin/2 from the caller's list's reference positions.  The particle's state, the first partial of
// each thread and the list generation are loaded before the first decision, as in the force launch.
template <int D>
__global__ __launch_bounds__(kBlock) void k_fire_mix_drift(FireArgs a)
{
    __shared__ double red4[4][kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < a.lp.N;
    const int ii = live ? i : a.lp.N - 1;
    const int32_t halt = a.flags[MD_FLAG_OVERFLOW] | a.flags[MD_FLAG_CELL_OVERFLOW] | a.flags[MD_FLAG_STALE];
    md_fire_state s = *a.st_in;
    const int gen = a.sync ? 0 : a.ctl[2 * (a.step % 3) + 1];  // the list generation of this step
    uint32_t ui[D];
    float f[D], v[D];
    load_pos<D>(a.pos, ii, ui);
#pragma unroll
    for (int q = 0; q < D; ++q) {
        f[q] = a.force[(size_t)ii * D + q];
        v[q] = a.vel[(size_t)ii * D + q];
    }
    double P, vv, ff, fm;
    fire_part_first(a.partials, a.apply ? a.nparts : 0, P, vv, ff, fm);
    uint32_t ref[D];
    load_pos<D>(a.gen[gen].pos_ref, ii, ref);
    if (halt) return;
    if (!s.converged && a.apply) {
        fire_totals(a.partials, a.nparts, P, vv, ff, fm, red4);
        fire_rules(s, P, vv, ff, fm, a, 0);
        if (blockIdx.x == 0 && threadIdx.x == 0) a.flags[MD_FLAG_STEPS] = (int32_t)s.steps;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.st_out != a.st_in) *a.st_out = s;
    if (s.converged) return;
    bool req = false;
    if (live) {
        const double dt = s.dt, mv = s.mix_v, mf = s.mix_f;
        uint32_t un[D];
        float step2 = 0.0f, f2 = 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const float vq = (float)(mv * (double)v[q] + mf * (double)f[q]);
            a.vel[(size_t)i * D + q] = vq;
            const float dx = (float)(dt * (double)vq + 0.5 * dt * dt * (double)f[q]);
            un[q] = shift_coord(ui[q], dx, a.box.inv_s[q]);
            step2 = __builtin_fmaf(dx, dx, step2);
            f2 = __builtin_fmaf(f[q], f[q], f2);
        }
        store_pos<D>(a.pos, i, un);
        float d2 = 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const float dq = tdisp(un[q], ref[q], a.box.s[q]);
            d2 = __builtin_fmaf(dq, dq, d2);
        }
        const float ahead = a.sync ? 0.0f : sqrtf(step2) + (float)(dt * dt) * sqrtf(f2);
        req = !(sqrtf(d2) + a.kappa * ahead <= a.lp.half_skin);  // NaN requests a rebuild
    }
    wave_flag(req, a.sync ? &a.ctl[kTrigWord] : &a.ctl[6 + a.step % 3]);
}

// One workgroup: the rules after the forces of a step in a fixed order (the first evaluation of fire_init, or
// the last step of a fire_step call), from st_in into st_out.
__global__ __launch_bounds__(kBlock) void k_fire_reduce(FireArgs a, int init)
{
    __shared__ double red4[4][kBlock / 64];
    if (frozen(a.flags)) return;
    md_fire_state s = *a.st_in;
    if (!s.converged) {
        double P, vv, ff, fm;
        fire_part_first(a.partials, a.nparts, P, vv, ff, fm);
        fire_totals(a.partials, a.nparts, P, vv, ff, fm, red4);
        fire_rules(s, P, vv, ff, fm, a, init);
    }
    if (threadIdx.x != 0) return;
    *a.st_out = s;
    a.flags[MD_FLAG_STEPS] = (int32_t)s.steps;
}

constexpr int kRedBlocks = 256;  // workgroups of the two-pass reductions

// ------------------------------------------------------------------------------------------------
// velocity Verlet with forces from elsewhere (a neural potential): the two half kicks and the drift

// v += dt/2 F; r += dt v; raises ctl[kTrigWord] when a particle is now farther than skin/2 from pos_ref.
template <int D>
__global__ __launch_bounds__(kBlock) void k_kick_drift(uint32_t *pos, float *vel, const float *force, int N,
                                                       DevBox b, const uint32_t *pos_ref, float half_skin, float dt,
                                                       int32_t *ctl)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < N) {
        uint32_t ui[D], un[D];
        load_pos<D>(pos, i, ui);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            float v = __builtin_fmaf(0.5f * dt, force[(size_t)i * D + q], vel[(size_t)i * D + q]);
            vel[(size_t)i * D + q] = v;
            un[q] = shift_coord(ui[q], dt * v, b.inv_s[q]);
        }
        store_pos<D>(pos, i, un);
        far = disp2<D>(un, pos_ref, i, b) > half_skin * half_skin;
    }
    wave_flag(far, &ctl[kTrigWord]);
}

__global__ __launch_bounds__(kBlock) void k_kick(float *vel, const float *force, int64_t n, float h)
{
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < n) vel[q] = __builtin_fmaf(h, force[q], vel[q]);
}

// Forces from a list with W lanes per particle (the loop of the step kernel), for calls that need no energies:
// the lanes of a particle split its sub-rows and combine through shuffles; lane 0 writes the force.
template <int D, int KIND, bool MULTI, int W>
__global__ __launch_bounds__(kBlock) void k_force_lanes(DevBox b, DevPot p, const uint32_t *__restrict__ pos,
                                                        const int32_t *__restrict__ species, int N, int capW,
                                                        const int32_t *__restrict__ idx,
                                                        const int32_t *__restrict__ count, float *__restrict__ force,
                                                        int32_t *flags)
{
    int gt = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    int i = gt / W, l = gt % W;
    bool live = i < N;
    int ii = live ? i : N - 1;  // dead lanes shadow the last particle so the lane reduction stays uniform
    uint32_t ui[D];
    load_pos<D>(pos, ii, ui);
    int si = MULTI ? species[ii] : 0;
    float F[D];
#pragma unroll
    for (int q = 0; q < D; ++q) F[q] = 0.0f;
    int n = live ? min(count[(size_t)ii * W + l], capW) : 0;
    lane_force<D, KIND, MULTI, W>(b, p, pos, species, N, capW, idx, n, ii, l, ui, si, F);
    bool bad = false;
    if (live && l == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            bad = bad || !isfinite(F[q]);
            force[(size_t)i * D + q] = F[q];
        }
    }
    wave_flag(bad, &flags[MD_FLAG_NONFINITE]);
}

// ------------------------------------------------------------------------------------------------
// constant-temperature steps and gradient descent (the caller computes forces between launches)

// BAOA of a BAOAB Langevin step (Leimkuhler and Matthews): v += dt/2 F, x += dt/2 v, v = c1 v + c2 xi,
// x += dt/2 v (both drifts applied as one shift), and the rebuild trigger of k_kick_drift.
template <int D>
__global__ __launch_bounds__(kBlock) void k_langevin_baoa(uint32_t *pos, float *vel, const float *force, int N,
                                                          DevBox b, const uint32_t *pos_ref, float half_skin,
                                                          float dt, float c1, float c2, uint64_t seed,
                                                          const uint64_t *step, int32_t *ctl)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < N) {
        float z[4];
        normals4((uint64_t)i, step[0], seed, z);
        uint32_t ui[D], un[D];
        load_pos<D>(pos, i, ui);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            float v = __builtin_fmaf(0.5f * dt, force[(size_t)i * D + q], vel[(size_t)i * D + q]);
            float vo = __builtin_fmaf(c1, v, c2 * z[q]);
            vel[(size_t)i * D + q] = vo;
            un[q] = shift_coord(ui[q], 0.5f * dt * (v + vo), b.inv_s[q]);
        }
        store_pos<D>(pos, i, un);
        far = disp2<D>(un, pos_ref, i, b) > half_skin * half_skin;
    }
    wave_flag(far, &ctl[kTrigWord]);
}

// Overdamped step x += a_f F (+ a_n xi): Brownian dynamics (Euler-Maruyama) or, without noise, gradient descent.
template <int D, bool NOISE>
__global__ __launch_bounds__(kBlock) void k_overdamped(uint32_t *pos, const float *force, int N, DevBox b,
                                                       const uint32_t *pos_ref, float half_skin, float a_f, float a_n,
                                                       uint64_t seed, const uint64_t *step, int32_t *ctl)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    bool far = false;
    if (i < N) {
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (NOISE) normals4((uint64_t)i, step[0], seed, z);
        uint32_t ui[D], un[D];
        load_pos<D>(pos, i, ui);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            float dx = a_f * force[(size_t)i * D + q];
            if (NOISE) dx = __builtin_fmaf(a_n, z[q], dx);
            un[q] = shift_coord(ui[q], dx, b.inv_s[q]);
        }
        store_pos<D>(pos, i, un);
        far = disp2<D>(un, pos_ref, i, b) > half_skin * half_skin;
    }
    wave_flag(far, &ctl[kTrigWord]);
}

__global__ void k_step_advance(uint64_t *step)
{
    if (threadIdx.x == 0) step[0] += 1;
}

__global__ void k_step_advance_by(uint64_t *step, int32_t n)
{
    if (threadIdx.x == 0) step[0] += (uint64_t)n;
}

// Half step of a Nose-Hoover chain over time h (Martyna, Tuckerman, Tobias and Klein 1996, one stage): 2K from
// the kinetic-energy partials (fixed order), thermostat momenta down the chain, positions, the velocity factor,
// momenta back up.  One workgroup; thread 0 updates the chain.
__global__ __launch_bounds__(kBlock) void k_nhc_chain(const double *partials, int n, md_nhc_state *st, double h)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += kBlock) s += partials[q];
    s = block_sum(s, red);
    if (threadIdx.x != 0) return;
    const int M = st->M;
    if (M < 1 || M > 8) {  // not a chain: leave the velocities as they are
        st->scale = 1.0;
        return;
    }
    const double kT = st->kT, nf = (double)st->n_dof;
    double K2 = 2.0 * s;
    double *p = st->p, *Q = st->Q;
    auto G = [&](int k) { return k == 0 ? K2 - nf * kT : p[k - 1] * p[k - 1] / Q[k - 1] - kT; };
    p[M - 1] += 0.5 * h * G(M - 1);
    for (int k = M - 2; k >= 0; --k) {
        double f = exp(-0.25 * h * p[k + 1] / Q[k + 1]);
        p[k] = (p[k] * f + 0.5 * h * G(k)) * f;
    }
    for (int k = 0; k < M; ++k) st->eta[k] += h * p[k] / Q[k];
    double sc = exp(-h * p[0] / Q[0]);
    K2 *= sc * sc;
    for (int k = 0; k < M - 1; ++k) {
        double f = exp(-0.25 * h * p[k + 1] / Q[k + 1]);
        p[k] = (p[k] * f + 0.5 * h * G(k)) * f;
    }
    p[M - 1] += 0.5 * h * G(M - 1);
    st->scale = sc;
}

__global__ __launch_bounds__(kBlock) void k_scale_by(float *v, int64_t n, const md_nhc_state *st)
{
    double f = st->scale;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBlock)
        v[q] = (float)((double)v[q] * f);
}

__global__ void k_clear_trigger(int32_t *ctl)
{
    if (threadIdx.x == 0) ctl[kTrigWord] = 0;
}

// sum over workgroup partials of (a - b)^2 in double
__global__ __launch_bounds__(kBlock) void k_sqdiff_partial(const float *a, const float *b, int64_t n, double *partials)
{
    __shared__ double red[kBlock];
    int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double v = 0.0;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kBlock) {
        double d = (double)a[q] - (double)b[q];
        v += d * d;
    }
    v = block_sum(v, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ void k_fire_state_init(md_fire_state *st, double dt, double alpha)
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
}

// An empty system is at its minimum: max |F| = 0 passes any positive tolerance.
__global__ void k_fire_state_empty(md_fire_state *st, double f_tol)
{
    st->fmax = 0.0;
    st->power = 0.0;
    st->converged = 0.0 < f_tol ? 1 : 0;
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

// Plain streaming copy of n 16-byte words (the reference kernel for calibrating memory counters).
__global__ __launch_bounds__(kBlock) void k_copy_words(const uint4 *__restrict__ a, uint4 *__restrict__ b, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBlock) b[q] = a[q];
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

// v *= sqrt(dim (N - 1) T / sum v^2), with sum v^2 = 2 ke[0].
__global__ __launch_bounds__(kBlock) void k_rescale(float *v, int64_t n, const double *ke, double target)
{
    double f = ke[0] > 0.0 ? sqrt(target / (2.0 * ke[0])) : 1.0;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBlock)
        v[q] = (float)((double)v[q] * f);
}

// Smallest squared pair distance over the list rows of a workgroup's particles (double partials).
template <int D>
__global__ __launch_bounds__(kBlock) void k_min_r2_partial(DevBox b, const uint32_t *__restrict__ pos, int N,
                                                           const int32_t *__restrict__ idx,
                                                           const int32_t *__restrict__ count, int W, int capW,
                                                           double *partials)
{
    __shared__ double red[kBlock];
    int i = blockIdx.x * kBlock + threadIdx.x;
    double m = 1e300;
    if (i < N) {
        uint32_t ui[D];
        load_pos<D>(pos, i, ui);
        for (int l = 0; l < W; ++l) {
            int n = min(count[(size_t)i * W + l], capW);
            for (int t = 0; t < n; ++t) {
                uint32_t uj[D];
                load_pos<D>(pos, idx[((size_t)t * N + i) * W + l], uj);
                double r2 = 0.0;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    double d = tdisp_d(ui[q], uj[q], b.sd[q]);
                    r2 += d * d;
                }
                m = fmin(m, r2);
            }
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_min_final(const double *partials, int n, double *out)
{
    __shared__ double red[kBlock];
    double m = 1e300;
    for (int q = threadIdx.x; q < n; q += kBlock) m = fmin(m, partials[q]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

__global__ void k_sqrt_mean(double *x, double n)
{
    x[0] = sqrt(x[0] / n);
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

static constexpr int kMaxBlocks = 1 << 16;
static constexpr int kMaxPerCell = 252;                 // bin occupancy fits the 8-bit field of a stencil entry
static constexpr int64_t kMaxBytes = (int64_t)1 << 32;  // list and bin arrays stay below 4 GiB
static constexpr float kKappa = 2.0f;
static constexpr int kSparseCell = 8;  // below this mean cell occupancy the standalone build goes per particle
static constexpr float kFireKappa = 3.0f;  // FIRE speeds up (dt grows, v mixes toward F): a wider margin

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
            b.cw[k] = (float)((double)L / nc);
            b.lo[k] = nc >= 3 ? -1 : 0;
            b.hi[k] = nc >= 3 ? 1 : 0;
            b.C *= nc;
        } else {
            b.nc[k] = 1;
        }
    }
    b.iso = b.s[0] == b.s[1] && (box->dim == 2 || b.s[1] == b.s[2]);
    return true;
}

bool md_make_pot(const md_potential *pot, DevPot &p)
{
    if (!pot || (pot->kind != MD_LJ && pot->kind != MD_SOFT_SPHERE && pot->kind != MD_MORSE &&
                 pot->kind != MD_BUCKINGHAM))
        return false;
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
    if (pot->kind == MD_MORSE && !(pot->r_cut > 0.0f && pot->alpha > 0.0f)) return false;
    if (pot->kind == MD_BUCKINGHAM && !(pot->r_cut > 0.0f)) return false;
    p.mk = (float)((double)pot->alpha * 1.4426950408889634);  // alpha log2(e)
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
            p.sigd[q] = s;
            p.inv_sig[q] = (float)(1.0 / s);
            p.eps_over_sig[q] = (float)(e / s);
            p.eps_over_alpha[q] = (float)(e / pot->alpha);
            if (pot->kind == MD_MORSE) {
                double xc = exp(-(double)pot->alpha * (rc - s));
                p.a12[q] = (float)(2.0 * pot->alpha * e);
                p.c12[q] = (float)e;
                p.ushift[q] = pot->shift ? (float)(e * xc * (xc - 2.0)) : 0.0f;
            }
            if (pot->kind == MD_BUCKINGHAM) {
                const double c = pot->coef[q];
                if (!isfinite(c)) return false;
                p.a12[q] = (float)(e / s);
                p.a6[q] = (float)(6.0 * c);
                p.c12[q] = (float)e;
                p.c6[q] = (float)c;
                p.inv_sig[q] = (float)(1.4426950408889634 / s);  // log2(e) / rho
                p.ushift[q] = pot->shift ? (float)(e * exp(-rc / s) - c / pow(rc, 6.0)) : 0.0f;
            }
        }
    return true;
}

int md_partials_blocks()
{
    return kMaxBlocks;
}

float md_max_cutoff(const md_potential *pot)
{
    if (pot->kind == MD_LJ || pot->kind == MD_MORSE || pot->kind == MD_BUCKINGHAM) return pot->r_cut;
    float m = 0.0f;
    for (int q = 0; q < pot->n_species * pot->n_species; ++q) m = fmaxf(m, (float)pot->sigma[q]);
    return m;
}

static bool box_ok(const md_box *box, float r)
{
    for (int k = 0; k < box->dim; ++k)
        if (!(r < 0.5f * box->L[k])) return false;
    return true;
}

// Cells of the whole list: C per system times the number of systems of a segmented list.
static int list_cells(const DevBox &b, const md_nlist *nl)
{
    return nl->segment > 0 ? b.C * (nl->N / nl->segment) : b.C;
}

// List parameters for the kernels.  The packed 16-bit candidate test (isotropic boxes) bounds the error of
// R16 = sum d_k^2 (d_k the wrapped difference of the upper 16 bits of the coordinates, unit u = L / 2^16) against the
// exact R = sum e_k^2 by |R16 - R| < 2 sqrt(D R) + D, valid while |e_k| < 32767.  With T = r_list^2 / u^2 and
// T1, T2 = T (1 -+ 1e-9) (room for the rounding of the defining double expression, relative error below 1e-15):
// R16 < floor(T1 - 2 sqrt(D T1) - D) implies R < T1, and R16 >= ceil(T2 + 2 sqrt(D T2) + D) implies R >= T2.  A
// displacement with |e_k| >= 32767 gives R16 >= 32767^2 (saturating sums), so pk_hi <= 32767^2 rejects it, as it
// must.  The packed test is used only when the uncertain band is within 10 % of T.
static ListParams make_lp(const md_nlist *nl, int M, const DevBox &b, int dim)
{
    ListParams v;
    v.N = nl->N;
    v.cap = nl->capacity;
    v.W = nl->lanes;
    v.capW = nl->capacity / nl->lanes;
    v.M = M;
    v.seg = nl->segment;
    v.cells = list_cells(b, nl);
    float rl2 = nl->r_list * nl->r_list;
    v.rl2f_lo = rl2 * (1.0f - 1e-5f);
    v.rl2f_hi = rl2 * (1.0f + 1e-5f);
    v.rl2 = (double)nl->r_list * (double)nl->r_list;
    v.half_skin = 0.5f * nl->skin;
    for (int q = 0; q < 3; ++q) {
        const double r = b.s[q] > 0.0f ? 0.5 * (double)nl->skin * (1.0 + 1e-4) / (double)b.s[q] + 16.0 : 0.0;
        v.reach[q] = (uint32_t)fmin(r, 2147483647.0);
    }
    v.kappa = kKappa;
    v.pk = 0;
    v.pk_lo = v.pk_hi = 0;
    if (b.iso) {
        const double u = (double)b.s[0] * 65536.0;  // exact: b.s[0] = L / 2^32
        const double T = v.rl2 / (u * u), T1 = T * (1.0 - 1e-9), T2 = T * (1.0 + 1e-9);
        const double lo = floor(T1 - 2.0 * sqrt(dim * T1) - dim);
        const double hi = ceil(T2 + 2.0 * sqrt(dim * T2) + dim);
        if (lo >= 0.9 * T && hi <= 1.1 * T && hi <= 32767.0 * 32767.0) {
            v.pk = 1;
            v.pk_lo = (int32_t)lo;
            v.pk_hi = (int32_t)hi;
        }
    }
    return v;
}

static inline int nblk(int64_t n)
{
    return (int)((n + kBlock - 1) / kBlock);
}

// dispatch over (dim, kind, species) template instances
#define MD_DISPATCH(D_, KIND_, MULTI_, ...)                                   \
    do {                                                                     \
        if (D_ == 3) {                                                       \
            constexpr int D = 3;                                             \
            if (KIND_ == 0) {                                                \
                constexpr int KIND = 0;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else if (KIND_ == 2) {                                         \
                constexpr int KIND = 2;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else if (KIND_ == 3) {                                         \
                constexpr int KIND = 3;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else {                                                         \
                constexpr int KIND = 1;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            }                                                                \
        } else {                                                             \
            constexpr int D = 2;                                             \
            if (KIND_ == 0) {                                                \
                constexpr int KIND = 0;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else if (KIND_ == 2) {                                         \
                constexpr int KIND = 2;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else if (KIND_ == 3) {                                         \
                constexpr int KIND = 3;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            } else {                                                         \
                constexpr int KIND = 1;                                      \
                if (MULTI_) { constexpr bool MULTI = true; __VA_ARGS__; }    \
                else { constexpr bool MULTI = false; __VA_ARGS__; }          \
            }                                                                \
        }                                                                    \
    } while (0)

// dispatch over the lane count
#define MD_LANES(W_, ...)                                                    \
    do {                                                                     \
        switch (W_) {                                                        \
        case 1: { constexpr int W = 1; __VA_ARGS__; } break;                 \
        case 2: { constexpr int W = 2; __VA_ARGS__; } break;                 \
        case 4: { constexpr int W = 4; __VA_ARGS__; } break;                 \
        default: { constexpr int W = 8; __VA_ARGS__; } break;                \
        }                                                                    \
    } while (0)

static bool lanes_ok(int W)
{
    return W == 1 || W == 2 || W == 4 || W == 8;
}

// Particle arrays of an empty system (N = 0) may be NULL: nothing reads them.
static bool given(const void *ptr, int64_t n)
{
    return ptr != nullptr || n == 0;
}

static bool nl_ok(const md_nlist *nl, int N)
{
    if (nl && (nl->segment < 0 || (nl->segment > 0 && N % nl->segment != 0))) return false;
    return nl && nl->N == N && lanes_ok(nl->lanes) && nl->capacity >= nl->lanes && nl->capacity % nl->lanes == 0 &&
           given(nl->idx, N) && given(nl->count, N) && given(nl->pos_ref, N) && nl->flags && nl->r_list > 0.0f &&
           nl->skin >= 0.0f;
}

static ListGen caller_gen(const md_nlist *nl)
{
    return ListGen{nl->idx, nl->count, nl->pos_ref};
}

static Bins ctx_bins(md_ctx *ctx, int g)
{
    return Bins{ctx->bin_cnt[g], ctx->bin_mem[g]};
}

static md_status check_common(md_ctx *ctx, const md_box *box, int32_t N)
{
    if (!ctx || !box || (box->dim != 2 && box->dim != 3) || N < 0) return MD_ERR_ARG;
    if (N > ctx->N_cap || box->dim > ctx->dim_cap) return MD_ERR_CAPACITY;
    return MD_OK;
}

static md_status check_list(md_ctx *ctx, const md_box *box, const md_nlist *nl, int32_t N, DevBox &b)
{
    if (!nl_ok(nl, N)) return MD_ERR_ARG;
    if (!box_ok(box, nl->r_list)) return MD_ERR_BOX;
    if (!make_box(box, nl->r_list, b)) return MD_ERR_ARG;
    int64_t C = nl->segment > 0 ? (int64_t)b.C * (N / nl->segment) : b.C;
    if (C > ctx->C_cap || C >= (1 << 24)) return MD_ERR_CAPACITY;  // cell numbers fit 24 bits of a stencil entry
    if ((int64_t)N * nl->lanes > (int64_t)kBlock * kMaxBlocks) return MD_ERR_CAPACITY;
    if ((int64_t)N * nl->capacity * 4 >= kMaxBytes || N >= (1 << 24)) return MD_ERR_CAPACITY;
    return MD_OK;
}

static ListKey list_key(const md_nlist *nl, const DevBox &b, int dim, int M)
{
    ListKey k;
    memset(&k, 0, sizeof(k));
    k.idx = nl->idx;
    k.count = nl->count;
    k.pos_ref = nl->pos_ref;
    k.N = nl->N;
    k.dim = dim;
    k.cap = nl->capacity;
    k.W = nl->lanes;
    k.M = M;
    k.seg = nl->segment;
    k.r_list = nl->r_list;
    k.skin = nl->skin;
    for (int q = 0; q < 3; ++q) k.L[q] = b.s[q];  // L / 2^32: the same box exactly when the same scales
    return k;
}

static bool same_key(const ListKey &a, const ListKey &b)
{
    return a.idx == b.idx && a.count == b.count && a.pos_ref == b.pos_ref && a.N == b.N && a.dim == b.dim &&
           a.cap == b.cap && a.W == b.W && a.M == b.M && a.seg == b.seg && a.r_list == b.r_list &&
           a.skin == b.skin && a.L[0] == b.L[0] && a.L[1] == b.L[1] && a.L[2] == b.L[2];
}

// Counting-sort bins of generation 0 and rows of the caller's list; with a gate, every launch
// returns at once unless *gate != 0 on the device.
static md_status launch_build(md_ctx *ctx, int dim, const DevBox &b, const uint32_t *pos, int32_t N,
                              const md_nlist *nl, hipStream_t s, const int32_t *gate)
{
    CountSort cs = ctx->cs;
    Bins bins = ctx_bins(ctx, 0);
    ListParams lp = make_lp(nl, ctx->M_cap, b, dim);
    ListGen g = caller_gen(nl);
    int32_t *ok = ctx->ctl + kListOkWord;
    int C = lp.cells;  // cells over all systems of a segmented list
    // one wave per cell (four per workgroup); enough workgroups to copy the reference positions when cells are few
    int64_t want = ((int64_t)C + 3) / 4, copy = (int64_t)N * dim / (4 * kBlock);
    if (copy > want) want = copy;
    int rows_grid = (int)(want < 1 ? 1 : (want > kMaxBlocks ? kMaxBlocks : want));
    // sparsely filled cells (fewer than kSparseCell particles per cell on average) are built one particle per W
    // lanes; denser ones one wave per cell
    const bool sparse = (int64_t)N < (int64_t)kSparseCell * C;
    const int pp_grid = nblk((int64_t)N * lp.W);
    if (sparse) {
        if (dim == 3) {
            hipLaunchKernelGGL(k_cs_count<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, lp.seg, b, cs, gate);
            hipLaunchKernelGGL(k_cs_scan, dim3(1), dim3(kScan), 0, s, cs, C, bins, lp.M, nl->flags, ok, gate);
            hipLaunchKernelGGL(k_cs_place, dim3(nblk(N)), dim3(kBlock), 0, s, cs, N, gate);
            hipLaunchKernelGGL(k_cs_rank_fill<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, cs, bins, lp.M, g.count,
                               lp.W, gate);
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows_pp<3, W>), dim3(pp_grid), dim3(kBlock), 0, s, pos, b, bins,
                                              lp, g, nl->flags, ok, gate));
        } else {
            hipLaunchKernelGGL(k_cs_count<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, lp.seg, b, cs, gate);
            hipLaunchKernelGGL(k_cs_scan, dim3(1), dim3(kScan), 0, s, cs, C, bins, lp.M, nl->flags, ok, gate);
            hipLaunchKernelGGL(k_cs_place, dim3(nblk(N)), dim3(kBlock), 0, s, cs, N, gate);
            hipLaunchKernelGGL(k_cs_rank_fill<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, cs, bins, lp.M, g.count,
                               lp.W, gate);
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows_pp<2, W>), dim3(pp_grid), dim3(kBlock), 0, s, pos, b, bins,
                                              lp, g, nl->flags, ok, gate));
        }
    } else if (dim == 3) {
        hipLaunchKernelGGL(k_cs_count<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, lp.seg, b, cs, gate);
        hipLaunchKernelGGL(k_cs_scan, dim3(1), dim3(kScan), 0, s, cs, C, bins, lp.M, nl->flags, ok, gate);
        hipLaunchKernelGGL(k_cs_place, dim3(nblk(N)), dim3(kBlock), 0, s, cs, N, gate);
        hipLaunchKernelGGL(k_cs_rank_fill<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, cs, bins, lp.M, g.count,
                           lp.W, gate);
        if (lp.pk)
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows<3, W, true>), dim3(rows_grid), dim3(kBlock), 0, s, pos,
                                              b, bins, lp, g, nl->flags, ok, gate));
        else
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows<3, W, false>), dim3(rows_grid), dim3(kBlock), 0, s, pos,
                                              b, bins, lp, g, nl->flags, ok, gate));
    } else {
        hipLaunchKernelGGL(k_cs_count<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, lp.seg, b, cs, gate);
        hipLaunchKernelGGL(k_cs_scan, dim3(1), dim3(kScan), 0, s, cs, C, bins, lp.M, nl->flags, ok, gate);
        hipLaunchKernelGGL(k_cs_place, dim3(nblk(N)), dim3(kBlock), 0, s, cs, N, gate);
        hipLaunchKernelGGL(k_cs_rank_fill<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, N, cs, bins, lp.M, g.count,
                           lp.W, gate);
        if (lp.pk)
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows<2, W, true>), dim3(rows_grid), dim3(kBlock), 0, s, pos,
                                              b, bins, lp, g, nl->flags, ok, gate));
        else
            MD_LANES(lp.W, hipLaunchKernelGGL((k_build_rows<2, W, false>), dim3(rows_grid), dim3(kBlock), 0, s, pos,
                                              b, bins, lp, g, nl->flags, ok, gate));
    }
    // generation-0 bins now belong to nl (a gated build that did not run leaves both as they were)
    ctx->bins_key = list_key(nl, b, dim, lp.M);
    ctx->bins_key_set = true;
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

extern "C" {

const char *md_version(void)
{
    return "md-gfx950 0.3";
}

md_status md_ctx_create(int device, md_ctx **out)
{
    if (!out) return MD_ERR_ARG;
    *out = nullptr;
    HIP_OK(hipSetDevice(device));
    md_ctx *c = new md_ctx();
    c->device = device;
    if (hipMalloc(&c->partials, sizeof(double) * 4 * kMaxBlocks) != hipSuccess ||
        hipMalloc(&c->own_flags, sizeof(int32_t) * MD_NFLAGS) != hipSuccess ||
        hipMalloc(&c->ctl, sizeof(int32_t) * kCtlWords) != hipSuccess ||
        hipMalloc(&c->queue, sizeof(int32_t) * 4) != hipSuccess ||
        hipMalloc(&c->nn_partial, sizeof(float) * (size_t)kNNTrainWaves * kNNParams) != hipSuccess ||
        hipMalloc(&c->fire_slots, sizeof(md_fire_state) * 2) != hipSuccess ||
        hipMemset(c->own_flags, 0, sizeof(int32_t) * MD_NFLAGS) != hipSuccess ||
        hipMemset(c->ctl, 0, sizeof(int32_t) * kCtlWords) != hipSuccess) {
        (void)hipFree(c->partials);
        (void)hipFree(c->own_flags);
        (void)hipFree(c->ctl);
        (void)hipFree(c->queue);
        (void)hipFree(c->nn_partial);
        (void)hipFree(c->fire_slots);
        delete c;
        return MD_ERR_HIP;
    }
    *out = c;
    return MD_OK;
}

static void free_scratch(md_ctx *c)
{
    void *ptrs[] = {c->pos_alt, c->cs.cell_of, c->cs.slot, c->cs.sorted_idx, c->cs.cell_count, c->cs.cell_start,
                    c->bin_cnt[0], c->bin_cnt[1], c->bin_mem[0], c->bin_mem[1],
                    c->g1_idx, c->g1_count, c->g1_pos_ref};
    for (void *p : ptrs) (void)hipFree(p);
    c->pos_alt = nullptr;
    c->cs = CountSort{};
    for (int g = 0; g < 2; ++g) {
        c->bin_cnt[g] = nullptr;
        c->bin_mem[g] = nullptr;
    }
    c->g1_idx = c->g1_count = nullptr;
    c->g1_pos_ref = nullptr;
}

md_status md_ctx_destroy(md_ctx *ctx)
{
    if (!ctx) return MD_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_scratch(ctx);
    (void)hipFree(ctx->partials);
    (void)hipFree(ctx->own_flags);
    (void)hipFree(ctx->ctl);
    (void)hipFree(ctx->queue);
    (void)hipFree(ctx->nn_partial);
    (void)hipFree(ctx->fire_slots);
    delete ctx;
    return MD_OK;
}

md_status md_ctx_reserve(md_ctx *ctx, int32_t N, int32_t dim, int32_t max_cells, int32_t capacity, int32_t lanes,
                         int32_t max_per_cell)
{
    if (!ctx || N < 0 || (dim != 2 && dim != 3) || max_cells < 1 || capacity < 1 || !lanes_ok(lanes) ||
        max_per_cell < 1 || max_per_cell > kMaxPerCell)
        return MD_ERR_ARG;
    // kernels address lists and bins with 32-bit byte offsets
    if ((int64_t)N * capacity * 4 >= kMaxBytes || (int64_t)max_cells * max_per_cell * 16 >= kMaxBytes)
        return MD_ERR_CAPACITY;
    if (N <= ctx->N_cap && dim <= ctx->dim_cap && max_cells <= ctx->C_cap && capacity <= ctx->cap_cap &&
        lanes <= ctx->W_cap && max_per_cell <= ctx->M_cap)
        return MD_OK;
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipDeviceSynchronize());
    int32_t n = N > ctx->N_cap ? N : ctx->N_cap;
    int32_t d = dim > ctx->dim_cap ? dim : ctx->dim_cap;
    int32_t C = max_cells > ctx->C_cap ? max_cells : ctx->C_cap;
    int32_t cap = capacity > ctx->cap_cap ? capacity : ctx->cap_cap;
    int32_t W = lanes > ctx->W_cap ? lanes : ctx->W_cap;
    int32_t M = max_per_cell > ctx->M_cap ? max_per_cell : ctx->M_cap;
    M = (M + 3) / 4 * 4;  // bins are read in chunks of four records
    free_scratch(ctx);
    ctx->bins_key_set = false;
    ctx->N_cap = ctx->dim_cap = ctx->C_cap = ctx->cap_cap = ctx->W_cap = ctx->M_cap = 0;
    size_t nn = (size_t)(n > 0 ? n : 1);
    HIP_OK(hipMalloc(&ctx->pos_alt, sizeof(uint32_t) * nn * d));
    HIP_OK(hipMalloc(&ctx->cs.cell_of, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->cs.slot, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->cs.sorted_idx, sizeof(int32_t) * nn));
    HIP_OK(hipMalloc(&ctx->cs.cell_count, sizeof(int32_t) * (size_t)C));
    HIP_OK(hipMemset(ctx->cs.cell_count, 0, sizeof(int32_t) * (size_t)C));  // each scan re-zeroes what it read
    HIP_OK(hipDeviceSynchronize());  // the zeroes land before any stream's first build
    HIP_OK(hipMalloc(&ctx->cs.cell_start, sizeof(int32_t) * ((size_t)C + 1)));
    for (int g = 0; g < 2; ++g) {
        HIP_OK(hipMalloc(&ctx->bin_cnt[g], sizeof(int32_t) * (size_t)C));
        HIP_OK(hipMalloc(&ctx->bin_mem[g], sizeof(uint32_t) * 4 * (size_t)C * M));
    }
    // second list generation: idx sized for any capacity <= cap, count for any lane count <= W
    HIP_OK(hipMalloc(&ctx->g1_idx, sizeof(int32_t) * nn * cap));
    HIP_OK(hipMalloc(&ctx->g1_count, sizeof(int32_t) * nn * W));
    HIP_OK(hipMalloc(&ctx->g1_pos_ref, sizeof(uint32_t) * nn * d));
    ctx->N_cap = n;
    ctx->dim_cap = d;
    ctx->C_cap = C;
    ctx->cap_cap = cap;
    ctx->W_cap = W;
    ctx->M_cap = M;
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

md_status nl_build(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, md_nlist *nl, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!given(pos, N)) return MD_ERR_ARG;
    DevBox b;
    st = check_list(ctx, box, nl, N, b);
    if (st != MD_OK) return st;
    if (N == 0) return MD_OK;
    return launch_build(ctx, box->dim, b, pos, N, nl, (hipStream_t)stream, nullptr);
}

md_status pair_energy_force(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                            const int32_t *species, int32_t N, const md_nlist *nl, float *force, double *energy,
                            double *virial, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    DevPot p;
    if (!given(pos, N) || !md_make_pot(pot, p)) return MD_ERR_ARG;
    bool multi = pot->n_species > 1;
    if (multi && !given(species, N)) return MD_ERR_ARG;
    if (nl && !nl_ok(nl, N)) return MD_ERR_ARG;
    if (nl && !md_list_covers(nl, md_max_cutoff(pot))) return MD_ERR_ARG;
    if (!box_ok(box, nl ? nl->r_list : md_max_cutoff(pot))) return MD_ERR_BOX;
    DevBox b;
    if (!make_box(box, 0.0f, b)) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    bool ew = energy || virial;
    // without a list the non-finite flag goes to the context's own flag words
    int32_t *flags = nl ? nl->flags : ctx->own_flags;
    int grid = nblk(N);
    if (nl) {
        int W = nl->lanes, capW = nl->capacity / nl->lanes;
        if (ew) {
            MD_DISPATCH(box->dim, pot->kind, multi,
                        hipLaunchKernelGGL((k_pair_nl<D, KIND, MULTI, true>), dim3(grid), dim3(kBlock), 0, s, b, p,
                                           pos, species, N, nl->idx, nl->count, W, capW, force, energy, virial,
                                           flags));
        } else if (force) {
            // forces only: W lanes per particle over the balanced sub-rows
            int lgrid = nblk((int64_t)N * W);
            MD_DISPATCH(box->dim, pot->kind, multi,
                        MD_LANES(W, hipLaunchKernelGGL((k_force_lanes<D, KIND, MULTI, W>), dim3(lgrid), dim3(kBlock),
                                                       0, s, b, p, pos, species, N, capW, nl->idx, nl->count, force,
                                                       flags)));
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

static md_status run_checks(md_ctx *ctx, const md_box *box, const md_potential *pot, const md_nlist *nl, int32_t N,
                            const int32_t *species, DevBox &b, DevPot &p)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!md_make_pot(pot, p)) return MD_ERR_ARG;
    if (pot->n_species > 1 && !given(species, N)) return MD_ERR_ARG;
    st = check_list(ctx, box, nl, N, b);
    if (st != MD_OK) return st;
    if (!md_list_covers(nl, md_max_cutoff(pot))) return MD_ERR_ARG;
    if (nl->capacity > ctx->cap_cap || nl->lanes > ctx->W_cap) return MD_ERR_CAPACITY;
    return MD_OK;
}

// Langevin parameters of a fused run (langevin_run); NULL for velocity Verlet.
struct LangevinCfg {
    float c1, c2;
    uint64_t seed;
    uint64_t *step;
};

static md_status md_run(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                        float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt, int32_t n_steps,
                        void *stream, const LangevinCfg *lv)
{
    DevBox b;
    DevPot p;
    if (!given(pos, N) || !given(vel, N) || !given(force, N) || n_steps < 0 || !isfinite(dt) || (nl && nl->segment != 0))
        return MD_ERR_ARG;
    md_status st = run_checks(ctx, box, pot, nl, N, species, b, p);
    if (st != MD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (N == 0 || n_steps == 0) {
        // an empty system still uses up its noise steps, as the composed Langevin step does
        if (lv && n_steps > 0) hipLaunchKernelGGL(k_step_advance_by, dim3(1), dim3(64), 0, s, lv->step, n_steps);
        return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
    }
    bool multi = pot->n_species > 1;
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctx->ctl);
    // The list the caller holds is used again when generation-0 bins belong to it and the device finds it complete
    // and still valid for pos with room for the first steps; otherwise (or for any other list) a fresh list and
    // generation-0 bins are built for the input positions.
    const ListKey key = list_key(nl, b, box->dim, ctx->M_cap);
    if (ctx->bins_key_set && same_key(key, ctx->bins_key)) {
        if (box->dim == 3)
            hipLaunchKernelGGL(k_verlet_check<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, nl->pos_ref, b,
                               N, dt, 0.5f * nl->skin, ctx->ctl);
        else
            hipLaunchKernelGGL(k_verlet_check<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, nl->pos_ref, b,
                               N, dt, 0.5f * nl->skin, ctx->ctl);
        st = launch_build(ctx, box->dim, b, pos, N, nl, s, ctx->ctl + kTrigWord);
    } else {
        st = launch_build(ctx, box->dim, b, pos, N, nl, s, nullptr);
    }
    if (st != MD_OK) return st;
    StepArgs a;
    a.box = b;
    a.lp = make_lp(nl, ctx->M_cap, b, box->dim);
    a.gen[0] = caller_gen(nl);
    a.gen[1] = ListGen{ctx->g1_idx, ctx->g1_count, ctx->g1_pos_ref};
    a.bins[0] = ctx_bins(ctx, 0);
    a.bins[1] = ctx_bins(ctx, 1);
    a.flags = nl->flags;
    a.ctl = ctx->ctl;
    a.vel = vel;
    a.force = force;
    a.species = species;
    a.dt = dt;
    uint32_t *buf[2] = {pos, ctx->pos_alt};
    a.pos_in = buf[0];
    a.pos_out = buf[1];
    a.step = 0;
    a.last = 0;
    a.langevin = lv != nullptr;
    a.c1 = lv ? lv->c1 : 0.0f;
    a.c2 = lv ? lv->c2 : 0.0f;
    a.seed = lv ? lv->seed : 0;
    a.noise_step = lv ? lv->step : nullptr;
    if (box->dim == 3)
        hipLaunchKernelGGL(k_verlet_begin<3>, dim3(nblk(N)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_verlet_begin<2>, dim3(nblk(N)), dim3(kBlock), 0, s, a);
    HIP_OK(hipGetLastError());
    int grid = nblk((int64_t)N * a.lp.W);
    for (int32_t sidx = 1; sidx <= n_steps; ++sidx) {
        a.step = sidx;
        a.pos_in = buf[sidx & 1];
        a.pos_out = buf[(sidx + 1) & 1];
        a.last = sidx == n_steps;
        MD_DISPATCH(box->dim, pot->kind, multi,
                    MD_LANES(a.lp.W, hipLaunchKernelGGL((k_md_step<D, KIND, MULTI, W>), dim3(grid), dim3(kBlock), 0,
                                                        s, a, p)));
    }
    HIP_OK(hipGetLastError());
    if (n_steps & 1) {
        int n = N * box->dim;
        hipLaunchKernelGGL(k_copy_u32, dim3(nblk(n)), dim3(kBlock), 0, s, n, buf[1], buf[0]);
    }
    if (box->dim == 3)
        hipLaunchKernelGGL(k_list_finalize<3>, dim3(grid), dim3(kBlock), 0, s, ctx->ctl, a.gen[0], a.gen[1], a.lp);
    else
        hipLaunchKernelGGL(k_list_finalize<2>, dim3(grid), dim3(kBlock), 0, s, ctx->ctl, a.gen[0], a.gen[1], a.lp);
    hipLaunchKernelGGL(k_bins_finalize, dim3(nblk((int64_t)b.C * a.lp.M)), dim3(kBlock), 0, s, ctx->ctl, nl->flags,
                       a.bins[0], a.bins[1], b.C, a.lp.M);
    if (lv) hipLaunchKernelGGL(k_step_advance_by, dim3(1), dim3(64), 0, s, lv->step, n_steps);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status verlet_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                      float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt, int32_t n_steps,
                      void *stream)
{
    return md_run(ctx, box, pot, pos, vel, force, species, N, nl, dt, n_steps, stream, nullptr);
}

md_status langevin_run(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                       float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt, float gamma, float kT,
                       uint64_t seed, uint64_t *step, int32_t n_steps, void *stream)
{
    if (!step || !(gamma >= 0.0f) || !(kT >= 0.0f) || !isfinite(gamma) || !isfinite(kT)) return MD_ERR_ARG;
    const double c1 = exp(-(double)gamma * (double)dt);
    LangevinCfg lv{(float)c1, (float)sqrt((1.0 - c1 * c1) * (double)kT), seed, step};
    return md_run(ctx, box, pot, pos, vel, force, species, N, nl, dt, n_steps, stream, &lv);
}

// FIRE steps.  A call builds the list for pos, then runs each step as two launches: the mixing launch (the rules
// of the previous step, the velocity mixing and the drift, and the rebuild request) and the force launch (the
// rebuild work of the two-generation list pipeline when a rebuild is under way, then the forces); with
// sync_rebuild, the device-gated full rebuild runs between the two instead of the pipeline.  The state of
// step q lives in the caller's struct for q = 1 and in the context's two slots after that; a last one-workgroup
// launch applies the rules of the last step into the caller's struct.  fire_init evaluates the first forces.
static md_status fire_run(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                          float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                          md_fire_state *fst, int32_t n_steps, double f_tol, int init, hipStream_t s)
{
    DevBox b;
    DevPot p;
    if (!given(pos, N) || !given(vel, N) || !given(force, N) || !fst || !fp || n_steps < 0 || (nl && nl->segment != 0))
        return MD_ERR_ARG;
    md_status st = run_checks(ctx, box, pot, nl, N, species, b, p);
    if (st != MD_OK) return st;
    if (N == 0) {
        if (init) hipLaunchKernelGGL(k_fire_state_empty, dim3(1), dim3(1), 0, s, fst, f_tol);
        return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
    }
    if (!init && n_steps == 0) return MD_OK;
    bool multi = pot->n_species > 1;
    st = launch_build(ctx, box->dim, b, pos, N, nl, s, nullptr);
    if (st != MD_OK) return st;
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctx->ctl);
    FireArgs a;
    a.box = b;
    a.lp = make_lp(nl, ctx->M_cap, b, box->dim);
    a.list = caller_gen(nl);
    a.gen[0] = a.list;
    a.gen[1] = ListGen{ctx->g1_idx, ctx->g1_count, ctx->g1_pos_ref};
    a.bins[0] = ctx_bins(ctx, 0);
    a.bins[1] = ctx_bins(ctx, 1);
    a.flags = nl->flags;
    a.ctl = ctx->ctl;
    a.pos = pos;
    a.vel = vel;
    a.force = force;
    a.species = species;
    a.st_in = fst;
    a.st_out = fst;
    a.partials = ctx->partials;
    a.apply = 0;
    a.step = 0;
    a.sync = fp->sync_rebuild != 0;
    a.pp = (int64_t)N < (int64_t)kSparseCell * a.lp.cells;  // the standalone build's choice
    a.kappa = kFireKappa;
    a.f_tol = f_tol;
    a.dt_max = fp->dt_max;
    a.f_inc = fp->f_inc;
    a.f_dec = fp->f_dec;
    a.alpha_start = fp->alpha_start;
    a.f_alpha = fp->f_alpha;
    a.n_min = fp->n_min;
    const int grid = nblk((int64_t)N * a.lp.W);
    a.nparts = grid;
    if (init) {
        MD_DISPATCH(box->dim, pot->kind, multi,
                    MD_LANES(a.lp.W, hipLaunchKernelGGL((k_fire_force<D, KIND, MULTI, W>), dim3(grid), dim3(kBlock),
                                                        0, s, a, p)));
        hipLaunchKernelGGL(k_fire_reduce, dim3(1), dim3(kBlock), 0, s, a, 1);
        return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
    }
    md_fire_state *slot = ctx->fire_slots;
    for (int32_t q = 1; q <= n_steps; ++q) {
        a.step = q;
        a.apply = q >= 2;
        a.st_in = q <= 2 ? fst : slot + ((q - 1) & 1);
        a.st_out = q == 1 ? fst : slot + (q & 1);
        if (box->dim == 3)
            hipLaunchKernelGGL(k_fire_mix_drift<3>, dim3(nblk(N)), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL(k_fire_mix_drift<2>, dim3(nblk(N)), dim3(kBlock), 0, s, a);
        a.st_in = a.st_out;
        if (a.sync) {
            st = launch_build(ctx, box->dim, b, pos, N, nl, s, ctx->ctl + kTrigWord);
            if (st != MD_OK) return st;
        }
        MD_DISPATCH(box->dim, pot->kind, multi,
                    MD_LANES(a.lp.W, hipLaunchKernelGGL((k_fire_step<D, KIND, MULTI, W>), dim3(grid), dim3(kBlock),
                                                        0, s, a, p)));
    }
    a.st_out = fst;
    hipLaunchKernelGGL(k_fire_reduce, dim3(1), dim3(kBlock), 0, s, a, 0);
    HIP_OK(hipGetLastError());
    if (box->dim == 3)
        hipLaunchKernelGGL(k_list_finalize<3>, dim3(grid), dim3(kBlock), 0, s, ctx->ctl, a.gen[0], a.gen[1], a.lp);
    else
        hipLaunchKernelGGL(k_list_finalize<2>, dim3(grid), dim3(kBlock), 0, s, ctx->ctl, a.gen[0], a.gen[1], a.lp);
    hipLaunchKernelGGL(k_bins_finalize, dim3(nblk((int64_t)b.C * a.lp.M)), dim3(kBlock), 0, s, ctx->ctl, nl->flags,
                       a.bins[0], a.bins[1], b.C, a.lp.M);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status fire_init(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos, float *vel,
                    float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                    md_fire_state *st, double f_tol, void *stream)
{
    if (!st || !fp) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    md_status r = check_common(ctx, box, N);
    if (r != MD_OK) return r;
    hipLaunchKernelGGL(k_fire_state_init, dim3(1), dim3(1), 0, s, st, (double)fp->dt_start, (double)fp->alpha_start);
    HIP_OK(hipGetLastError());
    return fire_run(ctx, box, pot, (uint32_t *)pos, vel, force, species, N, nl, fp, st, 1, f_tol, 1, s);
}

md_status fire_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                    float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                    md_fire_state *st, int32_t n_steps, double f_tol, void *stream)
{
    return fire_run(ctx, box, pot, pos, vel, force, species, N, nl, fp, st, n_steps, f_tol, 0, (hipStream_t)stream);
}

md_status md_sum(md_ctx *ctx, const double *x, int64_t n, double *out, void *stream)
{
    if (!ctx || !given(x, n) || !out || n < 0) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sum_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, x, n, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_kinetic_energy(md_ctx *ctx, const float *vel, int32_t N, int32_t dim, double *out, void *stream)
{
    if (!ctx || !given(vel, N) || !out || N < 0 || (dim != 2 && dim != 3)) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_ke_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, (int64_t)N * dim, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

// Partial sums of md_kinetic_energy_noalloc: one double per reduction workgroup.  Every GPU the library runs on
// holds its own copy until the process ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[kRedBlocks];

static constexpr int kMaxDevices = 64;
static double *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device, looked up once per device.
static md_status scratch_address(double **out)
{
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MD_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MD_ERR_HIP;
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return MD_OK;
}

md_status md_kinetic_energy_noalloc(const float *vel, int32_t N, int32_t dim, double *out, void *stream)
{
    if (!vel || !out || N < 0 || (dim != 2 && dim != 3)) return MD_ERR_ARG;
    if ((int64_t)N * dim > (int64_t)INT32_MAX) return MD_ERR_CAPACITY;
    double *partials = nullptr;
    md_status st = scratch_address(&partials);
    if (st != MD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // every partial is written before the final sum reads it, so nothing needs clearing between calls
    hipLaunchKernelGGL(k_ke_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, (int64_t)N * dim, partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_kick_drift(md_ctx *ctx, const md_box *box, uint32_t *pos, float *vel, const float *force, int32_t N,
                        const md_nlist *nl, float dt, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!given(pos, N) || !given(vel, N) || !given(force, N) || !nl_ok(nl, N) || !isfinite(dt) || nl->segment != 0)
        return MD_ERR_ARG;
    DevBox b;
    if (!make_box(box, 0.0f, b)) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    if (box->dim == 3)
        hipLaunchKernelGGL(k_kick_drift<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, N, b, nl->pos_ref,
                           0.5f * nl->skin, dt, ctx->ctl);
    else
        hipLaunchKernelGGL(k_kick_drift<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, N, b, nl->pos_ref,
                           0.5f * nl->skin, dt, ctx->ctl);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

static md_status step_common(md_ctx *ctx, const md_box *box, const uint32_t *pos, const float *force, int32_t N,
                             const md_nlist *nl, DevBox &b)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!given(pos, N) || !given(force, N) || !nl_ok(nl, N) || nl->segment != 0) return MD_ERR_ARG;
    if (!make_box(box, 0.0f, b)) return MD_ERR_ARG;
    return MD_OK;
}

md_status md_langevin_baoa(md_ctx *ctx, const md_box *box, uint32_t *pos, float *vel, const float *force, int32_t N,
                           const md_nlist *nl, float dt, float gamma, float kT, uint64_t seed, uint64_t *step,
                           void *stream)
{
    DevBox b;
    md_status st = step_common(ctx, box, pos, force, N, nl, b);
    if (st != MD_OK) return st;
    if (!vel || !step || !isfinite(dt) || !(gamma >= 0.0f) || !(kT >= 0.0f)) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (N > 0) {
        double c1 = exp(-(double)gamma * (double)dt);
        float c2 = (float)sqrt((1.0 - c1 * c1) * (double)kT);
        if (box->dim == 3)
            hipLaunchKernelGGL(k_langevin_baoa<3>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, N, b,
                               nl->pos_ref, 0.5f * nl->skin, dt, (float)c1, c2, seed, step, ctx->ctl);
        else
            hipLaunchKernelGGL(k_langevin_baoa<2>, dim3(nblk(N)), dim3(kBlock), 0, s, pos, vel, force, N, b,
                               nl->pos_ref, 0.5f * nl->skin, dt, (float)c1, c2, seed, step, ctx->ctl);
    }
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

static md_status overdamped(md_ctx *ctx, const md_box *box, uint32_t *pos, const float *force, int32_t N,
                            const md_nlist *nl, float a_f, float a_n, uint64_t seed, uint64_t *step, void *stream)
{
    DevBox b;
    md_status st = step_common(ctx, box, pos, force, N, nl, b);
    if (st != MD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool noise = a_n > 0.0f;
    if (N > 0) {
        if (box->dim == 3) {
            if (noise)
                hipLaunchKernelGGL((k_overdamped<3, true>), dim3(nblk(N)), dim3(kBlock), 0, s, pos, force, N, b,
                                   nl->pos_ref, 0.5f * nl->skin, a_f, a_n, seed, step, ctx->ctl);
            else
                hipLaunchKernelGGL((k_overdamped<3, false>), dim3(nblk(N)), dim3(kBlock), 0, s, pos, force, N, b,
                                   nl->pos_ref, 0.5f * nl->skin, a_f, a_n, seed, step, ctx->ctl);
        } else {
            if (noise)
                hipLaunchKernelGGL((k_overdamped<2, true>), dim3(nblk(N)), dim3(kBlock), 0, s, pos, force, N, b,
                                   nl->pos_ref, 0.5f * nl->skin, a_f, a_n, seed, step, ctx->ctl);
            else
                hipLaunchKernelGGL((k_overdamped<2, false>), dim3(nblk(N)), dim3(kBlock), 0, s, pos, force, N, b,
                                   nl->pos_ref, 0.5f * nl->skin, a_f, a_n, seed, step, ctx->ctl);
        }
    }
    if (noise) hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_brownian_step(md_ctx *ctx, const md_box *box, uint32_t *pos, const float *force, int32_t N,
                           const md_nlist *nl, float dt, float gamma, float kT, uint64_t seed, uint64_t *step,
                           void *stream)
{
    if (!isfinite(dt) || !(gamma > 0.0f) || !(kT >= 0.0f) || (kT > 0.0f && !step)) return MD_ERR_ARG;
    float a_n = (float)sqrt(2.0 * (double)kT * (double)dt / (double)gamma);
    return overdamped(ctx, box, pos, force, N, nl, dt / gamma, a_n, seed, step, stream);
}

md_status md_gradient_step(md_ctx *ctx, const md_box *box, uint32_t *pos, const float *force, int32_t N,
                           const md_nlist *nl, float dt, void *stream)
{
    if (!isfinite(dt)) return MD_ERR_ARG;
    return overdamped(ctx, box, pos, force, N, nl, dt, 0.0f, 0, nullptr, stream);
}

md_status md_nhc_half(md_ctx *ctx, float *vel, int32_t N, int32_t dim, md_nhc_state *state, double h, void *stream)
{
    if (!ctx || !vel || !state || N < 0 || (dim != 2 && dim != 3) || !isfinite(h)) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int64_t n = (int64_t)N * dim;
    hipLaunchKernelGGL(k_ke_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, n, ctx->partials);
    hipLaunchKernelGGL(k_nhc_chain, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, state, h);
    hipLaunchKernelGGL(k_scale_by, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, n, state);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status nl_update(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, md_nlist *nl, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!given(pos, N) || (nl && nl->segment != 0)) return MD_ERR_ARG;
    DevBox b;
    st = check_list(ctx, box, nl, N, b);
    if (st != MD_OK) return st;
    if (N == 0) return MD_OK;
    hipStream_t s = (hipStream_t)stream;
    st = launch_build(ctx, box->dim, b, pos, N, nl, s, ctx->ctl + kTrigWord);
    if (st != MD_OK) return st;
    hipLaunchKernelGGL(k_clear_trigger, dim3(1), dim3(64), 0, s, ctx->ctl);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_kick(md_ctx *ctx, float *vel, const float *force, int32_t N, int32_t dim, float h, void *stream)
{
    if (!ctx || !given(vel, N) || !given(force, N) || N < 0 || (dim != 2 && dim != 3) || !isfinite(h)) return MD_ERR_ARG;
    int64_t n = (int64_t)N * dim;
    if (n == 0) return MD_OK;
    hipLaunchKernelGGL(k_kick, dim3(nblk(n)), dim3(kBlock), 0, (hipStream_t)stream, vel, force, n, h);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_min_distance(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, const md_nlist *nl,
                          double *out, void *stream)
{
    md_status st = check_common(ctx, box, N);
    if (st != MD_OK) return st;
    if (!pos || !out || !nl_ok(nl, N)) return MD_ERR_ARG;
    DevBox b;
    if (!make_box(box, 0.0f, b)) return MD_ERR_ARG;
    if (N == 0) return MD_OK;
    int grid = nblk(N);
    if (grid > 4 * kMaxBlocks) return MD_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    int W = nl->lanes, capW = nl->capacity / nl->lanes;
    if (box->dim == 3)
        hipLaunchKernelGGL(k_min_r2_partial<3>, dim3(grid), dim3(kBlock), 0, s, b, pos, N, nl->idx, nl->count, W,
                           capW, ctx->partials);
    else
        hipLaunchKernelGGL(k_min_r2_partial<2>, dim3(grid), dim3(kBlock), 0, s, b, pos, N, nl->idx, nl->count, W,
                           capW, ctx->partials);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, grid, out);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_rms_diff(md_ctx *ctx, const float *a, const float *b, int64_t n, double *out, void *stream)
{
    if (!ctx || !a || !b || !out || n <= 0) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sqdiff_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, a, b, n, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, out);
    hipLaunchKernelGGL(k_sqrt_mean, dim3(1), dim3(1), 0, s, out, (double)n);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_copy_words(md_ctx *ctx, void *dst, const void *src, int64_t n16, void *stream)
{
    if (!ctx || !dst || !src || n16 < 0) return MD_ERR_ARG;
    if (n16 == 0) return MD_OK;
    int64_t blocks = (n16 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_copy_words, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(kBlock), 0,
                       (hipStream_t)stream, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_rescale_velocities(md_ctx *ctx, float *vel, int32_t N, int32_t dim, double T, void *stream)
{
    if (!ctx || !vel || N < 2 || (dim != 2 && dim != 3) || !(T >= 0.0)) return MD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    double *ke = ctx->partials + kRedBlocks;  // past the partial sums
    int64_t n = (int64_t)N * dim;
    hipLaunchKernelGGL(k_ke_partial, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, n, ctx->partials);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, ctx->partials, kRedBlocks, ke);
    hipLaunchKernelGGL(k_rescale, dim3(kRedBlocks), dim3(kBlock), 0, s, vel, n, ke, (double)dim * (N - 1) * T);
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
