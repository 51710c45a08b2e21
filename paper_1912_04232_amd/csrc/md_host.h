// Host-side internals shared by the library's translation units: the context and helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/md.h"
#include "md_device.h"

#define HIP_OK(x)                                    \
    do {                                             \
        if ((x) != hipSuccess) return MD_ERR_HIP;    \
    } while (0)

struct CountSort {
    int32_t *cell_of;
    int32_t *slot;
    int32_t *sorted_idx;
    int32_t *cell_count;
    int32_t *cell_start;
};

// Control words of the context (device memory, kCtlWords int32).  ctl[kTrigWord] is the rebuild trigger: a
// kernel that moves positions sets it when a particle has moved more than skin/2 from the list's reference
// positions, and nl_update rebuilds (on the device) and clears it.
constexpr int kCtlWords = 16;
constexpr int kTrigWord = 10;
// ctl[kListOkWord] is 1 while the list that generation-0 bins belong to is complete: a build sets it (0 when a cell
// or a row did not fit) and a Verlet run clears it when it ends frozen (a list that overflowed or went stale).  It
// survives k_ctl_init, so the next verlet_step can decide on the device whether that list can be used again.
constexpr int kListOkWord = 12;

// Identity of the list that generation-0 bins belong to (host side): the caller's list arrays, its sizes and the
// box.  A verlet_step whose list has the same identity may use it again (the device confirms it is still valid).
struct ListKey {
    const void *idx, *count, *pos_ref;
    int32_t N, dim, cap, W, M, seg;
    float r_list, skin, L[3];
};

struct md_ctx {
    int device = 0;
    int32_t N_cap = 0, dim_cap = 0, C_cap = 0, cap_cap = 0, M_cap = 0, W_cap = 0;
    uint32_t *pos_alt = nullptr;
    CountSort cs = {};
    int32_t *bin_cnt[2] = {nullptr, nullptr};
    uint32_t *bin_mem[2] = {nullptr, nullptr};  // [C][M][4] member records
    int32_t *g1_idx = nullptr, *g1_count = nullptr;
    uint32_t *g1_pos_ref = nullptr;
    int32_t *ctl = nullptr;        // kCtlWords
    double *partials = nullptr;    // 4 * kMaxBlocks doubles
    md_fire_state *fire_slots = nullptr;  // two FIRE states a fire_step call alternates between
    int32_t *own_flags = nullptr;  // MD_NFLAGS words for calls made without a neighbor list
    int32_t *queue = nullptr;      // work counter of batched launches
    float *nn_partial = nullptr;   // partial weight gradients of the neural-potential training pass
    ListKey bins_key = {};         // the list generation-0 bins were last built for (valid when bins_key_set)
    bool bins_key_set = false;
};

// neural-potential training: parameter count and the number of partial gradients (one per wave)
constexpr int kNNParams = 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1;
constexpr int kNNTrainWaves = 512;

// ctx->partials holds this many doubles (4 per workgroup of the largest reduction launch).
int md_partials_blocks();


// Pair-potential coefficients for the kernels; false for an invalid potential.
bool md_make_pot(const md_potential *pot, md::DevPot &p);
// Largest interaction range of the potential (LJ cutoff, or the largest soft-sphere sigma).
float md_max_cutoff(const md_potential *pot);
// A list is used while every particle stays within skin/2 of its reference position, so it holds every pair
// within r_list - skin: true when that covers `range` (up to float rounding of r_list and skin).
inline bool md_list_covers(const md_nlist *nl, float range)
{
    return (double)nl->r_list - (double)nl->skin >= (double)range * (1.0 - 1e-6);
}
