/*
 * md.h - C ABI of the MI355X (gfx950) short-range molecular-dynamics core.
 *
 * The operations follow the statement of the problem in "JAX, M.D.: A
 * Framework for Differentiable Physics" (arXiv:1912.04232):
 *   - a periodic space with a nearest-image displacement and a shift
 *     (Sec. 3.2.1 "Spaces"),
 *   - a pair energy U = 1/2 sum_{i != j} u(r_ij) and forces F = -grad U
 *     (Sec. 3.2.2 "Interactions", Sec. 3.3.2 "Energy Functions"),
 *   - a cell list and a neighbor list with a halo ("skin") that is rebuilt
 *     when particles have moved too far (Sec. 3.2.3 "Spatial Partitioning",
 *     Sec. 3.1 "Benchmarks"),
 *   - constant-energy (NVE) dynamics and FIRE descent, each an init/update
 *     pair (Sec. 3.3.1 "Dynamics and Simulations").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is DEVICE memory owned by the caller.  The library
 *    never frees or reallocates caller memory.  Scratch memory (second
 *    position buffer, cell list, reduction partials) belongs to the md_ctx
 *    and is allocated only by md_ctx_create / md_ctx_reserve.
 *  - Positions are torus coordinates: pos[i*dim + k] is a uint32 fraction of
 *    the box edge, x = pos * L_k / 2^32, so the box is [0, L_x) x [0, L_y)
 *    (x [0, L_z)).  The nearest-image displacement along k is the signed
 *    32-bit wrap of pos_ik - pos_jk times L_k / 2^32, exact in integers.
 *    md_positions_from_float / md_positions_to_float convert.
 *  - Velocities and forces are float, row-major [N][dim].  Per-particle
 *    energies and virials are double [N].  Masses are 1.
 *  - dim is 2 or 3.  Boxes are orthorhombic with origin 0.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Calls enqueue work and return without waiting, except md_flags_read
 *    and md_ctx_* which synchronise as documented.
 *  - An empty system (N = 0) is valid for nl_build, nl_update,
 *    pair_energy_force, verlet_step, fire_init, fire_step, md_kick_drift,
 *    md_kick, md_kinetic_energy and md_sum (and flock_step): nothing is
 *    computed on particles, and the particle arrays (positions, velocities,
 *    forces, species, the list's idx / count / pos_ref) may be NULL.  fire_init
 *    of an empty system reports max |F| = 0 and converged.
 *  - Errors the host can see are returned at once and nothing is enqueued:
 *    NULL pointers, dim not in {2,3}, N < 0, sizes above what md_ctx_reserve
 *    provided (MD_ERR_CAPACITY), r_list >= L_k/2 (MD_ERR_BOX).  Conditions
 *    found on the device are written to nl->flags (see MD_FLAG_*) and read
 *    by the caller when it chooses.  Nothing is printed; no C++ exception
 *    crosses this interface.
 *  - One md_ctx per stream: two calls that share a ctx must not overlap.
 */
#ifndef MD_H
#define MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,            /* NULL pointer, bad dim, bad size or parameter */
    MD_ERR_BOX = -2,            /* r_list >= L/2 in some dimension (nearest image ambiguous) */
    MD_ERR_CAPACITY = -3,       /* N or cell count above the reserved scratch size */
    MD_ERR_HIP = -4,            /* a HIP runtime call failed */
    MD_ERR_NOT_CONVERGED = -5,  /* reported by helpers that poll convergence */
    MD_ERR_NONFINITE = -6,      /* reported by helpers that poll the non-finite flag */
} md_status;

/* Periodic orthorhombic box [0,L_0) x [0,L_1) (x [0,L_2)) (Sec. 3.2.1). */
typedef struct {
    int32_t dim;   /* 2 or 3 */
    float L[3];    /* edge lengths; L[2] ignored when dim == 2 */
} md_box;

enum { MD_LJ = 0, MD_SOFT_SPHERE = 1, MD_MORSE = 2, MD_BUCKINGHAM = 3 };

/*
 * Pair potential with S species (Sec. 3.3.2; species matrices as in App. A).
 *   MD_LJ          u = 4 eps_ab [(sigma_ab/r)^12 - (sigma_ab/r)^6] for r < r_cut,
 *                  minus u(r_cut) when shift != 0; 0 beyond r_cut.
 *   MD_SOFT_SPHERE u = eps_ab/alpha (1 - r/sigma_ab)^alpha for r < sigma_ab, else 0.
 *   MD_MORSE       u = eps_ab [(1 - exp(-alpha (r - sigma_ab)))^2 - 1] for r < r_cut (well depth eps_ab at
 *                  r = sigma_ab, range alpha > 0), minus u(r_cut) when shift != 0; 0 beyond r_cut.
 *   MD_BUCKINGHAM  u = eps_ab exp(-r/sigma_ab) - coef_ab / r^6 for r < r_cut (exponential repulsion of
 *                  strength eps_ab and range sigma_ab > 0, dispersion coefficient coef_ab), minus u(r_cut) when
 *                  shift != 0; 0 beyond r_cut.
 *                  MD_MORSE and MD_BUCKINGHAM are accepted by the list, dense and step entry points; the replica
 *                  entry points (fire_batched, envelope_grad, fire_unrolled_grad) take MD_LJ and MD_SOFT_SPHERE only.
 * sigma, epsilon and coef are S x S row-major (entry a*S+b), symmetric, S <= 8; coef is read for MD_BUCKINGHAM only.
 */
typedef struct {
    int32_t kind;
    int32_t n_species;
    double sigma[64];
    double epsilon[64];
    float alpha;      /* soft-sphere exponent, >= 1 (2 = harmonic); Morse range */
    float r_cut;      /* Lennard-Jones / Morse / Buckingham cutoff distance (absolute) */
    int32_t shift;    /* energy shift at the cutoff on/off */
    int32_t reserved;
    double coef[64];  /* Buckingham dispersion coefficients */
} md_potential;

/* Device flag words in md_nlist.flags (int32 each). */
enum {
    MD_FLAG_OVERFLOW = 0,      /* a row needed more than `capacity` entries; the list is invalid */
    MD_FLAG_MAXCOUNT = 1,      /* largest row length seen by any build (the capacity needed) */
    MD_FLAG_NONFINITE = 2,     /* a non-finite force was produced */
    MD_FLAG_REBUILDS = 3,      /* number of builds performed (incremented by every build) */
    MD_FLAG_CELL_OVERFLOW = 4, /* a cell held more than max_per_cell particles; the list is invalid */
    MD_FLAG_STALE = 5,         /* a force used a list older than skin/2 allows; the run is invalid */
    MD_FLAG_MAXCELL = 6,       /* largest cell occupancy seen (the max_per_cell needed) */
    MD_FLAG_STEPS = 7,         /* index of the last step of verlet_step / fire_step that ran */
    MD_NFLAGS = 8
};

/*
 * Neighbor list (Sec. 3.2.3): row i holds the indices j of all particles with
 * |d(r_i, r_j)| < r_list, j != i (both directions, "full" list), split into
 * `lanes` (W = 1, 2, 4 or 8) interleaved sub-rows that W GPU lanes walk
 * together: entry t of sub-row l of particle i is idx[(t*N + i)*W + l], and
 * count[i*W + l] is that sub-row's length (at most capacity/W).  A build
 * numbers the accepted neighbors in a fixed order (the particle's own cell
 * first, then the other cells of its 27 (9 in 2D) cell stencil in stencil
 * order, each cell's members in bin order: by index after nl_build, by their
 * order in the previous bins after a rebuild inside verlet_step)
 * and deals them round-robin to the sub-rows: neighbor n goes to sub-row
 * n % W at position n / W, so sub-row lengths differ by at most one and a
 * build is deterministic.
 * r_list = cutoff + skin; the list stays valid while every particle has moved
 * less than skin/2 from pos_ref, the positions at the last build (Sec. 3.1:
 * the list is rebuilt when particles have moved farther than the halo allows).
 * segment > 0 splits the N particles into N/segment independent periodic
 * systems of `segment` particles each (same box; no pair across systems), as
 * used for batches of configurations; nl_build, pair_energy_force and the
 * neural-potential calls accept such lists, verlet_step and fire_step do not.
 */
typedef struct {
    int32_t N;
    int32_t capacity;    /* entries per row, a multiple of lanes */
    int32_t lanes;       /* W: 1, 2, 4 or 8 */
    int32_t segment;     /* 0, or the size of each independent system (divides N) */
    float r_list;        /* list radius */
    float skin;          /* r_list - cutoff; rebuild when a particle moved > skin/2 */
    int32_t *idx;        /* [capacity/W][N][W] */
    int32_t *count;      /* [N][W] */
    uint32_t *pos_ref;   /* [N][dim] positions at the last build */
    int32_t *flags;      /* [MD_NFLAGS] */
} md_nlist;

typedef struct md_ctx md_ctx;

/* Create a context on HIP device `device` (makes it current). */
md_status md_ctx_create(int device, md_ctx **out);
/* Synchronise the device and free the context's scratch. */
md_status md_ctx_destroy(md_ctx *ctx);
/*
 * Reserve scratch for up to N particles in `dim` dimensions, up to max_cells
 * cells holding up to max_per_cell particles each, and a second neighbor-list
 * generation of up to `capacity` entries per row in up to `lanes` sub-rows
 * (used while rebuilding during verlet_step).  This is the only call that allocates; it
 * synchronises the device when it has to grow.  Every other call returns
 * MD_ERR_CAPACITY when it would need more than was reserved.
 */
md_status md_ctx_reserve(md_ctx *ctx, int32_t N, int32_t dim, int32_t max_cells, int32_t capacity, int32_t lanes,
                         int32_t max_per_cell);
/* Number of cells the cell list uses for this box and list radius, per system (host only); a segmented
 * list of S systems needs S times as many (md_ctx_reserve's max_cells). */
int32_t md_cell_count(const md_box *box, float r_list);

/* x (float [N][dim], any real value) -> torus coordinates pos (nearest 2^-32 L, wrapped). */
md_status md_positions_from_float(const md_box *box, const float *x, uint32_t *pos, int32_t N, void *stream);
/* pos -> x = pos * L / 2^32 rounded to float. */
md_status md_positions_to_float(const md_box *box, const uint32_t *pos, float *x, int32_t N, void *stream);

/*
 * Build the neighbor list of `pos` (Sec. 3.2.3): counting-sort cell binning
 * with cells of edge >= r_list (27 or 9 stencil cells; a dimension with fewer
 * than 3 cells is scanned whole) into bins of max_per_cell members (more
 * raises MD_FLAG_CELL_OVERFLOW), then one candidate scan per particle: by
 * one wave per cell (the cell's stencil candidates in its lanes) when cells
 * hold 8 or more particles on average, else by the W lanes of each particle
 * over the stencil cells its slab distances allow.  Either way the set of
 * each row is the same.  The
 * predicate is r2 < r_list^2 with r2 evaluated in IEEE double as
 * d_0*d_0 + d_1*d_1 (+ d_2*d_2), d_k = (double)wrap32(pos_ik - pos_jk) *
 * (L_k / 2^32): a single-precision filter decides pairs far from the
 * boundary and the double expression decides the rest.  Copies pos to
 * nl->pos_ref, raises MD_FLAG_OVERFLOW when a row does not fit and updates
 * MD_FLAG_MAXCOUNT / MD_FLAG_REBUILDS.  nl->N must equal N.
 */
md_status nl_build(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, md_nlist *nl, void *stream);

/*
 * Forces, and optionally per-particle energies and virials (Sec. 3.2.2):
 *   force[i]  = sum_j f(r_ij)/r_ij * d(r_i, r_j)         (float, [N][dim])
 *   energy[i] = 1/2 sum_j u(r_ij)                        (double [N] or NULL)
 *   virial[i] = 1/2 sum_j r_ij f(r_ij),  f = -du/dr      (double [N] or NULL)
 * over the neighbor list when nl != NULL (its pairs beyond the cutoff add
 * nothing), or over all N(N-1) ordered pairs when nl == NULL (dense).  A list must have
 * r_list - skin >= the potential's range (MD_ERR_ARG otherwise): it is used while particles stay
 * within skin/2 of pos_ref, so only pairs within r_list - skin are sure to be in it.
 * Pair arithmetic is single precision; energy and virial sums are double.
 * species may be NULL when pot->n_species == 1.  force may be NULL.
 */
md_status pair_energy_force(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                            const int32_t *species, int32_t N, const md_nlist *nl, float *force,
                            double *energy, double *virial, void *stream);

/*
 * n_steps of velocity-Verlet NVE (Sec. 3.3.1), unit masses:
 *   v += dt/2 F;  r = shift(r, dt v);  F = F(r);  v += dt/2 F.
 * On entry `force` must hold F(pos).  The call keeps nl when the last call on ctx that
 * built a list built this one (same arrays, sizes and box; nl_build, nl_update, fire_* or
 * a verlet_step that ended with it), no build or run since found it incomplete, and on the
 * device every particle is within skin/2 of nl->pos_ref by a margin of three steps of
 * dt |v| + dt^2 |F|; otherwise it first rebuilds nl for pos.  Between calls the list arrays
 * belong to the library: a caller that edits them must call nl_build before the next run.
 * Then it enqueues one launch per step, in which nl->lanes lanes share a particle.  The list is kept valid on the
 * device with no host synchronisation: when a particle's displacement from the reference positions of the list the
 * next step uses (after a build step, the new list's) plus twice its last step (and dt^2 |F|) would exceed
 * nl->skin/2, the next two launches rebuild it into a second generation while forces still use the current one,
 * and the launch after that switches (Sec. 3.1: the list is rebuilt when particles have moved too far for the
 * halo).  Every step checks
 * that the list it uses is within skin/2 of the positions and raises
 * MD_FLAG_STALE otherwise.  On return pos, vel, force and nl hold the state
 * after n_steps.  If a build overflows (MD_FLAG_OVERFLOW / _CELL_OVERFLOW) or
 * a list went stale, the remaining steps do nothing, MD_FLAG_STEPS tells the
 * last step that ran, and the state is partial: the caller re-runs from its
 * own copy of the input with larger capacities (or shorter calls).
 */
md_status verlet_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                      float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt,
                      int32_t n_steps, void *stream);

/* FIRE parameters (Bitzek et al. 2006, cited in Sec. 3.3.1). */
typedef struct {
    float dt_start, dt_max, f_inc, f_dec, alpha_start, f_alpha;
    int32_t n_min;
    int32_t sync_rebuild;  /* fire_step's list upkeep: 0 pipelined, 1 before each force evaluation (see fire_step);
                              the batched and unrolled minimizers ignore it */
} md_fire_params;

/* FIRE scalars, kept in DEVICE memory by the caller (one struct). */
typedef struct {
    double dt;        /* current time step */
    double alpha;     /* current mixing factor */
    double fmax;      /* max_i |F_i| after the last step */
    double power;     /* P = F . v of the last step */
    double mix_v;     /* velocity update still to apply before the next drift: */
    double mix_f;     /*   v = mix_v v + mix_f F  (0, 0 after P <= 0)        */
    int64_t steps;    /* steps taken since fire_init */
    int32_t n_pos;    /* steps since P was last <= 0 */
    int32_t converged;/* 1 once max_i |F_i| < f_tol */
} md_fire_state;

/*
 * FIRE descent init (Sec. 3.3.1, App. A "fire_descent"): rebuilds nl for pos,
 * vel = 0, force = F(pos), st = {dt_start, alpha_start, n_pos 0}, fmax and
 * converged from the initial forces against f_tol.
 */
md_status fire_init(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                    float *vel, float *force, const int32_t *species, int32_t N, md_nlist *nl,
                    const md_fire_params *fp, md_fire_state *st, double f_tol, void *stream);
/*
 * Up to n_steps FIRE steps (unit masses), each:
 *   r = shift(r, dt v + dt^2/2 F); F' = F(r); v += dt/2 (F + F'); F = F';
 *   stop once max_i |F_i| < f_tol;  P = F.v;  v = (1-a) v + a |v| F/|F|;
 *   P > 0: n_pos++, and when n_pos > n_min: dt = min(dt f_inc, dt_max), a *= f_alpha
 *   else : dt *= f_dec, v = 0, a = alpha_start, n_pos = 0.
 * Steps after convergence do nothing, so the call can be enqueued in fixed
 * chunks; st->converged / st->steps tell the caller where it stopped.  The
 * call rebuilds nl for pos first.  Each step starts with a launch that
 * applies the rules of the previous step, the velocity mixing and the drift,
 * and ends with the force launch.  The list is kept up on the device in one
 * of two ways (fp->sync_rebuild):
 *   0  pipelined, two launches per step, as in verlet_step: a particle that
 *      comes within 3 steps of its current displacement of skin/2 from the
 *      list's reference positions starts a rebuild whose bins and rows are
 *      made inside the next two force launches, into the context's second
 *      list (rows one particle per W lanes when cells are sparse, as in
 *      nl_build).  A step that moves a particle farther than that margin allows
 *      (the large early steps from an overlapping start) leaves the list
 *      stale: MD_FLAG_STALE is set and the call freezes.
 *   1  before each force evaluation a full rebuild runs when a particle is
 *      farther than skin/2 from the reference positions (five more launches
 *      per step, which return at once when no rebuild is due); never stale.
 * At the end of the call nl holds the list in use.  A list that went stale
 * or overflowed sets its flag and freezes the call; st is then left as it
 * was at the start.  The velocity mixing decided by a step is applied at
 * the start of the next one (st->mix_v, st->mix_f).  Global sums are double
 * and summed in a fixed order: every workgroup of the mixing launch sums the
 * force launch's per-workgroup partials itself and gets the same values.
 * Scratch: the context's partials, control words, second list and two state
 * slots (calls on one context are serialized by its stream).
 */
md_status fire_step(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                    float *force, const int32_t *species, int32_t N, md_nlist *nl, const md_fire_params *fp,
                    md_fire_state *st, int32_t n_steps, double f_tol, void *stream);

/*
 * A batch of independent periodic 2D replicas of uneven size (the batched
 * minimizations of Sec. 4.2, which the paper vectorizes over diameters and
 * random keys).  Replica b owns particles offset[b] .. offset[b+1]-1 of the
 * concatenated arrays and has its own box.  max_n and max_cells are host-side
 * bounds the caller promises (largest replica, largest cell count for cells
 * of edge >= the interaction range); a replica that exceeds the per-workgroup
 * limits (4096 particles, 3072 cells) is skipped and reported with status -1.
 */
typedef struct {
    int32_t B;               /* number of replicas */
    int32_t dim;             /* 2 */
    int32_t max_n;           /* largest replica size (host bound) */
    int32_t max_cells;       /* largest cell count (host bound) */
    const int32_t *offset;   /* [B+1], offset[0] = 0 */
    const float *box;        /* [B][dim] box edges */
    uint32_t *pos;           /* [offset[B]][dim] torus coordinates, updated in place */
    const int32_t *species;  /* [offset[B]] or NULL when the potential has one species */
} md_batch;

/* Launch shape of fire_batched, chosen by the caller (e.g. by timing trial launches): threads per replica
 * workgroup (512: 8 particles per thread, or 1024: 4) and the cell edge as a multiple (1 to 4) of the
 * interaction range (larger cells: fewer cells to sort, more candidates per particle). */
typedef struct {
    int32_t threads;
    float cell_factor;
} md_batch_config;

/*
 * FIRE (same rules as fire_step, v = 0 and dt_start / alpha_start at the
 * start) on every replica of the batch in one launch: one workgroup per
 * replica at a time, replicas taken from a work queue, positions and the cell
 * list held in LDS (cell list rebuilt for each force evaluation, so no
 * neighbor list or skin is involved).  Outputs per replica: final energy
 * (double), max_i |F_i|, steps taken, status (1 converged, 0 not converged
 * within max_steps, -1 replica too large).  All outputs are device arrays of
 * length B.  Calls that share a ctx must not overlap (the work queue lives in
 * the ctx).  cfg may be NULL (512 threads, cells of the interaction range);
 * MD_ERR_ARG for another thread count or a cell factor outside [1, 4].  Both
 * change only the order of floating-point sums (a particle's pair terms, the
 * workgroup reductions), not the method.
 */
md_status fire_batched(md_ctx *ctx, const md_batch *batch, const md_potential *pot, const md_fire_params *fp,
                       const md_batch_config *cfg, int32_t max_steps, double f_tol, double *energy, double *fmax,
                       int32_t *steps, int32_t *status, void *stream);

/*
 * Gradient of each replica's energy U = 1/2 sum_{i != j} u(r_ij) with respect
 * to the pair parameters at fixed positions: g_sigma[b][a*S+c] =
 * 1/2 sum over ordered pairs (i, j) with species (a, c) of du/dsigma, likewise
 * g_eps (entries (a,c) and (c,a) of a symmetric matrix are one parameter: add
 * both).  At a converged FIRE minimum this is the derivative of the minimized
 * energy E*(theta) (envelope theorem), which the paper obtains by
 * differentiating through the minimizer (Sec. 4.2); diameters enter through
 * sigma_ab = (d_a + d_b)/2 (App. A).  energy [B] and status [B] may be NULL.
 * Pair arithmetic is single precision, sums double.  S <= 4.
 */
md_status envelope_grad(md_ctx *ctx, const md_batch *batch, const md_potential *pot, double *g_sigma,
                        double *g_eps, double *energy, int32_t *status, void *stream);

/* Parameter families for envelope_grad_wrt and md_diameter_grad. */
enum {
    MD_WRT_SIGMA = 0,          /* the S*S ordered entries of sigma (as g_sigma of envelope_grad) */
    MD_WRT_EPSILON = 1,        /* the S*S ordered entries of epsilon */
    MD_WRT_DIAMETER = 2,       /* per-species diameters d_s = sigma_ss, sigma_ab = (d_a + d_b)/2 (App. A): S values */
    MD_WRT_EPSILON_COMMON = 3  /* one epsilon shared by every pair: 1 value */
};
/* How the box moves with the diameters. */
enum {
    MD_BOX_FIXED = 0,    /* positions and box fixed */
    MD_BOX_PACKING = 1   /* 2D box edge at fixed packing fraction, L^2 proportional to sum_s n_s d_s^2 (n_s disks of
                            species s in the replica), positions fractional (App. A's rescaled box) */
};

/*
 * Derivative of each replica's energy U at the batch positions with respect to one parameter family (Sec. 4.2:
 * at a converged FIRE minimum this is the derivative of the minimized energy E* by the envelope theorem; App. A differentiates with respect to the
 * small-disk diameter with the box rescaled):
 *   MD_WRT_SIGMA, MD_WRT_EPSILON: the ordered entries as envelope_grad computes them;
 *   MD_WRT_EPSILON_COMMON: their sum over the entries of epsilon;
 *   MD_WRT_DIAMETER: dU/dd_s = 1/2 sum_c (G_sc + G_cs), G_ab = dU/dsigma_ab; with MD_BOX_PACKING (soft spheres
 *     only, whose u depends on r / sigma) plus (n_s d_s / sum_t n_t d_t^2) dU/dln L, dU/dln L = -sum_ab sigma_ab G_ab
 *     (minus the virial).
 * grad: device double [B][m] (m = S*S, S or 1 as above), or, when weights (device double [B]) is given, [m] holding
 * sum_b weights[b] dU_b/dtheta, summed in a fixed order (the product a reverse pass needs).  energy [B] and status
 * [B] as in envelope_grad, may be NULL.  MD_ERR_ARG: an unknown family or box, MD_WRT_DIAMETER with sigma not
 * following the mixing rule (relative 1e-12), MD_BOX_PACKING with another family or potential.  MD_ERR_CAPACITY:
 * B (2 S^2 + m) doubles above the context's reduction buffer (4 x 65536).  Pair arithmetic single precision, sums
 * and the chain rule double.
 */
md_status envelope_grad_wrt(md_ctx *ctx, const md_batch *batch, const md_potential *pot, int32_t wrt, int32_t box,
                            const double *weights, double *grad, double *energy, int32_t *status, void *stream);

/*
 * Per-species diameter derivatives out[b][s] (or, with weights [B], out[s] = sum_b weights[b] dU_b/dd_s) from
 * dU/dsigma_ab g_sigma [B][S*S] computed elsewhere (e.g. dE_K/dsigma of fire_unrolled_grad), by the chain rule of
 * envelope_grad_wrt's MD_WRT_DIAMETER: sigma_ab = (d_a + d_b)/2, d_s = sigma_ss of each replica's sigma matrix
 * (sigma [B][S*S], device, or NULL for pot->sigma, which must then follow the mixing rule), and with MD_BOX_PACKING
 * the box term (n_s d_s / sum_t n_t d_t^2) dln[b], dln [B] = dU/dln L at fixed fractional positions (e.g. g_lnc of
 * fire_unrolled_grad), or NULL for soft spheres (minus the virial from g_sigma).  Every pointer is device memory.
 */
md_status md_diameter_grad(md_ctx *ctx, const md_batch *batch, const md_potential *pot, const double *sigma,
                           const double *g_sigma, const double *dln, int32_t box, const double *weights, double *out,
                           void *stream);

/*
 * Bytes of device workspace fire_unrolled_grad needs for B replicas holding
 * total_n particles in all and K steps: 40 K B bytes of step records
 * (rounded up to a multiple of 256), then 24 (K + 1) total_n bytes of
 * particle records.  0 for a negative argument.
 */
uint64_t fire_unrolled_workspace_bytes(int32_t B, int64_t total_n, int32_t K);

/*
 * Reverse mode through K FIRE steps.  Sec. 4.2 differentiates the minimized
 * energy by differentiating through the minimizer; App. A does so for a fixed
 * 300 FIRE steps on 128 disks whose box is rescaled with the small diameter.
 * For every replica of the batch: K steps with the rules of fire_batched
 * (v = 0, dt_start, alpha_start at the start; no convergence test) from the
 * batch positions, then E_K = U(x_K) and its derivatives by transposing the
 * steps in reverse order.  The branch decisions (P > 0) and the dt / alpha
 * schedule are held fixed, as automatic differentiation of the loop does.
 * sigma: NULL, or a device array [B][S*S] giving each replica its own sigma
 * matrix (symmetric, positive; e.g. one diameter per replica, as the paper
 * vectorizes the minimization over diameters and random keys); epsilon,
 * alpha, r_cut and shift come from pot.
 * Outputs, all device arrays:
 *   energy [B]             E_K
 *   g_sigma, g_eps [B][S*S] dE_K / d entry (a,c) of the ordered species
 *                          matrices; a symmetric parameter is the (a,c) plus
 *                          the (c,a) value, and sigma_ab = (d_a + d_b)/2 turns
 *                          them into per-species diameter derivatives
 *   g_lnc [B]              dE_K / d ln c for the box scaled to c L at fixed
 *                          fractional start positions u / 2^32 and fixed time
 *                          parameters (App. A's rescaled box)
 *   rbar0 [offset[B]][2]   dE_K / dR_0 in fractional coordinates R = u / 2^32,
 *                          or NULL
 *   mixed [B][K]           1 where step k had P > 0, else 0; or NULL
 *   status [B]             1 done, -1 replica above 256 particles, -2 the
 *                          workspace is too small for the replica; or NULL
 * The batch positions are left at R_K.  workspace is caller-owned device
 * memory of fire_unrolled_workspace_bytes(B, offset[B], K) bytes.  It
 * receives the trajectory: for replica b, K records of 5 doubles (dt, alpha,
 * |w|, |F'|, P > 0) at byte 40 K b, and from byte
 * round256(40 K B) + 24 (K + 1) offset[b], one block of 24 n_b bytes per
 * state k = 0..K: positions u_k [n_b][2] uint32, forces F_k [n_b][2] float,
 * pre-mixing velocities w_k [n_b][2] float.
 * One wavefront per replica, dense pair sums over the nearest image.  Soft
 * sphere or LJ with S <= 4 and symmetric positive sigma / epsilon
 * (MD_ERR_ARG otherwise); max_n <= 256 (MD_ERR_CAPACITY otherwise).  Pair
 * arithmetic is single precision (the soft-sphere overlap from the double
 * distance); reductions, step scalars and parameter sums are double.
 */
md_status fire_unrolled_grad(md_ctx *ctx, const md_batch *batch, const md_potential *pot, const double *sigma,
                             const md_fire_params *fp, int32_t K, void *workspace, uint64_t workspace_bytes, double *energy, double *g_sigma,
                             double *g_eps, double *g_lnc, float *rbar0, uint8_t *mixed, int32_t *status,
                             void *stream);

/*
 * Neural pair potential (Sec. 3.2.4 featurizations, Sec. 4.1 per-atom networks, forces as -grad E by
 * Sec. 3.3.2): K = 16 radial basis functions
 *   G_i^k = sum_{j != i, r_ij < r_c} exp(-eta (r_ij - mu_k)^2) (cos(pi r_ij / r_c) + 1)/2,
 *   mu_k = mu0 + k (mu1 - mu0)/(K-1), eta given, or 1/(2 ((mu1 - mu0)/(K-1))^2) when 0,
 * and an MLP with H = 64: x = (G - m)/s, E_i = w3 . sp(W2 sp(W1 x + b1) + b2) + b3, sp = softplus.
 * W1, W2 are BF16 (the MFMA operands, the model's own values), everything else float.  All pointers are
 * device memory.  The network's parameters as one float vector theta (nn_param_count() = 5313 entries):
 * W1 [H][K], b1 [H], W2 [H][H], b2 [H], w3 [H], b3; b1, b2, w3 and b3 may point into it.
 */
typedef struct {
    int32_t K;              /* 16 */
    int32_t H;              /* 64 */
    float mu0, mu1, r_c;    /* basis centres and cutoff */
    float eta;              /* Gaussian width parameter (> 0), or 0 for 1/(2 Delta^2), Delta the centre spacing */
    const uint16_t *W1;     /* bf16 [H][K] */
    const uint16_t *W2;     /* bf16 [H][H] */
    const float *b1, *b2;   /* [H] */
    const float *w3;        /* [H] */
    const float *b3;        /* [1] output bias */
    const float *m, *s;     /* [K] descriptor shift and scale */
} md_nn_params;

/* Number of network parameters (the length of theta). */
int32_t nn_param_count(void);
/* Descriptor normalisation of md_nn_params (m, s) from training descriptors G [N][K] (device float): mean[k] and
 * the population standard deviation scale[k] over the N rows (1 where it is below 1e-8), in double and in a fixed
 * order.  N >= 1. */
md_status nn_descriptor_stats(md_ctx *ctx, const float *G, int32_t N, float *mean, float *scale, void *stream);
/* G[i][k] (float [N][K]) over a neighbor list with r_list - skin >= r_c (3D; a segmented list gives each
 * system's; MD_ERR_ARG for a list that does not cover r_c). */
md_status nn_descriptors(md_ctx *ctx, const md_box *box, const md_nn_params *nn, const uint32_t *pos, int32_t N,
                         const md_nlist *nl, float *G, void *stream);
/*
 * Per-atom energies Ei [N] and input gradients e[i][k] = dE_i/dG_i^k [N][K].  BF16 MFMA with FP32
 * accumulation; each activation operand enters as a pair of BF16 numbers (value and remainder), so only the
 * weights are rounded to BF16.
 */
md_status nn_mlp(md_ctx *ctx, const md_nn_params *nn, const float *G, int32_t N, float *Ei, float *e, void *stream);
/* F_i = -sum_j sum_k (e_i^k + e_j^k) g_k'(r_ij) (r_i - r_j)/r_ij over the list (3D). */
md_status nn_forces(md_ctx *ctx, const md_box *box, const md_nn_params *nn, const uint32_t *pos, int32_t N,
                    const md_nlist *nl, const float *e, float *force, void *stream);
/*
 * Training (Sec. 4.1: energy and force loss over configurations).  For N = S * segment atoms of S systems
 * (a segmented list), with reference energies E_ref [S] (double) and forces F_ref [N][3]:
 *   L = (1/S) sum_s ((E_s - E_ref_s)/segment)^2 + lam_F/(3N) sum_i |F_i - F_ref_i|^2,  E_s = sum of Ei over s.
 * nn_loss writes loss[0] (double), gE[s] = dL/dE_i for the atoms of system s, and lam[i] = dL/dF_i [N][3].
 * S <= 262144.
 */
md_status nn_loss(md_ctx *ctx, const float *Ei, const float *F, const double *E_ref, const float *F_ref, int32_t N,
                  int32_t segment, float lam_F, double *loss, float *gE, float *lam, void *stream);
/*
 * Pair adjoint of the force map at fixed positions: ebar[i][k] = dL/de_i^k
 *   = -sum_j g_k'(r_ij) (r_i - r_j)/r_ij . (lam_i - lam_j)   [N][K].
 */
md_status nn_pair_adjoint(md_ctx *ctx, const md_box *box, const md_nn_params *nn, const uint32_t *pos, int32_t N,
                          const md_nlist *nl, const float *lam, float *ebar, void *stream);
/*
 * Weight gradient grad[5313] (layout of theta) of the loss: the network's reverse pass with seed gE (per
 * system of `segment` atoms; segment 0: one system, gE[0]) plus the reverse pass of its tangent along
 * ebar_i / s, which carries the force term.  Weight-gradient products are BF16 MFMA with FP32 accumulation;
 * the partial gradients (one per wave, in the context) are summed in a fixed order.
 */
md_status nn_mlp_grad(md_ctx *ctx, const md_nn_params *nn, const float *G, int32_t N, int32_t segment,
                      const float *gE, const float *ebar, float *grad, void *stream);
/*
 * One Adam step (Kingma and Ba, bias-corrected; step >= 1) on theta [n = 5313] with moments m, v, and the
 * BF16 copies W1 [H][K], W2 [H][H] of the updated weights (round to nearest even).
 */
md_status nn_adam(md_ctx *ctx, float *theta, float *m, float *v, const float *grad, int32_t n, int32_t step, float lr,
                  float beta1, float beta2, float eps, uint16_t *W1, uint16_t *W2, void *stream);
/* BF16 copies W1, W2 of the weights in theta. */
md_status nn_cast_weights(md_ctx *ctx, const float *theta, uint16_t *W1, uint16_t *W2, void *stream);

/*
 * Velocity Verlet with forces computed elsewhere (e.g. nn_forces), Sec. 3.3.1: one step is
 *   md_kick_drift (v += dt/2 F; r += dt v, the shift of Sec. 3.2.1)  ->  nl_update  ->  new forces F
 *   ->  md_kick (v += dt/2 F).
 * md_kick_drift also marks, on the device, that a particle has moved more than skin/2 from nl->pos_ref;
 * nl_update then rebuilds the list (as nl_build) only if so, deciding on the device (no host round trip:
 * its launches return at once otherwise).  Lists with segment != 0 are rejected.
 */
md_status md_kick_drift(md_ctx *ctx, const md_box *box, uint32_t *pos, float *vel, const float *force, int32_t N,
                        const md_nlist *nl, float dt, void *stream);
md_status nl_update(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, md_nlist *nl, void *stream);
/* vel[q] += h force[q] for q < N dim. */
md_status md_kick(md_ctx *ctx, float *vel, const float *force, int32_t N, int32_t dim, float h, void *stream);

/*
 * Half list (each pair once) from a full list, for comparing the Newton's-third-law force pass with the
 * full-list pass (Sec. 3.2.3 lists): hidx [hcap][N] and hcount [N] (caller-owned device arrays) receive each
 * pair of nl once, in row i when (i < j) differs from (i + j odd) (so rows hold about half their neighbors);
 * any lane count, segment 0.  *overflow (device int32) is set to 1 when a row has more than hcap entries (the
 * row is then truncated).
 */
md_status nl_half(md_ctx *ctx, const md_nlist *nl, int32_t *hidx, int32_t *hcount, int32_t hcap, int32_t *overflow,
                  void *stream);
/*
 * Forces from a half list: every pair evaluated once, F_i += f_ij and F_j -= f_ij through float atomics, so the
 * summation order (and the last bits of the forces) varies between runs.  force [N][dim] is overwritten.  The
 * half list must come from a list valid for pos (the caller checks, e.g. with nl_update).
 */
md_status pair_force_half(md_ctx *ctx, const md_box *box, const md_potential *pot, const uint32_t *pos,
                          const int32_t *species, int32_t N, const int32_t *hidx, const int32_t *hcount, int32_t hcap,
                          float *force, void *stream);

/*
 * Constant temperature and gradient descent (Sec. 3.3.1 names Nose-Hoover, Langevin and Brownian NVT and a
 * gradient-descent minimizer beside NVE and FIRE; the discretizations are published schemes, unit masses).
 * Each step, like md_kick_drift, moves positions by the shift of Sec. 3.2.1 and marks on the device when a
 * particle has moved more than skin/2 from nl->pos_ref; the caller then runs nl_update and new forces.
 * Noise: xi for particle i at step s is Philox4x64-10 (Salmon et al., SC'11) at counter (i, s, 0, 0) with key
 * (seed, 0); the top 24 bits of each output word plus half a unit, over 2^24, are uniforms in (0, 1) and
 * Box-Muller turns (u0, u1), (u2, u3) into four standard normals, the first dim used.  *step is a device
 * counter the call reads and then advances by one (so captured graphs replay with fresh noise).
 *
 * Langevin (BAOAB, Leimkuhler and Matthews 2013): one step is
 *   md_langevin_baoa (v += dt/2 F; x += dt/2 v; v = c1 v + c2 xi; x += dt/2 v) -> nl_update -> new forces F
 *   -> md_kick (v += dt/2 F),   c1 = exp(-gamma dt), c2 = sqrt((1 - c1^2) kT).
 */
md_status md_langevin_baoa(md_ctx *ctx, const md_box *box, uint32_t *pos, float *vel, const float *force, int32_t N,
                           const md_nlist *nl, float dt, float gamma, float kT, uint64_t seed, uint64_t *step,
                           void *stream);
/*
 * Langevin (BAOAB) fused like verlet_step: n_steps steps of
 *   v += dt/2 F; x += dt/2 v; v = c1 v + c2 xi; x += dt/2 v; F = F(x); v += dt/2 F
 * in one launch per step, with the list rebuilt on the device inside the run exactly as in verlet_step (same list
 * arguments, flags and reuse rules), c1 = exp(-gamma dt), c2 = sqrt((1 - c1^2) kT).  The normals of particle i at
 * noise step t are those md_langevin_baoa draws (Philox4x64-10 at counter (i, t, 0, 0), key (seed, 0)); the steps
 * use t = step[0], step[0] + 1, ... and step[0] (device memory, required) advances by n_steps.  On entry force
 * holds F(x); on return pos, vel, force are the state after the last step.  The arithmetic of a coordinate is that
 * of md_langevin_baoa -> forces -> md_kick; forces summed over a list rebuilt at other steps may differ in the last
 * bits.  Errors as verlet_step; also gamma < 0, kT < 0 or a NULL step.
 */
md_status langevin_run(md_ctx *ctx, const md_box *box, const md_potential *pot, uint32_t *pos, float *vel,
                       float *force, const int32_t *species, int32_t N, md_nlist *nl, float dt, float gamma, float kT,
                       uint64_t seed, uint64_t *step, int32_t n_steps, void *stream);
/* Brownian dynamics (overdamped Langevin, Euler-Maruyama): x += (dt/gamma) F + sqrt(2 kT dt / gamma) xi, then
 * nl_update and new forces.  gamma > 0; with kT = 0 no noise is drawn and step may be NULL. */
md_status md_brownian_step(md_ctx *ctx, const md_box *box, uint32_t *pos, const float *force, int32_t N,
                           const md_nlist *nl, float dt, float gamma, float kT, uint64_t seed, uint64_t *step,
                           void *stream);
/* Gradient descent (steepest descent): x += dt F, then nl_update and new forces. */
md_status md_gradient_step(md_ctx *ctx, const md_box *box, uint32_t *pos, const float *force, int32_t N,
                           const md_nlist *nl, float dt, void *stream);

/*
 * Flocking energy model (Sec. 4.3, App. B): boids with positions R_i (uint32 torus coordinates, [N][2]) and
 * headings theta_i (float [N]), N_i = (cos theta_i, sin theta_i), rho(r; Rc) = (1/alpha)(1 - r/Rc)^alpha below Rc.
 *   E_align    = 1/2 sum_{i != j} J_align rho(r_ij; R_align)(1 - N_i . N_j)^2, its position gradient stopped
 *   E_avoid    = 1/2 sum_{i != j} J_avoid rho(r_ij; R_avoid)
 *   E_cohesion = sum_i 1/2 J_coh (1 - hat(dR_i) . N_i)^2, dR_i = mean over j with r_ij < R_coh of (R_j - R_i)
 *                (a boid with no such neighbor, or dR_i = 0, adds nothing)
 *   E_obstacle = sum_i sum_o J_obs rho(|R_i - C_o|; D_o)(1 - N_i . hat(R_i - C_o))^2 (disk o: center C_o, radius D_o)
 * Displacements are nearest images; obstacle centers are plain coordinates in [0, L).  Predators: see
 * md_flock_predators.
 */
typedef struct {
    float J_align, R_align;
    float J_avoid, R_avoid;
    float J_coh, R_coh;
    float J_obs;
    float alpha;        /* exponent of rho, >= 1 */
    float v;            /* speed along N_i */
    float dt;
    int32_t n_obstacles;  /* 0..16 */
    int32_t reserved;
    float obstacles[16][3];  /* (C_x, C_y, D) */
} md_flock_params;

/*
 * Predators (App. B): a two-player game.  Boids add E_boid-predator = sum_{i,p} J_flee rho(|R_i - R_p|; R_flee)
 * (1 - N_i . hat(R_i - R_p))^2 (the obstacle form with predator p as the disk center) to the energy they step on;
 * predator p steps on its own energy E_p = 1/2 J_chase (1 - hat(dR_p) . N_p)^2, dR_p = mean over boids within
 * R_chase of (R_j - R_p) (the cohesion form; nothing when no boid is in range), plus the obstacle terms with
 * J_obs, at speed v.  Both sides step from the state at the start of the step.  The predators' occasional sprint
 * is not part of this call.  pos [P][2] (uint32 torus coordinates) and theta [P] are device memory, updated in
 * place; each predator scans all N boids (its sums split over up to 64 workgroups and combined in a fixed order in
 * the context's reduction buffer), so P is meant to be small.
 */
typedef struct {
    int32_t P;           /* number of predators, 0..4096 */
    float J_flee, R_flee;
    float J_chase, R_chase;
    float v;
    uint32_t *pos;
    float *theta;
} md_flock_predators;

/*
 * One forward-Euler step of the flocking dynamics (App. B): R_i += dt (v N_i - dE/dR_i), theta_i -= dt dE/dtheta_i,
 * both from the state at the start of the step.  nl must be a full list (segment 0, any lane count) with
 * r_list - skin >= max(R_align, R_avoid, R_coh), valid for pos (nl_update after each step keeps it so: the call marks on
 * the device when a boid has moved more than skin/2 from nl->pos_ref).  The list's lanes (W) set how many GPU
 * lanes share a boid.  work is device scratch of 8 N floats owned by the caller (8-byte aligned); after the call
 * work[8i + 0..2] holds (dE/dx_i, dE/dy_i, dE/dtheta_i) of the step and work[8i + 6..7] the heading N_i it used.  box->dim must
 * be 2.  pred may be NULL (no predators); with predators, work[8i + 0..2] includes the flee term.  With N = 0 nothing
 * is enqueued for boids (their arrays may be NULL) and the predators still take their step: they swim at speed v
 * and descend their obstacle terms, with empty chase sums.  Errors:
 * MD_ERR_ARG (missing pointer, dim, list or parameters out of range, 8 N >= 2^31), MD_ERR_BOX (an edge not above
 * 2 r_list, or not above 2 R_flee or 2 R_chase).
 */
md_status flock_step(md_ctx *ctx, const md_box *box, uint32_t *pos, float *theta, int32_t N, const md_nlist *nl,
                     const md_flock_params *fp, const md_flock_predators *pred, float *work, void *stream);

/* Nose-Hoover chain state (Martyna, Klein and Tuckerman 1992), kept in DEVICE memory by the caller. */
typedef struct {
    double p[8];      /* thermostat momenta p_k = Q_k xi_k */
    double eta[8];    /* thermostat positions */
    double Q[8];      /* thermostat masses, k < M */
    double kT;        /* target temperature */
    double scale;     /* velocity factor applied by the last md_nhc_half */
    int32_t M;        /* chain length, 1..8 */
    int32_t n_dof;    /* degrees of freedom n_f (N dim) */
} md_nhc_state;

/*
 * Half step of the chain over time h (Martyna, Tuckerman, Tobias and Klein 1996, one stage): thermostat
 * forces G_1 = 2K - n_f kT, G_k = p_{k-1}^2 / Q_{k-1} - kT; momenta down the chain (each scaled by
 * exp(-h/4 p_{k+1}/Q_{k+1}) around its h/2 kick), eta += h p / Q, velocities scaled by exp(-h p_1 / Q_1), momenta
 * back up.  A Nose-Hoover step is md_nhc_half(dt/2) -> md_kick_drift -> nl_update -> forces -> md_kick(dt/2)
 * -> md_nhc_half(dt/2); H' = K + U + sum_k p_k^2 / (2 Q_k) + n_f kT eta_1 + kT sum_{k>1} eta_k is conserved.
 * K is summed in double in a fixed order; the chain update runs on the device (no host round trip).
 */
md_status md_nhc_half(md_ctx *ctx, float *vel, int32_t N, int32_t dim, md_nhc_state *state, double h, void *stream);
/* out[0] = the smallest pair distance over the rows of nl at pos (double, device memory; 1e150 if no row has
 * an entry): with the force RMSE, the check that a configuration stays where a network was trained. */
md_status md_min_distance(md_ctx *ctx, const md_box *box, const uint32_t *pos, int32_t N, const md_nlist *nl,
                          double *out, void *stream);
/* out[0] = sqrt(mean over q < n of (a[q] - b[q])^2) in double (device memory), e.g. a force RMSE. */
md_status md_rms_diff(md_ctx *ctx, const float *a, const float *b, int64_t n, double *out, void *stream);

/* out[0] = sum of x[0..n) in double, summed in a fixed order (deterministic). out is device memory. */
md_status md_sum(md_ctx *ctx, const double *x, int64_t n, double *out, void *stream);
/* out[0] = 1/2 sum_i |v_i|^2 in double (device memory). */
md_status md_kinetic_energy(md_ctx *ctx, const float *vel, int32_t N, int32_t dim, double *out, void *stream);
/*
 * md_kinetic_energy without a context, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): out[0] = 1/2 sum_i |v_i|^2 in double on the current HIP device.  Its 256 partial
 * sums live in a 2 KiB array of the library's own device memory, one copy per GPU, held until the process ends;
 * the call allocates nothing and needs no md_ctx.  Every call on one GPU shares that array, so calls that overlap
 * on one GPU (different streams without ordering) race; calls ordered on one stream do not.  N dim above
 * INT32_MAX returns MD_ERR_CAPACITY; NULL pointers, N < 0 or dim not in {2,3} return MD_ERR_ARG.
 */
md_status md_kinetic_energy_noalloc(const float *vel, int32_t N, int32_t dim, double *out, void *stream);
/* Scale vel [N][dim] so that sum |v_i|^2 = dim (N - 1) T (unit mass, net momentum assumed zero): velocity
 * rescaling to a temperature, for preparing configurations at a given T.  No host synchronisation. */
md_status md_rescale_velocities(md_ctx *ctx, float *vel, int32_t N, int32_t dim, double T, void *stream);

/* Copy nl->flags to host `out` (MD_NFLAGS ints) after synchronising `stream`. */
md_status md_flags_read(const md_nlist *nl, int32_t *out, void *stream);
/* Zero nl->flags (enqueued on `stream`). */
md_status md_flags_clear(md_nlist *nl, void *stream);

/* Copy n16 16-byte words src -> dst (device, 16-byte aligned): a plain streaming copy of known size, the
 * reference that memory-traffic counters of the other kernels are calibrated against. */
md_status md_copy_words(md_ctx *ctx, void *dst, const void *src, int64_t n16, void *stream);

/* Library version string. */
const char *md_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MD_H */
