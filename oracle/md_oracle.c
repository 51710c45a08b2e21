/*
 * FP64 brute-force reference ("oracle") for the short-range MD path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; it is used by tests/, by the smoke check and by the
 * cpu_baseline leg of bench.py.  It shares no code, header or constant with
 * the HIP path.
 *
 * Everything here is the plain definition, evaluated in IEEE double with no
 * FMA contraction (built with -ffp-contract=off), O(N^2) over all pairs:
 *
 *   space    : periodic box [0,L_x)x[0,L_y)(x[0,L_z)), displacement to the
 *              nearest image, metric = Euclidean norm    (paper Sec. 3.2.1)
 *   energy   : U = 1/2 sum_{i != j} u(r_ij)              (paper Sec. 3.2.2)
 *   forces   : F_i = -grad_i U, written analytically     (paper Sec. 3.2.2,
 *              Sec. 3.3.2 "quantity.force")
 *   potentials (paper Sec. 3.3.2 names them, the forms are the standard ones):
 *     Lennard-Jones  u = 4 eps [(s/r)^12 - (s/r)^6] (- u(r_c) if shifted),
 *                    0 for r >= r_c
 *     soft sphere    u = (eps/alpha) (1 - r/s)^alpha for r < s, else 0; the
 *                    same functional form the paper prints for its flocking
 *                    cutoff function (App. B, eq. "cutoff")
 *     Morse          u = eps [(1 - exp(-alpha (r - s)))^2 - 1] (- u(r_c) if
 *                    shifted), 0 for r >= r_c: well depth eps at r = s
 *     Buckingham     u = eps exp(-r/s) - c / r^6 (- u(r_c) if shifted), 0 for
 *                    r >= r_c: exponential repulsion of strength eps and range
 *                    s, dispersion coefficient c (a third S x S matrix)
 *   species mixing : s_ab, eps_ab given as S x S matrices (App. A builds
 *                    s_ab = (d_a + d_b)/2)
 *   neighbor set   : all ordered pairs with r^2 < r_list^2 (Sec. 3.2.3)
 *   dynamics       : velocity Verlet NVE, m = 1           (Sec. 3.3.1)
 *   minimizer      : FIRE (Bitzek et al. 2006, cited in Sec. 3.3.1)
 *   parameter gradient at fixed positions (envelope theorem, Sec. 4.2)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t kind;        /* 0 = Lennard-Jones, 1 = soft sphere, 2 = Morse, 3 = Buckingham */
    int32_t n_species;   /* S, 1..8 */
    double sigma[64];    /* S x S, row-major */
    double epsilon[64];  /* S x S, row-major */
    double alpha;        /* soft-sphere exponent; Morse range parameter */
    double r_cut;        /* Lennard-Jones / Morse / Buckingham cutoff distance */
    int32_t shift;       /* Lennard-Jones / Morse / Buckingham: subtract u(r_cut) from the energy */
    double coef[64];     /* Buckingham: the dispersion coefficient C_ab, S x S */
} orc_pot;

typedef struct {
    double dt_start, dt_max, f_inc, f_dec, alpha_start, f_alpha;
    int32_t n_min;
} orc_fire_params;

typedef struct {
    double dt, alpha;
    int64_t n_pos;
    int64_t steps;
    int32_t converged;
} orc_fire_state;

/* ------------------------------------------------------------------ space */

/* Displacement a - b folded to the nearest periodic image. */
static void displacement(int dim, const double *L, const double *a, const double *b, double *d)
{
    for (int k = 0; k < dim; ++k) {
        double t = a[k] - b[k];
        d[k] = t - L[k] * nearbyint(t / L[k]);
    }
}

static double norm2(int dim, const double *d)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += d[k] * d[k];
    return s;
}

/* ------------------------------------------------------------ potentials */

/* u(r) and f(r) = -du/dr for one pair with parameters (s, e) and, for Buckingham, c. */
static void pair_u(const orc_pot *p, double r, double s, double e, double c, double *u, double *f)
{
    *u = 0.0;
    *f = 0.0;
    if (p->kind == 0) {
        if (r >= p->r_cut) return;
        double sr6 = pow(s / r, 6.0);
        double sr12 = sr6 * sr6;
        *u = 4.0 * e * (sr12 - sr6);
        if (p->shift) {
            double sc6 = pow(s / p->r_cut, 6.0);
            *u -= 4.0 * e * (sc6 * sc6 - sc6);
        }
        *f = 24.0 * e * (2.0 * sr12 - sr6) / r;
    } else if (p->kind == 2) {
        /* Morse: u = e [(1 - exp(-a (r - s)))^2 - 1], minimum -e at r = s */
        if (r >= p->r_cut) return;
        double x = exp(-p->alpha * (r - s));
        *u = e * ((1.0 - x) * (1.0 - x) - 1.0);
        if (p->shift) {
            double xc = exp(-p->alpha * (p->r_cut - s));
            *u -= e * ((1.0 - xc) * (1.0 - xc) - 1.0);
        }
        *f = -2.0 * p->alpha * e * x * (1.0 - x);
    } else if (p->kind == 3) {
        /* Buckingham (the exponential-six form named in Sec. 3.3.2): u = e exp(-r/s) - c / r^6, e the
           repulsion strength, s its range, c the dispersion coefficient */
        if (r >= p->r_cut) return;
        *u = e * exp(-r / s) - c / pow(r, 6.0);
        if (p->shift) *u -= e * exp(-p->r_cut / s) - c / pow(p->r_cut, 6.0);
        *f = e / s * exp(-r / s) - 6.0 * c / pow(r, 7.0);
    } else {
        if (r >= s) return;
        double t = 1.0 - r / s;
        *u = e / p->alpha * pow(t, p->alpha);
        *f = e / s * pow(t, p->alpha - 1.0);
    }
}

/* Partial derivatives of u(r) with respect to s and e at fixed r. */
static void pair_du_dparam(const orc_pot *p, double r, double s, double e, double *du_ds, double *du_de)
{
    *du_ds = 0.0;
    *du_de = 0.0;
    if (p->kind == 0) {
        if (r >= p->r_cut) return;
        double sr6 = pow(s / r, 6.0);
        double sr12 = sr6 * sr6;
        double u = 4.0 * e * (sr12 - sr6);
        double dus = 4.0 * e * (12.0 * sr12 - 6.0 * sr6) / s;
        if (p->shift) {
            double sc6 = pow(s / p->r_cut, 6.0);
            u -= 4.0 * e * (sc6 * sc6 - sc6);
            dus -= 4.0 * e * (12.0 * sc6 * sc6 - 6.0 * sc6) / s;
        }
        *du_ds = dus;
        *du_de = u / e;
    } else {
        if (r >= s) return;
        double t = 1.0 - r / s;
        *du_ds = e * pow(t, p->alpha - 1.0) * r / (s * s);
        *du_de = pow(t, p->alpha) / p->alpha;
    }
}

/* ------------------------------------------------------- thread helpers */

typedef struct {
    void (*fn)(void *ctx, int64_t lo, int64_t hi);
    void *ctx;
    int64_t lo, hi;
} chunk_t;

static void *chunk_run(void *arg)
{
    chunk_t *c = (chunk_t *)arg;
    c->fn(c->ctx, c->lo, c->hi);
    return NULL;
}

static void parallel_for(int64_t n, int nthreads, void (*fn)(void *, int64_t, int64_t), void *ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads == 1 || n < 2 * nthreads) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[256];
    chunk_t ch[256];
    for (int t = 0; t < nthreads; ++t) {
        ch[t].fn = fn;
        ch[t].ctx = ctx;
        ch[t].lo = n * t / nthreads;
        ch[t].hi = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, chunk_run, &ch[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------- energy / force / virial */

typedef struct {
    int dim;
    const double *L;
    int64_t N;
    const double *x;
    const int32_t *species;
    const orc_pot *pot;
    const int64_t *rows;
    double *F, *e, *w;
} pair_ctx;

static void pair_rows_body(void *vctx, int64_t lo, int64_t hi)
{
    pair_ctx *c = (pair_ctx *)vctx;
    int dim = c->dim;
    int S = c->pot->n_species;
    for (int64_t q = lo; q < hi; ++q) {
        int64_t i = c->rows ? c->rows[q] : q;
        double Fi[3] = {0.0, 0.0, 0.0}, ei = 0.0, wi = 0.0;
        int si = c->species ? c->species[i] : 0;
        for (int64_t j = 0; j < c->N; ++j) {
            if (j == i) continue;
            int sj = c->species ? c->species[j] : 0;
            double d[3];
            displacement(dim, c->L, c->x + i * dim, c->x + j * dim, d);
            double r = sqrt(norm2(dim, d));
            double u, f;
            pair_u(c->pot, r, c->pot->sigma[si * S + sj], c->pot->epsilon[si * S + sj], c->pot->coef[si * S + sj], &u,
                   &f);
            if (u == 0.0 && f == 0.0) continue;
            for (int k = 0; k < dim; ++k) Fi[k] += f * d[k] / r;
            ei += 0.5 * u;
            wi += 0.5 * r * f;
        }
        if (c->F)
            for (int k = 0; k < dim; ++k) c->F[q * dim + k] = Fi[k];
        if (c->e) c->e[q] = ei;
        if (c->w) c->w[q] = wi;
    }
}

/*
 * Forces F_i, per-particle energies e_i = 1/2 sum_j u(r_ij) and per-particle
 * virials w_i = 1/2 sum_j r_ij f(r_ij) for the requested rows (rows == NULL:
 * every particle), each summed over all j != i.  sum_i e_i = U and
 * sum_i w_i = W = sum_{i<j} r_ij f(r_ij).  Any output may be NULL.
 */
int orc_pair_rows(int dim, const double *L, int64_t N, const double *x, const int32_t *species,
                  const orc_pot *pot, const int64_t *rows, int64_t nrows, double *F, double *e, double *w,
                  int nthreads)
{
    if (dim < 1 || dim > 3 || N < 0 || pot == NULL) return -1;
    pair_ctx c = {dim, L, N, x, species, pot, rows, F, e, w};
    parallel_for(rows ? nrows : N, nthreads, pair_rows_body, &c);
    return 0;
}

/* -------------------------------------------------------- neighbor set */

typedef struct {
    int dim;
    double s[3];
    int64_t N;
    const uint32_t *u;
    double rl2;
    const int64_t *rows;
    int32_t cap;
    int32_t *count, *idx;
} nbr_ctx;

static void nbr_body(void *vctx, int64_t lo, int64_t hi)
{
    nbr_ctx *c = (nbr_ctx *)vctx;
    int dim = c->dim;
    for (int64_t q = lo; q < hi; ++q) {
        int64_t i = c->rows ? c->rows[q] : q;
        int32_t n = 0;
        for (int64_t j = 0; j < c->N; ++j) {
            if (j == i) continue;
            double r2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                int32_t dk = (int32_t)(c->u[i * dim + k] - c->u[j * dim + k]);
                double d = (double)dk * c->s[k];
                r2 += d * d;
            }
            if (r2 < c->rl2) {
                if (n < c->cap) c->idx[q * c->cap + n] = (int32_t)j;
                ++n;
            }
        }
        c->count[q] = n;
    }
}

/*
 * Neighbor set on the discrete torus.  Positions are 32-bit fractions of the
 * box, x_k = u_k * L_k / 2^32.  The nearest-image displacement along k is
 * then (signed 32-bit wrap of u_ik - u_jk) * L_k / 2^32, which is exact in
 * integers; the pair (i, j) is a neighbor when
 *     r2 = d_0*d_0 + d_1*d_1 (+ d_2*d_2)   (IEEE double, left to right,
 *                                           d_k = (double)dk * (L_k/2^32))
 * is strictly below (double)r_list * (double)r_list.  This expression is the
 * definition of the set; it is evaluated here for every pair j != i.
 * Row q lists the accepted j in increasing order (up to cap entries);
 * count[q] is the full number found, which may exceed cap.
 */
int orc_neighbors(int dim, const double *L, int64_t N, const uint32_t *u, float r_list, const int64_t *rows,
                  int64_t nrows, int32_t cap, int32_t *count, int32_t *idx, int nthreads)
{
    if (dim < 1 || dim > 3 || N < 0) return -1;
    nbr_ctx c;
    c.dim = dim;
    for (int k = 0; k < 3; ++k) c.s[k] = k < dim ? L[k] / 4294967296.0 : 0.0;
    c.N = N;
    c.u = u;
    c.rl2 = (double)r_list * (double)r_list;
    c.rows = rows;
    c.cap = cap;
    c.count = count;
    c.idx = idx;
    parallel_for(rows ? nrows : N, nthreads, nbr_body, &c);
    return 0;
}

/* ---------------------------------------------------- velocity Verlet */

static void wrap(int dim, const double *L, double *x)
{
    for (int k = 0; k < dim; ++k) {
        x[k] -= L[k] * floor(x[k] / L[k]);
        if (x[k] >= L[k]) x[k] -= L[k]; /* floor rounding at the top edge */
    }
}

/*
 * n_steps of velocity Verlet with unit masses (paper Sec. 3.2.2, m r'' = -grad U):
 *   v += dt/2 F;  x = wrap(x + dt v);  F = F(x);  v += dt/2 F.
 * F must hold the forces at the input positions.
 */
int orc_verlet(int dim, const double *L, int64_t N, double *x, double *v, double *F, const int32_t *species,
               const orc_pot *pot, double dt, int64_t n_steps, int nthreads)
{
    for (int64_t s = 0; s < n_steps; ++s) {
        for (int64_t i = 0; i < N; ++i) {
            for (int k = 0; k < dim; ++k) {
                v[i * dim + k] += 0.5 * dt * F[i * dim + k];
                x[i * dim + k] += dt * v[i * dim + k];
            }
            wrap(dim, L, x + i * dim);
        }
        int rc = orc_pair_rows(dim, L, N, x, species, pot, NULL, N, F, NULL, NULL, nthreads);
        if (rc) return rc;
        for (int64_t i = 0; i < N * dim; ++i) v[i] += 0.5 * dt * F[i];
    }
    return 0;
}

/* -------------------------------------------------------------- FIRE */

/*
 * FIRE (Bitzek, Koskinen, Gahler, Moseler, Gumbsch, PRL 97, 170201 (2006)),
 * unit masses.  Each step:
 *   1. x = wrap(x + dt v + dt^2/2 F)
 *   2. F' = F(x)
 *   3. v = v + dt/2 (F + F');  F = F'
 *   4. stop when max_i |F_i| < f_tol
 *   5. P = F . v  (over all N*dim components)
 *   6. v = (1 - a) v + a |v| F/|F|
 *   7. P > 0: n_pos += 1; if n_pos > n_min: dt = min(dt f_inc, dt_max), a *= f_alpha
 *      else : dt *= f_dec, v = 0, a = alpha_start, n_pos = 0
 * The caller initialises v (normally 0), F = F(x), st->dt = dt_start,
 * st->alpha = alpha_start, st->n_pos = 0.  Before the first step the
 * convergence test is applied to the input forces as well.
 */
int orc_fire(int dim, const double *L, int64_t N, double *x, double *v, double *F, const int32_t *species,
             const orc_pot *pot, const orc_fire_params *fp, orc_fire_state *st, int64_t max_steps, double f_tol,
             int nthreads)
{
    double *Fn = (double *)malloc(sizeof(double) * (size_t)(N * dim + 1));
    if (!Fn) return -2;
    st->converged = 0;
    double fmax2 = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double f2 = norm2(dim, F + i * dim);
        if (f2 > fmax2) fmax2 = f2;
    }
    if (sqrt(fmax2) < f_tol) {
        st->converged = 1;
        free(Fn);
        return 0;
    }
    for (int64_t s = 0; s < max_steps; ++s) {
        double dt = st->dt;
        for (int64_t i = 0; i < N; ++i) {
            for (int k = 0; k < dim; ++k)
                x[i * dim + k] += dt * v[i * dim + k] + 0.5 * dt * dt * F[i * dim + k];
            wrap(dim, L, x + i * dim);
        }
        int rc = orc_pair_rows(dim, L, N, x, species, pot, NULL, N, Fn, NULL, NULL, nthreads);
        if (rc) {
            free(Fn);
            return rc;
        }
        for (int64_t q = 0; q < N * dim; ++q) {
            v[q] += 0.5 * dt * (F[q] + Fn[q]);
            F[q] = Fn[q];
        }
        st->steps += 1;
        fmax2 = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double f2 = norm2(dim, F + i * dim);
            if (f2 > fmax2) fmax2 = f2;
        }
        if (sqrt(fmax2) < f_tol) {
            st->converged = 1;
            break;
        }
        double P = 0.0, vv = 0.0, ff = 0.0;
        for (int64_t q = 0; q < N * dim; ++q) {
            P += F[q] * v[q];
            vv += v[q] * v[q];
            ff += F[q] * F[q];
        }
        double vn = sqrt(vv), fn = sqrt(ff);
        for (int64_t q = 0; q < N * dim; ++q)
            v[q] = (1.0 - st->alpha) * v[q] + st->alpha * vn * F[q] / fn;
        if (P > 0.0) {
            st->n_pos += 1;
            if (st->n_pos > fp->n_min) {
                st->dt = fmin(st->dt * fp->f_inc, fp->dt_max);
                st->alpha *= fp->f_alpha;
            }
        } else {
            st->dt *= fp->f_dec;
            for (int64_t q = 0; q < N * dim; ++q) v[q] = 0.0;
            st->alpha = fp->alpha_start;
            st->n_pos = 0;
        }
    }
    free(Fn);
    return 0;
}

/* ------------------------------------------- gradient w.r.t. parameters */

/*
 * dU/dsigma_ab and dU/deps_ab at fixed positions, with every ordered pair of
 * species (a, b) treated as an independent entry: G_ab = 1/2 sum over ordered
 * pairs (i, j), i != j, s_i = a, s_j = b, of du/dsigma (resp. du/deps).  For a
 * symmetric matrix whose entries (a,b) and (b,a) are one parameter, the
 * derivative is G_ab + G_ba for a != b.
 */
int orc_param_grad(int dim, const double *L, int64_t N, const double *x, const int32_t *species,
                   const orc_pot *pot, double *g_sigma, double *g_eps)
{
    if (pot->kind == 2 || pot->kind == 3) return -3; /* parameter derivatives: Lennard-Jones and soft spheres */
    int S = pot->n_species;
    for (int q = 0; q < S * S; ++q) {
        g_sigma[q] = 0.0;
        g_eps[q] = 0.0;
    }
    for (int64_t i = 0; i < N; ++i) {
        int si = species ? species[i] : 0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            int sj = species ? species[j] : 0;
            double d[3];
            displacement(dim, L, x + i * dim, x + j * dim, d);
            double r = sqrt(norm2(dim, d));
            double ds, de;
            pair_du_dparam(pot, r, pot->sigma[si * S + sj], pot->epsilon[si * S + sj], &ds, &de);
            g_sigma[si * S + sj] += 0.5 * ds;
            g_eps[si * S + sj] += 0.5 * de;
        }
    }
    return 0;
}
