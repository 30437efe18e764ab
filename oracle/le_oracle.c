/*
 * le_oracle.c -- plain FP64 CPU oracle for Lees-Edwards shear-flow MD.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this code.  It shares no code, header, table
 * or helper with the HIP library; it is written from the paper (Xu, Vance,
 * Tretyakov, Stuehn, Brinkmann, "Implementation and Parallel Optimization of
 * the Lees-Edwards Boundary Condition in ESPResSo++", arXiv 2109.11083) and is
 * deliberately slow and literal.  Build: gcc -O2 -ffp-contract=off (no FMA
 * contraction, so every sum and product below rounds exactly as written).
 *
 * Axes: flow x, gradient y, vorticity z.  The paper uses gradient z; every
 * formula here is the paper's with its z and y exchanged.
 *
 * Conventions shared with the library contract (stated, not shared code):
 *   arrays are SoA [3][n] (x block, then y, then z) indexed by tag;
 *   the image of the box directly above (gradient +L_y) is displaced by +Delta
 *   along x, with Delta = shear_rate * L_y * t reduced into [0, L_x).
 *
 * Parity status per function is listed in the table at the end of this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double box[3];      /* L_x (flow), L_y (gradient), L_z (vorticity) */
    double shear_rate;  /* gamma_dot */
    double dt, kT, gamma, mass;
    double eps, sigma, rc;
    double fene_k, fene_r0;
    double lj_shift;    /* energy shift added to every pair inside rc (energy only) */
    double dpd_rc;      /* DPD weight-function cutoff (thermostat 1) */
    double angle_k;     /* cosine angle term k_a (Eq. angle); 0 = none */
    double force_cap;   /* > 0: pair-force magnitude limit of a warm-up run; 0 = none */
    uint64_t seed;
    int64_t n;
    int64_t n_chains;
    int32_t chain_len;  /* 0 => no bonds */
    int32_t thermostat; /* 0 Langevin on the peculiar velocity, 1 DPD, 2 Langevin on the lab velocity */
    int32_t velocity;   /* 0: u is the lab velocity; 1: u is the peculiar velocity (Eq. vi), the */
                        /* streaming velocity enters the drift only (Section 2.2)               */
    int32_t pad_;
} orc_params;

enum { ORC_OK = 0, ORC_E_BOND = -4, ORC_E_NONFINITE = -5, ORC_E_ARG = -1 };

/* ------------------------------------------------------------------------ */
/* O1. Lees-Edwards image offset (Section 2.1, Eq. pos_new; Fig. lebc).      */
/* The image box above moves with relative speed shear_rate*L_y; after n     */
/* steps of length dt its offset along the flow axis, taken modulo L_x, is   */
/* Delta_n.  The result lies in [0, L_x).                                    */
double orc_offset(int64_t n, double dt, double shear_rate, double Lx, double Ly)
{
    double sv = shear_rate * Ly;
    double t = (double)n * dt;
    double d = fmod(sv * t, Lx);
    if (d < 0.0) d += Lx;
    if (d >= Lx) d -= Lx;
    return d;
}

/* O2. Canonical periodic wrap of one coordinate into [0, L).  Returns the   */
/* net number k of box lengths that were subtracted (x_new = x_old - k*L up  */
/* to the rounding of that one subtraction), so that callers can apply the  */
/* matching Lees-Edwards shift (the "mod" of Eq. pos_new).                   */
double orc_wrap(double *x, double L)
{
    double k = floor(*x / L);
    double v = *x - k * L;
    if (v < 0.0) { v += L; k -= 1.0; }
    if (v >= L) { v -= L; k += 1.0; }
    *x = v;
    return k;
}

/* O3. Lees-Edwards boundary crossing (Eq. pos_new and the velocity jump of  */
/* the shear profile, Eq. shear-rate).  A particle that leaves through the   */
/* top face (y >= L_y) re-enters at the bottom; its flow coordinate moves by */
/* -Delta and its lab velocity by -shear_rate*L_y, so that its peculiar      */
/* velocity (Eq. vi) is unchanged.  The flow and vorticity coordinates are   */
/* then wrapped periodically.  x, u are [3][n].                              */
void orc_le_wrap(int64_t n, double *x, double *u, double Delta, const orc_params *p)
{
    const double Lx = p->box[0], Ly = p->box[1], Lz = p->box[2];
    const double sv = p->shear_rate * Ly;
    for (int64_t i = 0; i < n; ++i) {
        double *xi = &x[i], *yi = &x[n + i], *zi = &x[2 * n + i];
        double ky = orc_wrap(yi, Ly);
        *xi = *xi - ky * Delta;
        if (u) u[i] = u[i] - ky * sv;
        orc_wrap(xi, Lx);
        orc_wrap(zi, Lz);
    }
}

/* O4. Cell of a (wrapped) particle: the box is cut into nc[0]*nc[1]*nc[2]   */
/* equal cells (Section 2.3); id = (iz*ny + iy)*nx + ix.                     */
int32_t orc_cell_id(double x, double y, double z, const int32_t nc[3], const double box[3])
{
    double inv[3];
    int32_t ia[3];
    const double c[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        inv[a] = (double)nc[a] / box[a];
        int32_t k = (int32_t)(c[a] * inv[a]);
        if (k < 0) k = 0;
        if (k > nc[a] - 1) k = nc[a] - 1;
        ia[a] = k;
    }
    return (ia[2] * nc[1] + ia[1]) * nc[0] + ia[0];
}

/* Cell ids of all particles and the cell-sorted order: ascending (cell, tag). */
void orc_cells(int64_t n, const double *x, const int32_t nc[3], const double box[3],
               int32_t *cell_of, int32_t *order)
{
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    for (int64_t i = 0; i < n; ++i)
        cell_of[i] = orc_cell_id(x[i], x[n + i], x[2 * n + i], nc, box);
    /* stable counting sort by cell id, scanning tags in increasing order */
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) start[cell_of[i] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    for (int64_t i = 0; i < n; ++i) order[start[cell_of[i]]++] = (int32_t)i;
    free(start);
}

/* O5. Lees-Edwards minimum-image displacement d = q_i - q_j (Section 2.4:    */
/* r_ij = q_i - q_j), with the images of Eq. pos_new: the gradient image     */
/* index sy is chosen first, the flow coordinate is corrected by sy*Delta,    */
/* then the flow and vorticity images are chosen.  Returns r^2 summed in the */
/* fixed order (dx*dx + dy*dy) + dz*dz.  img (may be NULL) receives sx,sy,sz. */
static double nearest_int(double v) { return round(v); }

double orc_disp(const double *x, int64_t n, int64_t i, int64_t j, double Delta,
                const double box[3], double d[3], int32_t img[3])
{
    const double Lx = box[0], Ly = box[1], Lz = box[2];
    double dy0 = x[n + i] - x[n + j];
    double sy = nearest_int(dy0 / Ly);
    double dy = dy0 - sy * Ly;
    double dx0 = (x[i] - x[j]) - sy * Delta;
    double sx = nearest_int(dx0 / Lx);
    double dx = dx0 - sx * Lx;
    double dz0 = x[2 * n + i] - x[2 * n + j];
    double sz = nearest_int(dz0 / Lz);
    double dz = dz0 - sz * Lz;
    d[0] = dx; d[1] = dy; d[2] = dz;
    if (img) { img[0] = (int32_t)sx; img[1] = (int32_t)sy; img[2] = (int32_t)sz; }
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    return r2;
}

/* O6 (brute force). All unordered pairs (i<j) with r^2 < rcut^2, written in  */
/* increasing (i, j) order.  Returns the pair count (may exceed cap; only the */
/* first cap pairs are written).                                             */
int64_t orc_pairs_brute(int64_t n, const double *x, double Delta, const double box[3],
                        double rcut, int64_t *pairs, int64_t cap)
{
    const double rc2 = rcut * rcut;
    int64_t m = 0;
    double d[3];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double r2 = orc_disp(x, n, i, j, Delta, box, d, NULL);
            if (r2 < rc2) {
                if (m < cap) { pairs[2 * m] = i; pairs[2 * m + 1] = j; }
                ++m;
            }
        }
    return m;
}

/* O6 (cells).  The same set through a cell grid of side >= rcut rebuilt from  */
/* the current (wrapped) positions.  Rows that touch the gradient faces see   */
/* the whole neighbouring row of the image box, whatever the offset; all      */
/* other neighbour cells are the usual 3x3x3 periodic block (Section 2.3).    */
/* Every candidate is tested with O5 itself.  Visits each unordered pair once */
/* through the callback-free loop below (j > i).                             */
typedef struct {
    int32_t nc[3];
    int64_t ncell;
    int64_t *start;   /* [ncell+1] */
    int32_t *list;    /* [n] tags sorted by cell */
    int32_t *cell_of; /* [n] */
} orc_grid;

static void grid_build(orc_grid *g, int64_t n, const double *x, const double box[3], double rcut)
{
    for (int a = 0; a < 3; ++a) {
        int32_t k = (int32_t)floor(box[a] / rcut);
        if (k < 1) k = 1;
        g->nc[a] = k;
    }
    g->ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int64_t *)calloc((size_t)g->ncell + 1, sizeof(int64_t));
    g->list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_cells(n, x, g->nc, box, g->cell_of, g->list);
    for (int64_t i = 0; i < n; ++i) g->start[g->cell_of[i] + 1]++;
    for (int64_t c = 0; c < g->ncell; ++c) g->start[c + 1] += g->start[c];
}

static void grid_free(orc_grid *g)
{
    free(g->start); free(g->list); free(g->cell_of);
}

/* Enumerate the distinct neighbour cells of cell (ix,iy,iz) as described     */
/* above.  Writes at most 27 + 2*9*nx ids; returns the count.                 */
static int grid_neighbours(const orc_grid *g, int32_t ix, int32_t iy, int32_t iz, int64_t *out)
{
    const int32_t nx = g->nc[0], ny = g->nc[1], nz = g->nc[2];
    int m = 0;
    int32_t zs[3], ys[3];
    int nzs = 0, nys = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int32_t c = ((iz + dz) % nz + nz) % nz;
        int dup = 0;
        for (int q = 0; q < nzs; ++q) dup |= (zs[q] == c);
        if (!dup) zs[nzs++] = c;
    }
    for (int dy = -1; dy <= 1; ++dy) {
        int32_t c = iy + dy;
        int32_t w = ((c % ny) + ny) % ny;
        int dup = 0;
        for (int q = 0; q < nys; ++q) dup |= (ys[q] == w);
        if (!dup) ys[nys++] = w;
    }
    for (int a = 0; a < nzs; ++a)
        for (int b = 0; b < nys; ++b) {
            int32_t yy = ys[b];
            /* a row reached across a gradient face is offset by the shear */
            int crosses = (iy == 0 && yy == ny - 1) || (iy == ny - 1 && yy == 0) || ny < 3;
            if (crosses) {
                for (int32_t xx = 0; xx < nx; ++xx) out[m++] = ((int64_t)zs[a] * ny + yy) * nx + xx;
            } else {
                int32_t xs[3];
                int nxs = 0;
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t c = ((ix + dx) % nx + nx) % nx;
                    int dup = 0;
                    for (int q = 0; q < nxs; ++q) dup |= (xs[q] == c);
                    if (!dup) xs[nxs++] = c;
                }
                for (int q = 0; q < nxs; ++q) out[m++] = ((int64_t)zs[a] * ny + yy) * nx + xs[q];
            }
        }
    return m;
}

/* Loop over every unordered pair with r^2 < rcut^2 found through the grid. */
typedef void (*pair_fn)(void *ctx, int64_t i, int64_t j, const double d[3], double r2);

static void grid_pairs(int64_t n, const double *x, double Delta, const double box[3],
                       double rcut, pair_fn fn, void *ctx)
{
    orc_grid g;
    grid_build(&g, n, x, box, rcut);
    const double rc2 = rcut * rcut;
    int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(27 + 18 * g.nc[0] + 16));
    double d[3];
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = g.cell_of[i];
        int32_t ix = c % g.nc[0];
        int32_t iy = (c / g.nc[0]) % g.nc[1];
        int32_t iz = c / (g.nc[0] * g.nc[1]);
        int m = grid_neighbours(&g, ix, iy, iz, nb);
        for (int q = 0; q < m; ++q) {
            for (int64_t s = g.start[nb[q]]; s < g.start[nb[q] + 1]; ++s) {
                int64_t j = g.list[s];
                if (j <= i) continue;
                double r2 = orc_disp(x, n, i, j, Delta, box, d, NULL);
                if (r2 < rc2) fn(ctx, i, j, d, r2);
            }
        }
    }
    free(nb);
    grid_free(&g);
}

typedef struct { int64_t *pairs; int64_t cap; int64_t m; } pair_collect;

static void collect_pair(void *ctx, int64_t i, int64_t j, const double d[3], double r2)
{
    (void)d; (void)r2;
    pair_collect *pc = (pair_collect *)ctx;
    if (pc->m < pc->cap) { pc->pairs[2 * pc->m] = i; pc->pairs[2 * pc->m + 1] = j; }
    pc->m++;
}

/* Pairs via the grid (unordered, i<j, in grid visiting order). */
int64_t orc_pairs_cells(int64_t n, const double *x, double Delta, const double box[3],
                        double rcut, int64_t *pairs, int64_t cap)
{
    pair_collect pc = {pairs, cap, 0};
    grid_pairs(n, x, Delta, box, rcut, collect_pair, &pc);
    return pc.m;
}

/* ------------------------------------------------------------------------ */
/* O7. Pair force and energy (Eqs. lj and lj-shift).  f is the scalar such   */
/* that the force on i from j is f * d (d = q_i - q_j).  The force is the    */
/* plain truncated derivative of 4 eps[(s/r)^12 - (s/r)^6]; the WCA form of  */
/* Eq. lj-shift differs only by a constant, so it has the same force inside  */
/* its cutoff.  energy: V(r) + shift.                                        */
static void pair_lj(double r2, const orc_params *p, double *f, double *e)
{
    double s2 = (p->sigma * p->sigma) / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    *f = 24.0 * p->eps * (2.0 * s12 - s6) / r2;
    *e = 4.0 * p->eps * (s12 - s6) + p->lj_shift;
    /* Warm-up of overlapping starts (the equilibration before shear of      */
    /* Section 2.4): the magnitude |f| r of the pair force is limited to     */
    /* force_cap, its direction kept.  The energy is left as it is (it is    */
    /* not used while capped).                                               */
    if (p->force_cap > 0.0) {
        double lim = p->force_cap / sqrt(r2);
        if (*f > lim) *f = lim;
        if (*f < -lim) *f = -lim;
    }
}

/* O8. FENE bond (Eq. fene): V = -1/2 k R0^2 ln(1 - r^2/R0^2) for r < R0,     */
/* +infinity otherwise.  Force on i is -k d / (1 - r^2/R0^2).                 */
static int bond_fene(double r2, const orc_params *p, double *f, double *e)
{
    double R02 = p->fene_r0 * p->fene_r0;
    if (!(r2 < R02)) return ORC_E_BOND;
    double q = 1.0 - r2 / R02;
    *f = -p->fene_k / q;
    *e = -0.5 * p->fene_k * R02 * log(q);
    return ORC_OK;
}

typedef struct {
    const orc_params *p;
    double *F;        /* [3][n] accumulated conservative force */
    double *W;        /* [6] sum over pairs of d_a * F_b (xx,yy,zz,xy,xz,yz) */
    double *e;        /* potential energy */
    int64_t n;
} force_ctx;

static void add_pair_force(force_ctx *fc, int64_t i, int64_t j, const double d[3], double f, double e)
{
    const int64_t n = fc->n;
    for (int a = 0; a < 3; ++a) {
        double fa = f * d[a];
        fc->F[a * n + i] += fa;
        fc->F[a * n + j] -= fa;
    }
    if (fc->W) {
        double fx = f * d[0], fy = f * d[1], fz = f * d[2];
        fc->W[0] += d[0] * fx; fc->W[1] += d[1] * fy; fc->W[2] += d[2] * fz;
        fc->W[3] += d[0] * fy; fc->W[4] += d[0] * fz; fc->W[5] += d[1] * fz;
    }
    if (fc->e) *fc->e += e;
}

static void lj_pair_cb(void *ctx, int64_t i, int64_t j, const double d[3], double r2)
{
    force_ctx *fc = (force_ctx *)ctx;
    double f, e;
    pair_lj(r2, fc->p, &f, &e);
    add_pair_force(fc, i, j, d, f, e);
}

/* Bonds: linear chains, tag = chain*chain_len + k, bonded to k+1 in-chain. */
static int add_bonds(const double *x, double Delta, force_ctx *fc)
{
    const orc_params *p = fc->p;
    if (p->chain_len <= 0) return ORC_OK;
    double d[3];
    for (int64_t c = 0; c < p->n_chains; ++c)
        for (int32_t k = 0; k + 1 < p->chain_len; ++k) {
            int64_t i = c * p->chain_len + k, j = i + 1;
            double r2 = orc_disp(x, fc->n, i, j, Delta, p->box, d, NULL);
            double f, e;
            if (bond_fene(r2, p, &f, &e) != ORC_OK) return ORC_E_BOND;
            add_pair_force(fc, i, j, d, f, e);
        }
    return ORC_OK;
}

/* Cosine angle term of the KG chains (Eq. angle), read as the standard       */
/* bending potential k_a (1 - cos(theta - theta_0)) with theta_0 = 180 deg,   */
/* i.e. V = k_a (1 + cos theta), theta the angle at the middle bead j of       */
/* consecutive beads (a, j, b) between b1 = x_a - x_j and b2 = x_b - x_j      */
/* (Lees-Edwards nearest images): zero for a straight chain.  F = -grad V:    */
/*   F_a = -k_a [b2 / (l1 l2) - cos(theta) b1 / l1^2],  F_b likewise,          */
/*   F_j = -(F_a + F_b); virial of the angle b1 (x) F_a + b2 (x) F_b.           */
static void angle_cos(const double b1[3], const double b2[3], double k, double Fa[3], double Fb[3],
                      double *e)
{
    double l11 = b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2];
    double l22 = b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2];
    double l12 = sqrt(l11) * sqrt(l22);
    double c = (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / l12;
    *e = k * (1.0 + c);
    for (int a = 0; a < 3; ++a) {
        Fa[a] = -k * (b2[a] / l12 - c * b1[a] / l11);
        Fb[a] = -k * (b1[a] / l12 - c * b2[a] / l22);
    }
}

static void add_angles(const double *x, double Delta, force_ctx *fc)
{
    const orc_params *p = fc->p;
    const int64_t n = fc->n;
    if (p->chain_len < 3 || p->angle_k == 0.0) return;
    double b1[3], b2[3], Fa[3], Fb[3], e;
    for (int64_t c = 0; c < p->n_chains; ++c)
        for (int32_t k = 1; k + 1 < p->chain_len; ++k) {
            int64_t j = c * p->chain_len + k, a = j - 1, b = j + 1;
            orc_disp(x, n, a, j, Delta, p->box, b1, NULL);
            orc_disp(x, n, b, j, Delta, p->box, b2, NULL);
            angle_cos(b1, b2, p->angle_k, Fa, Fb, &e);
            for (int q = 0; q < 3; ++q) {
                fc->F[q * n + a] += Fa[q];
                fc->F[q * n + b] += Fb[q];
                fc->F[q * n + j] -= Fa[q] + Fb[q];
            }
            if (fc->W) {
                fc->W[0] += b1[0] * Fa[0] + b2[0] * Fb[0];
                fc->W[1] += b1[1] * Fa[1] + b2[1] * Fb[1];
                fc->W[2] += b1[2] * Fa[2] + b2[2] * Fb[2];
                fc->W[3] += b1[0] * Fa[1] + b2[0] * Fb[1];
                fc->W[4] += b1[0] * Fa[2] + b2[0] * Fb[2];
                fc->W[5] += b1[1] * Fa[2] + b2[1] * Fb[2];
            }
            if (fc->e) *fc->e += e;
        }
}

#ifdef _OPENMP
/* Timing build only (gcc -fopenmp, the CPU baseline of the benchmark): the   */
/* grid loop of O6 split over threads by particle i, each thread summing into */
/* its own force, virial and energy arrays, which are then added together.    */
/* The pairs and the force law are those of the serial loop; only the order   */
/* of the sums differs.  The parity tests use the serial build.              */
static void grid_forces_parallel(int64_t n, const double *x, double Delta, force_ctx *fc)
{
    const orc_params *p = fc->p;
    orc_grid g;
    grid_build(&g, n, x, p->box, p->rc);
    const double rc2 = p->rc * p->rc;
    const int nth = omp_get_max_threads();
    double *Fs = (double *)calloc((size_t)nth * 3 * (size_t)n, sizeof(double));
    double *Ws = (double *)calloc((size_t)nth * 7, sizeof(double));
#pragma omp parallel
    {
        const int t = omp_get_thread_num();
        force_ctx loc = {p, Fs + (size_t)t * 3 * (size_t)n, fc->W ? Ws + 7 * t : NULL,
                         fc->e ? Ws + 7 * t + 6 : NULL, n};
        int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(27 + 18 * g.nc[0] + 16));
        double d[3];
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int32_t c = g.cell_of[i];
            int32_t ix = c % g.nc[0];
            int32_t iy = (c / g.nc[0]) % g.nc[1];
            int32_t iz = c / (g.nc[0] * g.nc[1]);
            int m = grid_neighbours(&g, ix, iy, iz, nb);
            for (int q = 0; q < m; ++q)
                for (int64_t s = g.start[nb[q]]; s < g.start[nb[q] + 1]; ++s) {
                    int64_t j = g.list[s];
                    if (j <= i) continue;
                    double r2 = orc_disp(x, n, i, j, Delta, p->box, d, NULL);
                    if (r2 < rc2) lj_pair_cb(&loc, i, j, d, r2);
                }
        }
        free(nb);
#pragma omp for schedule(static)
        for (int64_t k = 0; k < 3 * n; ++k)
            for (int u = 0; u < nth; ++u) fc->F[k] += Fs[(size_t)u * 3 * (size_t)n + (size_t)k];
    }
    for (int u = 0; u < nth; ++u) {
        if (fc->W) for (int a = 0; a < 6; ++a) fc->W[a] += Ws[7 * u + a];
        if (fc->e) *fc->e += Ws[7 * u + 6];
    }
    free(Fs);
    free(Ws);
    grid_free(&g);
}
#endif

/* Threads of the timing build (no effect in the serial build); returns the  */
/* number in use.                                                            */
int orc_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Conservative forces (pairs + bonds) of a configuration, plus the virial   */
/* W_ab = sum_{i<j} d_a F_ij,b and the potential energy.  method 0: all      */
/* pairs by brute force; 1: through the grid of O6.  F, W6, energy may be    */
/* NULL except F.  Returns 0 or ORC_E_BOND.                                  */
int orc_forces(int64_t n, const double *x, double Delta, const orc_params *p, int method,
               double *F, double *W6, double *energy)
{
    force_ctx fc = {p, F, W6, energy, n};
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    if (W6) memset(W6, 0, sizeof(double) * 6);
    if (energy) *energy = 0.0;
    if (method == 0) {
        const double rc2 = p->rc * p->rc;
        double d[3];
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double r2 = orc_disp(x, n, i, j, Delta, p->box, d, NULL);
                if (r2 < rc2) lj_pair_cb(&fc, i, j, d, r2);
            }
    } else {
#ifdef _OPENMP
        if (omp_get_max_threads() > 1) grid_forces_parallel(n, x, Delta, &fc);
        else
#endif
        grid_pairs(n, x, Delta, p->box, p->rc, lj_pair_cb, &fc);
    }
    int rc = add_bonds(x, Delta, &fc);
    if (rc == ORC_OK) add_angles(x, Delta, &fc);
    return rc;
}

/* Conservative force on a few chosen particles, each summed over every other */
/* particle in increasing tag order (used to check large systems by sample).  */
int orc_forces_sample(int64_t n, const double *x, double Delta, const orc_params *p,
                      int64_t ns, const int64_t *idx, double *Fs /* [ns][3] */)
{
    const double rc2 = p->rc * p->rc;
    double d[3];
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = idx[s];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = orc_disp(x, n, i, j, Delta, p->box, d, NULL);
            if (r2 < rc2) {
                double f, e;
                pair_lj(r2, p, &f, &e);
                for (int a = 0; a < 3; ++a) acc[a] += f * d[a];
            }
        }
        if (p->chain_len > 0) {
            int64_t k = i % p->chain_len;
            int64_t nb[2] = {k > 0 ? i - 1 : -1, k + 1 < p->chain_len ? i + 1 : -1};
            for (int q = 0; q < 2; ++q) {
                if (nb[q] < 0) continue;
                double r2 = orc_disp(x, n, i, nb[q], Delta, p->box, d, NULL);
                double f, e;
                if (bond_fene(r2, p, &f, &e) != ORC_OK) return ORC_E_BOND;
                for (int a = 0; a < 3; ++a) acc[a] += f * d[a];
            }
            /* angles centred at i - 1 (i is its second end), at i, and at */
            /* i + 1 (i is its first end)                                   */
            if (p->chain_len >= 3 && p->angle_k != 0.0) {
                for (int64_t cj = i - 1; cj <= i + 1; ++cj) {
                    int64_t kc = k + (cj - i);
                    if (kc < 1 || kc + 1 >= p->chain_len) continue;
                    double b1[3], b2[3], Fa[3], Fb[3], e;
                    orc_disp(x, n, cj - 1, cj, Delta, p->box, b1, NULL);
                    orc_disp(x, n, cj + 1, cj, Delta, p->box, b2, NULL);
                    angle_cos(b1, b2, p->angle_k, Fa, Fb, &e);
                    for (int a = 0; a < 3; ++a)
                        acc[a] += (cj == i + 1) ? Fa[a] : (cj == i - 1) ? Fb[a] : -(Fa[a] + Fb[a]);
                }
            }
        }
        for (int a = 0; a < 3; ++a) Fs[3 * s + a] = acc[a];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O10. Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the  */
/* two 32x32->64 multiplies with the published multipliers, the key bumped   */
/* by the published Weyl constants between rounds.                           */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Thermostat noise of one particle at one step: counter (step lo, step hi,  */
/* tag, 0), key (seed lo, seed hi); each 32-bit word r maps to the uniform    */
/* (r + 1/2) 2^-32 - 1/2 in (-1/2, 1/2), the theta of Eqs. random and omega.  */
void orc_noise(uint64_t seed, int64_t step, int64_t tag, double theta[3])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)step), (uint32_t)((uint64_t)step >> 32), (uint32_t)tag, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox(ctr, key, r);
    for (int a = 0; a < 3; ++a) theta[a] = ((double)r[a] + 0.5) * (1.0 / 4294967296.0) - 0.5;
}

/* Uniform pair noise of the DPD random force (Eq. random): one Philox block */
/* per unordered pair and step, counter (step lo, step hi, smaller tag,      */
/* larger tag), key (seed lo, seed hi xor 0x44504421) so that the stream is  */
/* apart from the per-particle Langevin noise; word 0 maps to (-1/2, 1/2).   */
double orc_dpd_theta(uint64_t seed, int64_t step, int64_t ti, int64_t tj)
{
    int64_t a = ti < tj ? ti : tj, b = ti < tj ? tj : ti;
    uint32_t ctr[4] = {(uint32_t)((uint64_t)step), (uint32_t)((uint64_t)step >> 32), (uint32_t)a,
                       (uint32_t)b};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x44504421u};
    uint32_t r[4];
    orc_philox(ctr, key, r);
    return ((double)r[0] + 0.5) * (1.0 / 4294967296.0) - 0.5;
}

/* DPD thermostat (Eqs. dissipative, random, omega), read as the standard    */
/* pairwise form: for every pair with r < dpd_rc, with e = d/r the unit       */
/* displacement from j's image to i, v_ij = u_i - u_j - s_y gamma_dot L_y e_x */
/* the velocity of i relative to that image (an image one box up streams     */
/* faster by gamma_dot L_y) and w = 1 - r/dpd_rc,                             */
/*   F_i += [-gamma w^2 (e . v_ij) + sqrt(24 gamma kT / dt) w theta_ij] e,     */
/*   F_j -= the same.                                                          */
/* The total force is F^c plus these pair terms only (no per-particle drag). */
/* The pairs come from the brute-force loop (method 0) or the grid of O6     */
/* (method 1), which visit the same pair set.                                */
typedef struct {
    int64_t n, step;
    const double *x, *u;
    double *F;
    double Delta, sv, pref;
    const orc_params *p;
} dpd_ctx;

static void dpd_pair_cb(void *ctx, int64_t i, int64_t j, const double d_in[3], double r2_in)
{
    dpd_ctx *c = (dpd_ctx *)ctx;
    const int64_t n = c->n;
    const double *u = c->u;
    double d[3];
    int32_t img[3];
    double r2 = orc_disp(c->x, n, i, j, c->Delta, c->p->box, d, img);
    (void)d_in; (void)r2_in;
    double r = sqrt(r2);
    double e[3] = {d[0] / r, d[1] / r, d[2] / r};
    double v[3] = {(u[i] - u[j]) - (double)img[1] * c->sv, u[n + i] - u[n + j],
                   u[2 * n + i] - u[2 * n + j]};
    double w = 1.0 - r / c->p->dpd_rc;
    double ev = e[0] * v[0] + e[1] * v[1];
    ev = ev + e[2] * v[2];
    double f = -c->p->gamma * w * w * ev + c->pref * w * orc_dpd_theta(c->p->seed, c->step, i, j);
    for (int a = 0; a < 3; ++a) {
        c->F[a * n + i] += f * e[a];
        c->F[a * n + j] -= f * e[a];
    }
}

/* The DPD pair terms alone on a few chosen particles, each summed over every */
/* other particle in increasing tag order (to check large systems by sample);  */
/* out Gs[ns][3].  Same pair law as below, evaluated from i's side.             */
void orc_dpd_sample(int64_t n, const double *x, const double *u, double Delta, const orc_params *p,
                    int64_t step, int64_t ns, const int64_t *idx, double *Gs)
{
    const double sv = p->shear_rate * p->box[1];
    const double rd2 = p->dpd_rc * p->dpd_rc;
    const double pref = sqrt(24.0 * p->gamma * p->kT / p->dt);
    double d[3];
    int32_t img[3];
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t i = idx[s];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = orc_disp(x, n, i, j, Delta, p->box, d, img);
            if (!(r2 < rd2)) continue;
            double r = sqrt(r2);
            double e[3] = {d[0] / r, d[1] / r, d[2] / r};
            double v[3] = {(u[i] - u[j]) - (double)img[1] * sv, u[n + i] - u[n + j],
                           u[2 * n + i] - u[2 * n + j]};
            double w = 1.0 - r / p->dpd_rc;
            double ev = e[0] * v[0] + e[1] * v[1];
            ev = ev + e[2] * v[2];
            double f = -p->gamma * w * w * ev + pref * w * orc_dpd_theta(p->seed, step, i, j);
            for (int a = 0; a < 3; ++a) acc[a] += f * e[a];
        }
        for (int a = 0; a < 3; ++a) Gs[3 * s + a] = acc[a];
    }
}

static void thermostat_dpd(int64_t n, const double *x, const double *u, const double *Fc,
                           double *F, int64_t step, double Delta, const orc_params *p, int method)
{
    dpd_ctx c = {n, step, x, u, F, Delta, p->shear_rate * p->box[1],
                 sqrt(24.0 * p->gamma * p->kT / p->dt), p};
    const double rd2 = p->dpd_rc * p->dpd_rc;
    for (int64_t k = 0; k < 3 * n; ++k) F[k] = Fc[k];
    if (method == 0) {
        double d[3];
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double r2 = orc_disp(x, n, i, j, Delta, p->box, d, NULL);
                if (r2 < rd2) dpd_pair_cb(&c, i, j, d, r2);
            }
    } else {
        grid_pairs(n, x, Delta, p->box, p->dpd_rc, dpd_pair_cb, &c);
    }
}

/* Eq. langevin with the friction acting on the peculiar velocity           */
/* c = u - shear_rate (y - L_y/2) e_x (Eqs. shear-rate, vi): the total force  */
/* on one particle is F^c - gamma m c + sqrt(24 gamma m kT / dt) theta.       */
/* Thermostat 2 applies the friction to the lab velocity u instead (the      */
/* paper's xi_abs, Section 3.1), which drags the flow profile.  With         */
/* peculiar storage u already is c.                                          */
static void thermostat(int64_t n, const double *x, const double *u, const double *Fc,
                       double *F, int64_t step, const orc_params *p)
{
    const double Ly = p->box[1];
    const double pref = sqrt(24.0 * p->gamma * p->mass * p->kT / p->dt);
    const double sr = (p->thermostat == 2 || p->velocity == 1) ? 0.0 : p->shear_rate;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double c[3];
        c[0] = u[i] - sr * (x[n + i] - 0.5 * Ly);
        c[1] = u[n + i];
        c[2] = u[2 * n + i];
        double th[3];
        orc_noise(p->seed, step, i, th);
        for (int a = 0; a < 3; ++a)
            F[a * n + i] = Fc[a * n + i] - p->gamma * p->mass * c[a] + pref * th[a];
    }
}

/* O11. Irving-Kirkwood stress (Eq. tensor): sigma_ab = -(1/V)[sum_i m c_a   */
/* c_b + sum_{i<j} d_a F_ij,b] with the peculiar velocity c and conservative  */
/* forces only.  Order: xx, yy, zz, xy, xz, yz.  W6 is the pair virial.       */
void orc_stress(int64_t n, const double *x, const double *u, const double *W6,
                const orc_params *p, double *sig6)
{
    const double Ly = p->box[1];
    const double V = p->box[0] * p->box[1] * p->box[2];
    double K[6] = {0, 0, 0, 0, 0, 0};
    const double csr = p->velocity == 1 ? 0.0 : p->shear_rate;
    for (int64_t i = 0; i < n; ++i) {
        double cx = u[i] - csr * (x[n + i] - 0.5 * Ly);
        double cy = u[n + i], cz = u[2 * n + i];
        K[0] += p->mass * cx * cx; K[1] += p->mass * cy * cy; K[2] += p->mass * cz * cz;
        K[3] += p->mass * cx * cy; K[4] += p->mass * cx * cz; K[5] += p->mass * cy * cz;
    }
    for (int a = 0; a < 6; ++a) sig6[a] = -(K[a] + W6[a]) / V;
}

/* ------------------------------------------------------------------------ */
/* O9. One velocity-Verlet step n -> n+1 with the Lees-Edwards crossing and   */
/* the Langevin force on the peculiar velocity.  State (x, u, F) at step n,   */
/* F being the total force (conservative + thermostat) of step n.            */
/*   1) u += dt/(2m) F          2) x += dt u                                 */
/*   3) Delta_{n+1} (O1)        4) O3: every particle that crossed a face    */
/*                                 re-enters with the shift and velocity jump */
/*   5) F^c(x_{n+1}) (O7, O8)   6) F = F^c - gamma m c + P theta(n+1)         */
/*   7) u += dt/(2m) F                                                        */
/* Fc_out (may be NULL) receives F^c; W6 (may be NULL) its pair virial.       */
int orc_step(int64_t n, double *x, double *u, double *F, int64_t *step, const orc_params *p,
             int method, double *Fc_out, double *W6)
{
    const double h = 0.5 * p->dt / p->mass;
    for (int64_t k = 0; k < 3 * n; ++k) u[k] = u[k] + h * F[k];
    if (p->velocity == 1) {
        /* peculiar storage: x moves with u_x plus the streaming velocity at */
        /* the particle's height before the drift                            */
        for (int64_t i = 0; i < n; ++i)
            x[i] = x[i] + p->dt * (u[i] + p->shear_rate * (x[n + i] - 0.5 * p->box[1]));
        for (int64_t k = n; k < 3 * n; ++k) x[k] = x[k] + p->dt * u[k];
    } else {
        for (int64_t k = 0; k < 3 * n; ++k) x[k] = x[k] + p->dt * u[k];
    }
    int64_t s = *step + 1;
    double Delta = orc_offset(s, p->dt, p->shear_rate, p->box[0], p->box[1]);
    /* a peculiar velocity is continuous across the sheared faces: no jump */
    orc_le_wrap(n, x, p->velocity == 1 ? NULL : u, Delta, p);
    double *Fc = Fc_out ? Fc_out : (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int rc = orc_forces(n, x, Delta, p, method, Fc, W6, NULL);
    if (rc != ORC_OK) { if (!Fc_out) free(Fc); return rc; }
    if (p->thermostat == 1) thermostat_dpd(n, x, u, Fc, F, s, Delta, p, method);
    else thermostat(n, x, u, Fc, F, s, p);
    for (int64_t k = 0; k < 3 * n; ++k) u[k] = u[k] + h * F[k];
    for (int64_t k = 0; k < 3 * n; ++k)
        if (!isfinite(x[k]) || !isfinite(u[k])) { if (!Fc_out) free(Fc); return ORC_E_NONFINITE; }
    *step = s;
    if (!Fc_out) free(Fc);
    return ORC_OK;
}

/* Step-0 set-up: wrap the given state with Delta_{step0} (O3) and compute    */
/* the total force of that step (conservative + thermostat with theta(step0)). */
int orc_init(int64_t n, double *x, double *u, double *F, int64_t step0, const orc_params *p,
             int method)
{
    double Delta = orc_offset(step0, p->dt, p->shear_rate, p->box[0], p->box[1]);
    orc_le_wrap(n, x, p->velocity == 1 ? NULL : u, Delta, p);
    double *Fc = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int rc = orc_forces(n, x, Delta, p, method, Fc, NULL, NULL);
    if (rc == ORC_OK) {
        if (p->thermostat == 1) thermostat_dpd(n, x, u, Fc, F, step0, Delta, p, method);
        else thermostat(n, x, u, Fc, F, step0, p);
    }
    free(Fc);
    return rc;
}

/* Run nsteps; every sample_every steps (counted from the start of the run)   */
/* write the stress of the new state into stress_out[k][6].                  */
int orc_run(int64_t n, double *x, double *u, double *F, int64_t *step, const orc_params *p,
            int method, int64_t nsteps, int64_t sample_every, double *stress_out)
{
    double *Fc = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double W6[6];
    int64_t ns = 0;
    int rc = ORC_OK;
    for (int64_t k = 1; k <= nsteps; ++k) {
        rc = orc_step(n, x, u, F, step, p, method, Fc, W6);
        if (rc != ORC_OK) break;
        if (sample_every > 0 && stress_out && k % sample_every == 0) {
            orc_stress(n, x, u, W6, p, &stress_out[6 * ns]);
            ns++;
        }
    }
    free(Fc);
    return rc;
}

/* O12. Observables of a state: nbins-bin profiles along the gradient axis of */
/* the particle count, of the summed flow velocity (Fig. profile) and of the  */
/* summed peculiar kinetic term m c^2 (the temperature profile, three times   */
/* kT per particle in equilibrium), using the wrapped y and the lab u_x of    */
/* the wrapped image; kinetic temperature of the peculiar velocities          */
/* sum m c^2 / (3N - 3); centre-of-mass lab velocity.                         */
void orc_observables(int64_t n, const double *x, const double *u, double Delta, const orc_params *p,
                     int32_t nbins, double *count, double *sum_ux, double *sum_mc2, double *kT_kin,
                     double com[3])
{
    const double Ly = p->box[1];
    const double sv = p->shear_rate * Ly;
    (void)Delta;
    for (int32_t b = 0; b < nbins; ++b) { count[b] = 0.0; sum_ux[b] = 0.0; sum_mc2[b] = 0.0; }
    double k2 = 0.0;
    com[0] = com[1] = com[2] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double y = x[n + i];
        double ky = orc_wrap(&y, Ly);
        /* lab u_x of the in-box image */
        double ux = p->velocity == 1 ? u[i] + p->shear_rate * (y - 0.5 * Ly) : u[i] - ky * sv;
        int32_t b = (int32_t)(y / Ly * (double)nbins);
        if (b < 0) b = 0;
        if (b > nbins - 1) b = nbins - 1;
        count[b] += 1.0;
        sum_ux[b] += ux;
        double cx = p->velocity == 1 ? u[i] : u[i] - p->shear_rate * (x[n + i] - 0.5 * Ly);
        double mc2 = p->mass * (cx * cx + u[n + i] * u[n + i] + u[2 * n + i] * u[2 * n + i]);
        sum_mc2[b] += mc2;
        k2 += mc2;
        com[0] += ux; com[1] += u[n + i]; com[2] += u[2 * n + i];
    }
    *kT_kin = k2 / (3.0 * (double)n - 3.0);
    for (int a = 0; a < 3; ++a) com[a] /= (double)n;
}

/* Potential energy only (for conservation and derivative checks). */
int orc_energy(int64_t n, const double *x, double Delta, const orc_params *p, double *energy)
{
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int rc = orc_forces(n, x, Delta, p, 0, F, NULL, energy);
    free(F);
    return rc;
}

/*
 * Parity pins (tests/test_oracle_*.py):
 *   O1 offset         closed form, periodicity in L_x, sign of shear rate
 *   O2/O3 wrap        edge-case table in tests/golden, affine-flow invariance
 *   O4/O5/O6 cells    brute force vs grid, explicit sheared-image replication,
 *                     Delta = 0 reduces to the periodic minimum image
 *   O7/O8 forces      closed forms, finite differences of the energy
 *   O11 virial        affine-strain derivative of the energy
 *   O9 step           NVE energy drift, time reversal, exact momentum rule
 *   O10 Philox        the ROCm rocRAND engine on the host, uniform moments
 *   O12 observables   ideal-gas equipartition, linear velocity profile
 */
