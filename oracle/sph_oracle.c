/*
 * FP64 CPU oracle of the two-fluid SPH step with spin angular momentum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * It is deliberately plain: every particle gathers its neighbour set, sorts it by
 * particle id and sums in that order, all in double precision.  OpenMP only spreads
 * independent particles over threads; it does not change any result.
 *
 * What it computes (the discrete model is this project's reading of the paper; the
 * paper's own SPH operator list is an appendix figure that is not reproduced):
 *   - governing equations: Eq. 1 (inviscid component) and Eq. 2 (viscous component
 *     with shear + rotational viscosity and the spin term 2 eta_r curl(omega_0)),
 *     with the grad-div term dropped as the paper states for div v = 0 (Sec. 2.1);
 *   - Tait equation of state, Eq. 4, with beta_P = p_0 (Sec. 2.1);
 *   - local interaction force F_sn = C_l v_sn between unlike particles, each particle
 *     pulled toward the kernel-weighted mean velocity of its unlike neighbours with the
 *     reaction returned to them (Sec. 2.1, and the two passes of Algorithm 1);
 *   - interfacial (temperature-gradient) force between unlike particles, horizontal only
 *     (Sec. 2.1);
 *   - wall and dummy particles: inner wall layer gets summed density/pressure, outer
 *     layers keep their initial density and pressure (Sec. 3);
 *   - optional pressure filter and collision step of Algorithm 1, in this project's
 *     reading (the paper cites both models without their formulas);
 *   - velocity Verlet time integration (Sec. 2.3, Algorithm 1);
 *   - neighbour search by a cell-linked list (Sec. 2.3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_E_INVALID = 1, OR_E_DOMAIN = 5, OR_E_NONFINITE = 6, OR_E_CAP = 8 };
enum { OR_CUBIC = 0, OR_WENDLAND = 1 };
enum { OR_PERIODIC_BOX = 0, OR_CYLINDER_Z = 1, OR_OPEN = 2 };
enum { OR_FLUID = 0, OR_WALL_INNER = 1, OR_WALL_OUTER = 2 };

typedef struct {
    int32_t kernel;
    int32_t geometry;
    int32_t cell_factor;
    int32_t pad;
    double dx, h;
    double lo[3], hi[3];
    double rho0, c0, gamma;
    double mass[2];
    double eta, sigma_T, C_l, kappa_I;
    int32_t pressure_filter;   /* 0: none, 1: Shepard average of P (Algorithm 1)          */
    int32_t pad2;
    double coll_alpha;         /* collision distance / dx; 0: no collision step           */
    double coll_e;             /* restitution of the collision step, in [0, 1]            */
} or_params;

/* ------------------------------------------------------------------------------------
 * Smoothing kernels (3D, support radius 2h), q = r / h.
 * Cubic spline: W = 1/(pi h^3) * { 1 - 3/2 q^2 + 3/4 q^3 (q<1); 1/4 (2-q)^3 (q<2) }.
 * Wendland C2:  W = 21/(16 pi h^3) * (1 - q/2)^4 (2q + 1)  (q<2).
 * ---------------------------------------------------------------------------------- */
double or_W(int kernel, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    if (kernel == OR_CUBIC) {
        double s = 1.0 / (M_PI * h * h * h);
        if (q < 1.0) return s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
        double t = 2.0 - q;
        return s * 0.25 * t * t * t;
    } else {
        double s = 21.0 / (16.0 * M_PI * h * h * h);
        double t = 1.0 - 0.5 * q;
        return s * t * t * t * t * (2.0 * q + 1.0);
    }
}

/* dW/dr */
double or_dWdr(int kernel, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    if (kernel == OR_CUBIC) {
        double s = 1.0 / (M_PI * h * h * h);
        double dq;
        if (q < 1.0) dq = -3.0 * q + 2.25 * q * q;
        else { double t = 2.0 - q; dq = -0.75 * t * t; }
        return s * dq / h;
    } else {
        double s = 21.0 / (16.0 * M_PI * h * h * h);
        double t = 1.0 - 0.5 * q;
        /* d/dq [(1-q/2)^4 (2q+1)] = -2(1-q/2)^3(2q+1) + 2(1-q/2)^4 = -5 q (1-q/2)^3 */
        return s * (-5.0 * q * t * t * t) / h;
    }
}

/* F(r) = -W'(r)/r, so that grad_i W_ij = -F r_ij.  Finite limit at r = 0. */
static double kernel_F(int kernel, double h, double r)
{
    return -or_dWdr(kernel, h, r) / r;
}

/* Lattice normalisation: lambda = dx^3 * sum over integer n of W(|n| dx), n = 0 included.
 * A perfect cubic lattice of spacing dx with mass rho0 dx^3 / lambda then has density
 * exactly rho0 under the kernel-summed density. */
double or_lambda(int kernel, double h, double dx)
{
    int m = (int)ceil(2.0 * h / dx) + 1;
    double s = 0.0;
    for (int a = -m; a <= m; a++)
        for (int b = -m; b <= m; b++)
            for (int c = -m; c <= m; c++) {
                double r = dx * sqrt((double)(a * a + b * b + c * c));
                s += or_W(kernel, h, r);
            }
    return s * dx * dx * dx;
}

static void particle_masses(const or_params *p, double m[2])
{
    double dflt = p->rho0 * p->dx * p->dx * p->dx / or_lambda(p->kernel, p->h, p->dx);
    for (int s = 0; s < 2; s++) m[s] = p->mass[s] > 0.0 ? p->mass[s] : dflt;
}

/* ------------------------------------------------------------------------------------
 * Cell grid.  Periodic axis: n = floor(cf * L / (2h)), edge = L / n.
 * Open axis: n = ceil(cf * L / (2h)), edge = (2h) / cf.  Cell coordinate
 * c = floor((x - lo) / edge) with IEEE division; periodic axes clamp to [0, n-1], open
 * axes report a domain error outside it.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int n[3];
    int periodic[3];
    double edge[3];
    double L[3];
    int cf;
} grid_t;

static int is_periodic(const or_params *p, int a)
{
    if (p->geometry == OR_PERIODIC_BOX) return 1;
    if (p->geometry == OR_CYLINDER_Z) return a == 2;
    return 0;
}

static int make_grid(const or_params *p, grid_t *g)
{
    if (!(p->h > 0.0) || !(p->dx > 0.0) || p->cell_factor < 1 || p->cell_factor > 4) return OR_E_INVALID;
    if (p->gamma != 7.0) return OR_E_INVALID;
    double two_h = 2.0 * p->h;
    if (p->pressure_filter != 0 && p->pressure_filter != 1) return OR_E_INVALID;
    if (!(p->coll_alpha >= 0.0) || !(p->coll_alpha * p->dx < two_h)) return OR_E_INVALID;
    if (!(p->coll_e >= 0.0 && p->coll_e <= 1.0)) return OR_E_INVALID;
    g->cf = p->cell_factor;
    for (int a = 0; a < 3; a++) {
        g->L[a] = p->hi[a] - p->lo[a];
        if (!(g->L[a] > 0.0)) return OR_E_INVALID;
        g->periodic[a] = is_periodic(p, a);
        if (g->periodic[a]) {
            g->n[a] = (int)floor((double)g->cf * g->L[a] / two_h);
            if (g->n[a] < 2 * g->cf + 1) return OR_E_INVALID;
            g->edge[a] = g->L[a] / (double)g->n[a];
        } else {
            g->n[a] = (int)ceil((double)g->cf * g->L[a] / two_h);
            if (g->n[a] < 1) g->n[a] = 1;
            g->edge[a] = two_h / (double)g->cf;
        }
        if (g->n[a] > 1024) return OR_E_INVALID;
    }
    return OR_OK;
}

static int cell_coord(const or_params *p, const grid_t *g, int a, double x, int *c)
{
    double t = (x - p->lo[a]) / g->edge[a];
    if (!(t == t)) return OR_E_NONFINITE;
    double f = floor(t);
    if (g->periodic[a]) {
        if (f < 0.0) f = 0.0;
        if (f > (double)(g->n[a] - 1)) f = (double)(g->n[a] - 1);
    } else if (f < 0.0 || f > (double)(g->n[a] - 1)) {
        return OR_E_DOMAIN;
    }
    *c = (int)f;
    return OR_OK;
}

static uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t k = 0;
    for (int b = 0; b < 10; b++) {
        k |= ((x >> b) & 1u) << (3 * b);
        k |= ((y >> b) & 1u) << (3 * b + 1);
        k |= ((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

/* Search structure: particles bucketed by linear cell index, ascending id inside. */
typedef struct {
    grid_t g;
    int64_t ncell;
    int64_t *start;   /* ncell + 1 */
    int64_t *items;   /* n */
    int32_t *cxyz;    /* 3n */
} cells_t;

static void cells_free(cells_t *c)
{
    free(c->start); free(c->items); free(c->cxyz);
    memset(c, 0, sizeof(*c));
}

static int cells_build(const or_params *p, int64_t n, const double *x, cells_t *c)
{
    memset(c, 0, sizeof(*c));
    int st = make_grid(p, &c->g);
    if (st) return st;
    c->ncell = (int64_t)c->g.n[0] * c->g.n[1] * c->g.n[2];
    c->start = (int64_t *)calloc((size_t)c->ncell + 1, sizeof(int64_t));
    c->items = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    c->cxyz = (int32_t *)malloc((size_t)(n > 0 ? 3 * n : 1) * sizeof(int32_t));
    if (!c->start || !c->items || !c->cxyz) { cells_free(c); return OR_E_INVALID; }
    for (int64_t i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++) {
            st = cell_coord(p, &c->g, a, x[a * n + i], &c->cxyz[3 * i + a]);
            if (st) { cells_free(c); return st; }
        }
        int64_t lin = c->cxyz[3 * i] + (int64_t)c->g.n[0] * (c->cxyz[3 * i + 1] + (int64_t)c->g.n[1] * c->cxyz[3 * i + 2]);
        c->start[lin + 1]++;
    }
    for (int64_t k = 0; k < c->ncell; k++) c->start[k + 1] += c->start[k];
    int64_t *fill = (int64_t *)malloc((size_t)c->ncell * sizeof(int64_t));
    if (!fill) { cells_free(c); return OR_E_INVALID; }
    memcpy(fill, c->start, (size_t)c->ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        int64_t lin = c->cxyz[3 * i] + (int64_t)c->g.n[0] * (c->cxyz[3 * i + 1] + (int64_t)c->g.n[1] * c->cxyz[3 * i + 2]);
        c->items[fill[lin]++] = i;
    }
    free(fill);
    return OR_OK;
}

/* Minimum-image difference along axis a. */
static double min_image(const grid_t *g, int a, double d)
{
    if (g->periodic[a]) {
        double half = 0.5 * g->L[a];
        if (d > half) d -= g->L[a];
        else if (d < -half) d += g->L[a];
    }
    return d;
}

/* Pair test: (dx*dx + dy*dy) + dz*dz < (2h)^2, evaluated in this order. */
static int within(const or_params *p, const grid_t *g, int64_t n, const double *x,
                  int64_t i, int64_t j, double r[3])
{
    for (int a = 0; a < 3; a++) r[a] = min_image(g, a, x[a * n + i] - x[a * n + j]);
    double xx = r[0] * r[0];
    double yy = r[1] * r[1];
    double zz = r[2] * r[2];
    double r2 = (xx + yy) + zz;
    double cut = (2.0 * p->h) * (2.0 * p->h);
    return r2 < cut;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

typedef struct { int64_t *ids; int64_t cap; } nbuf_t;

static int nbuf_push(nbuf_t *b, int64_t *cnt, int64_t v)
{
    if (*cnt == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 512;
        int64_t *q = (int64_t *)realloc(b->ids, (size_t)nc * sizeof(int64_t));
        if (!q) return 0;
        b->ids = q; b->cap = nc;
    }
    b->ids[(*cnt)++] = v;
    return 1;
}

/* Neighbour set N(i), ascending by id.  brute != 0 scans all particles instead of cells. */
static int64_t neighbours(const or_params *p, const cells_t *c, int64_t n, const double *x,
                          int64_t i, int brute, nbuf_t *b)
{
    int64_t cnt = 0;
    double r[3];
    if (brute) {
        for (int64_t j = 0; j < n; j++)
            if (j != i && within(p, &c->g, n, x, i, j, r)) nbuf_push(b, &cnt, j);
        return cnt;
    }
    const grid_t *g = &c->g;
    int cf = g->cf;
    for (int oz = -cf; oz <= cf; oz++) {
        int cz = c->cxyz[3 * i + 2] + oz;
        if (g->periodic[2]) cz = (cz + g->n[2]) % g->n[2];
        else if (cz < 0 || cz >= g->n[2]) continue;
        for (int oy = -cf; oy <= cf; oy++) {
            int cy = c->cxyz[3 * i + 1] + oy;
            if (g->periodic[1]) cy = (cy + g->n[1]) % g->n[1];
            else if (cy < 0 || cy >= g->n[1]) continue;
            for (int ox = -cf; ox <= cf; ox++) {
                int cx = c->cxyz[3 * i] + ox;
                if (g->periodic[0]) cx = (cx + g->n[0]) % g->n[0];
                else if (cx < 0 || cx >= g->n[0]) continue;
                int64_t lin = cx + (int64_t)g->n[0] * (cy + (int64_t)g->n[1] * cz);
                for (int64_t k = c->start[lin]; k < c->start[lin + 1]; k++) {
                    int64_t j = c->items[k];
                    if (j != i && within(p, g, n, x, i, j, r)) nbuf_push(b, &cnt, j);
                }
            }
        }
    }
    qsort(b->ids, (size_t)cnt, sizeof(int64_t), cmp_i64);
    return cnt;
}

/* ------------------------------------------------------------------------------------
 * Exported: cell list in Morton order, for bit-exact comparison.
 * key_by_id[i] = Morton3(cx, cy, cz) (bit 0 = x); perm = particle ids stably sorted by
 * (key, id); cell_start[r] = first sorted position of the r-th cell in Morton order
 * (ncell + 1 entries).  Returns the total cell count through *ncell_out.
 * ---------------------------------------------------------------------------------- */
typedef struct { uint32_t key; int64_t id; } kid_t;

static int cmp_kid(const void *a, const void *b)
{
    const kid_t *x = (const kid_t *)a, *y = (const kid_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

int or_grid_dims(const or_params *p, int32_t n_out[3], double edge_out[3])
{
    grid_t g;
    int st = make_grid(p, &g);
    if (st) return st;
    for (int a = 0; a < 3; a++) { n_out[a] = g.n[a]; edge_out[a] = g.edge[a]; }
    return OR_OK;
}

int or_cells(const or_params *p, int64_t n, const double *x, uint32_t *key_by_id,
             uint32_t *perm, uint32_t *cell_start, int64_t *ncell_out)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    int64_t ncell = c.ncell;
    kid_t *kv = (kid_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(kid_t));
    uint32_t *ckeys = (uint32_t *)malloc((size_t)ncell * sizeof(uint32_t));
    for (int64_t i = 0; i < n; i++) {
        uint32_t k = morton3((uint32_t)c.cxyz[3 * i], (uint32_t)c.cxyz[3 * i + 1], (uint32_t)c.cxyz[3 * i + 2]);
        key_by_id[i] = k;
        kv[i].key = k; kv[i].id = i;
    }
    qsort(kv, (size_t)n, sizeof(kid_t), cmp_kid);
    for (int64_t k = 0; k < n; k++) perm[k] = (uint32_t)kv[k].id;
    /* Morton codes of every cell, sorted: the r-th entry is the r-th cell in Morton order. */
    int64_t q = 0;
    for (int cz = 0; cz < c.g.n[2]; cz++)
        for (int cy = 0; cy < c.g.n[1]; cy++)
            for (int cx = 0; cx < c.g.n[0]; cx++)
                ckeys[q++] = morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
    qsort(ckeys, (size_t)ncell, sizeof(uint32_t), cmp_u32);
    int64_t pos = 0;
    for (int64_t r = 0; r < ncell; r++) {
        while (pos < n && kv[pos].key < ckeys[r]) pos++;
        cell_start[r] = (uint32_t)pos;
    }
    cell_start[ncell] = (uint32_t)n;
    if (ncell_out) *ncell_out = ncell;
    free(kv); free(ckeys);
    cells_free(&c);
    return OR_OK;
}

/* Neighbour CSR by id (cols ascending).  Returns the number of entries, or -1 when the
 * capacity is too small, or -(status+100) on a cell-build error. */
int64_t or_neighbors(const or_params *p, int64_t n, const double *x, int brute,
                     int64_t *row_ptr, int32_t *cols, int64_t cap)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return -(int64_t)(st + 100);
    nbuf_t b = {0, 0};
    int64_t tot = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t cnt = neighbours(p, &c, n, x, i, brute, &b);
        for (int64_t k = 0; k < cnt; k++) {
            if (tot < cap) cols[tot] = (int32_t)b.ids[k];
            tot++;
        }
        row_ptr[i + 1] = tot;
    }
    free(b.ids);
    cells_free(&c);
    return tot > cap ? -1 : tot;
}

/* ------------------------------------------------------------------------------------
 * Density (kernel summation) and Tait EOS.
 *   fluid and inner wall:  rho_i = m_i (W(0) + sum_{j in N(i)} W_ij)
 *   outer wall:            rho_i = rho0, P_i = 0 (initial values kept)
 *   all:                   S_i = sum over unlike neighbours of W_ij
 *   P_i = B ((rho_i/rho0)^7 - 1), B = rho0 c0^2 / gamma, gamma = 7.
 * `mask` (may be NULL) restricts the evaluation to particles with mask[i] != 0.
 * ---------------------------------------------------------------------------------- */
static double tait(const or_params *p, double rho)
{
    double B = p->rho0 * p->c0 * p->c0 / p->gamma;
    double r = rho / p->rho0;
    double r2 = r * r;
    double r7 = (r2 * r2) * (r2 * r);
    return B * (r7 - 1.0);
}

static int density_impl(const or_params *p, const cells_t *c, int64_t n, const double *x,
                        const uint8_t *species, const uint8_t *kind, int brute,
                        const uint8_t *mask, double *rho, double *P, double *S)
{
    double m[2];
    particle_masses(p, m);
    double W0 = or_W(p->kernel, p->h, 0.0);
    int err = 0;
#pragma omp parallel
    {
        nbuf_t b = {0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            if (mask && !mask[i]) continue;
            int64_t cnt = neighbours(p, c, n, x, i, brute, &b);
            double sw = 0.0, su = 0.0, r[3];
            for (int64_t k = 0; k < cnt; k++) {
                int64_t j = b.ids[k];
                within(p, &c->g, n, x, i, j, r);
                double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double w = or_W(p->kernel, p->h, rr);
                sw += w;
                if (species[j] != species[i]) su += w;
            }
            S[i] = su;
            if (kind[i] == OR_WALL_OUTER) {
                rho[i] = p->rho0;
                P[i] = 0.0;
            } else {
                rho[i] = m[species[i]] * (W0 + sw);
                P[i] = tait(p, rho[i]);
            }
            if (!isfinite(rho[i]) || !isfinite(P[i])) err = 1;
        }
        free(b.ids);
    }
    return err ? OR_E_NONFINITE : OR_OK;
}

int or_density(const or_params *p, int64_t n, const double *x, const uint8_t *species,
               const uint8_t *kind, int brute, double *rho, double *P, double *S)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    st = density_impl(p, &c, n, x, species, kind, brute, NULL, rho, P, S);
    cells_free(&c);
    return st;
}

/* ------------------------------------------------------------------------------------
 * Pressure filter (Algorithm 1: after the pressures, before the pressure-gradient
 * forces).  The paper names the filter and cites its source without giving its formula;
 * the reading here is a Shepard (normalised kernel) average of the pressure over the
 * particle itself and its neighbours, weighted by volume:
 *   P~_i = (V_i P_i W(0) + sum_{j in N(i), src} V_j P_j W_ij)
 *        / (V_i W(0)     + sum_{j in N(i), src} V_j W_ij),     V = m / rho,
 * for fluid and inner-wall particles (the ones whose pressure comes from the equation of
 * state); the sources are the same two kinds.  Outer-wall particles keep their fixed
 * pressure and are not sources: theirs is a boundary value, not a pressure state.
 * Self term first, then neighbours in ascending id.  `mask` (may be NULL) restricts the
 * targets; P is read for their neighbours.
 * ---------------------------------------------------------------------------------- */
static int filter_impl(const or_params *p, const cells_t *c, int64_t n, const double *x,
                       const uint8_t *species, const uint8_t *kind, const double *rho,
                       const double *P, int brute, const uint8_t *mask, double *Pout)
{
    double m[2];
    particle_masses(p, m);
    double W0 = or_W(p->kernel, p->h, 0.0);
    int err = 0;
#pragma omp parallel
    {
        nbuf_t b = {0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            if (mask && !mask[i]) continue;
            if (kind[i] == OR_WALL_OUTER) {
                Pout[i] = P[i];
                continue;
            }
            double Vi = m[species[i]] / rho[i];
            double num = Vi * P[i] * W0, den = Vi * W0;
            int64_t cnt = neighbours(p, c, n, x, i, brute, &b);
            for (int64_t k = 0; k < cnt; k++) {
                int64_t j = b.ids[k];
                if (kind[j] == OR_WALL_OUTER) continue;
                double r[3];
                within(p, &c->g, n, x, i, j, r);
                double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double w = or_W(p->kernel, p->h, rr);
                double Vj = m[species[j]] / rho[j];
                num += Vj * P[j] * w;
                den += Vj * w;
            }
            Pout[i] = num / den;
            if (!isfinite(Pout[i])) err = 1;
        }
        free(b.ids);
    }
    return err ? OR_E_NONFINITE : OR_OK;
}

int or_pressure_filter(const or_params *p, int64_t n, const double *x, const uint8_t *species,
                       const uint8_t *kind, const double *rho, const double *P, int brute,
                       double *Pout)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    st = filter_impl(p, &c, n, x, species, kind, rho, P, brute, NULL, Pout);
    cells_free(&c);
    return st;
}

/* ------------------------------------------------------------------------------------
 * Collision step (Algorithm 1; a correction that keeps particles from coming closer than
 * their volume allows; the paper cites the model without its formula).  Reading: every
 * pair of particles closer than r_c = coll_alpha dx that is approaching (v_ij . r_ij < 0,
 * r_ij = x_i - x_j, v_ij = v_i - v_j) exchanges an impulse along r_ij that leaves it
 * receding with the fraction coll_e (restitution) of its approach speed, as an isolated
 * two-body collision would:
 *   v_i <- v_i - (1 + e) mu_ij (v_ij . r_ij) r_ij / |r_ij|^2,
 *   mu_ij = m_j / (m_i + m_j) for a fluid partner, 1 for a wall partner (walls move as
 *   imposed and are not changed).
 * Every term uses the velocities before the step (all pairs at once), so the impulses of
 * fluid pairs cancel in sum m v, and being central they cancel in sum m x × v too.
 * Fluid particles only; pairs in ascending id; the distance test is the neighbour test's
 * ((dx^2 + dy^2) + dz^2 < r_c^2 with r_c = coll_alpha * dx, squared once).
 * ---------------------------------------------------------------------------------- */
static int collide_impl(const or_params *p, const cells_t *c, int64_t n, const double *x,
                        const double *v, const uint8_t *species, const uint8_t *kind,
                        int brute, double *vout)
{
    double m[2];
    particle_masses(p, m);
    const double rc = p->coll_alpha * p->dx;
    const double rc2 = rc * rc;
    const double e1 = 1.0 + p->coll_e;
    int err = 0;
#pragma omp parallel
    {
        nbuf_t b = {0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            for (int a = 0; a < 3; a++) vout[a * n + i] = v[a * n + i];
            if (kind[i] != OR_FLUID) continue;
            double dv[3] = {0, 0, 0};
            int64_t cnt = neighbours(p, c, n, x, i, brute, &b);
            for (int64_t k = 0; k < cnt; k++) {
                int64_t j = b.ids[k];
                double r[3];
                within(p, &c->g, n, x, i, j, r);
                double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
                if (!(r2 < rc2)) continue;
                double vn = 0.0;
                for (int a = 0; a < 3; a++) vn += (v[a * n + i] - v[a * n + j]) * r[a];
                if (!(vn < 0.0)) continue;
                double mu = kind[j] == OR_FLUID ? m[species[j]] / (m[species[i]] + m[species[j]]) : 1.0;
                double g = -e1 * mu * vn / r2;
                for (int a = 0; a < 3; a++) dv[a] += g * r[a];
            }
            for (int a = 0; a < 3; a++) {
                vout[a * n + i] = v[a * n + i] + dv[a];
                if (!isfinite(vout[a * n + i])) err = 1;
            }
        }
        free(b.ids);
    }
    return err ? OR_E_NONFINITE : OR_OK;
}

int or_collide(const or_params *p, int64_t n, const double *x, const double *v,
               const uint8_t *species, const uint8_t *kind, int brute, double *vout)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    st = collide_impl(p, &c, n, x, v, species, kind, brute, vout);
    cells_free(&c);
    return st;
}

/* ------------------------------------------------------------------------------------
 * Pair forces and torques on fluid particles (walls get zero: their motion is imposed).
 * For j in N(i), r = x_i - x_j (minimum image), F_ij = -W'(r)/r, V = m/rho,
 * Pi_h = diag(1,1,0), S = inviscid, N = viscous (walls count as N):
 *   pressure      f_P = m_i m_j (P_i/rho_i^2 + P_j/rho_j^2) F_ij r              (all)
 *   interfacial   f_T = g_T Pi_h r,  g_T = -sigma_T m_i m_j (1/rho_i^2 + 1/rho_j^2) F_ij
 *                                                                         (unlike pairs)
 *   viscous       f_V = -4 eta V_i V_j F_ij u_ij,  u_ij = v_ij - 1/2 (w_i + w_j) x r
 *                                                                           (N-N pairs)
 *   mutual fric.  f_M = -C_l W_ij (V_i/S_i + V_j/S_j) v_ij                (unlike pairs)
 *   torque        tau = -1/2 r x (f_V + f_M) - 1/2 r x f_T  (added to i; the same tau
 *                 goes to j from j's own sum, so orbital + spin momentum is conserved)
 * a_i = sum f / m_i, alpha_i = sum tau / I_i, I_i = kappa_I m_i dx^2.
 * ---------------------------------------------------------------------------------- */
static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static int forces_impl(const or_params *p, const cells_t *c, int64_t n, const double *x,
                       const double *v, const double *w, const uint8_t *species,
                       const uint8_t *kind, const double *rho, const double *P,
                       const double *S, int brute, const uint8_t *mask,
                       double *acc, double *alpha)
{
    double m[2];
    particle_masses(p, m);
    int err = 0;
#pragma omp parallel
    {
        nbuf_t b = {0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            if (mask && !mask[i]) continue;
            double F[3] = {0, 0, 0}, N[3] = {0, 0, 0};
            if (kind[i] != OR_FLUID) {
                for (int a = 0; a < 3; a++) { acc[a * n + i] = 0.0; alpha[a * n + i] = 0.0; }
                continue;
            }
            double mi = m[species[i]];
            double Vi = mi / rho[i];
            int64_t cnt = neighbours(p, c, n, x, i, brute, &b);
            for (int64_t k = 0; k < cnt; k++) {
                int64_t j = b.ids[k];
                double r[3];
                within(p, &c->g, n, x, i, j, r);
                double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double Fij = kernel_F(p->kernel, p->h, rr);
                double Wij = or_W(p->kernel, p->h, rr);
                double mj = m[species[j]];
                double Vj = mj / rho[j];
                double vij[3];
                for (int a = 0; a < 3; a++) vij[a] = v[a * n + i] - v[a * n + j];
                int unlike = species[i] != species[j];
                int both_visc = species[i] == 1 && species[j] == 1;
                double f[3], fnc[3] = {0, 0, 0};

                double gp = mi * mj * (P[i] / (rho[i] * rho[i]) + P[j] / (rho[j] * rho[j])) * Fij;
                for (int a = 0; a < 3; a++) f[a] = gp * r[a];

                if (unlike) {
                    double gT = -p->sigma_T * mi * mj * (1.0 / (rho[i] * rho[i]) + 1.0 / (rho[j] * rho[j])) * Fij;
                    f[0] += gT * r[0];
                    f[1] += gT * r[1];
                    /* -1/2 r x (gT (r_x, r_y, 0)) */
                    N[0] += -0.5 * gT * (-r[2] * r[1]);
                    N[1] += -0.5 * gT * (r[2] * r[0]);
                }
                if (both_visc) {
                    double ws[3], wr[3], u[3];
                    for (int a = 0; a < 3; a++) ws[a] = 0.5 * (w[a * n + i] + w[a * n + j]);
                    cross(ws, r, wr);
                    for (int a = 0; a < 3; a++) u[a] = vij[a] - wr[a];
                    double gv = -4.0 * p->eta * Vi * Vj * Fij;
                    for (int a = 0; a < 3; a++) { f[a] += gv * u[a]; fnc[a] += gv * u[a]; }
                }
                if (unlike) {
                    double wgt = 0.0;
                    if (S[i] > 0.0) wgt += Vi / S[i];
                    if (S[j] > 0.0) wgt += Vj / S[j];
                    double gm = -p->C_l * Wij * wgt;
                    for (int a = 0; a < 3; a++) { f[a] += gm * vij[a]; fnc[a] += gm * vij[a]; }
                }
                double t[3];
                cross(r, fnc, t);
                for (int a = 0; a < 3; a++) { F[a] += f[a]; N[a] += -0.5 * t[a]; }
            }
            double I = p->kappa_I * mi * p->dx * p->dx;
            for (int a = 0; a < 3; a++) {
                acc[a * n + i] = F[a] / mi;
                alpha[a * n + i] = N[a] / I;
                if (!isfinite(acc[a * n + i]) || !isfinite(alpha[a * n + i])) err = 1;
            }
        }
        free(b.ids);
    }
    return err ? OR_E_NONFINITE : OR_OK;
}

int or_forces(const or_params *p, int64_t n, const double *x, const double *v, const double *w,
              const uint8_t *species, const uint8_t *kind, const double *rho, const double *P,
              const double *S, int brute, double *acc, double *alpha)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    st = forces_impl(p, &c, n, x, v, w, species, kind, rho, P, S, brute, NULL, acc, alpha);
    cells_free(&c);
    return st;
}

/* Density, EOS, the pressure filter (when enabled) and forces at the current state: the
 * evaluation that precedes the first half-kick of velocity Verlet.  P returns the
 * pressure the forces used (filtered, when the filter is enabled). */
int or_evaluate(const or_params *p, int64_t n, const double *x, const double *v,
                const double *w, const uint8_t *species, const uint8_t *kind, int brute,
                double *rho, double *P, double *S, double *acc, double *alpha)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    st = density_impl(p, &c, n, x, species, kind, brute, NULL, rho, P, S);
    if (!st && p->pressure_filter) {
        double *Pf = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!Pf) { cells_free(&c); return OR_E_INVALID; }
        st = filter_impl(p, &c, n, x, species, kind, rho, P, brute, NULL, Pf);
        if (!st) memcpy(P, Pf, (size_t)n * sizeof(double));
        free(Pf);
    }
    if (!st) st = forces_impl(p, &c, n, x, v, w, species, kind, rho, P, S, brute, NULL, acc, alpha);
    cells_free(&c);
    return st;
}

/* Density/pressure/S and accelerations of a subset of particles, from the full state.
 * Densities are evaluated for the subset and all its neighbours (the forces need them),
 * and with the pressure filter for their neighbours too. */
int or_eval_subset(const or_params *p, int64_t n, const double *x, const double *v,
                   const double *w, const uint8_t *species, const uint8_t *kind,
                   int64_t n_sub, const int64_t *idx, double *rho_s, double *P_s,
                   double *S_s, double *acc_s, double *alpha_s)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    uint8_t *need = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *sub = (uint8_t *)calloc((size_t)n, 1);
    double *rho = (double *)malloc((size_t)n * sizeof(double));
    double *P = (double *)malloc((size_t)n * sizeof(double));
    double *S = (double *)malloc((size_t)n * sizeof(double));
    double *acc = (double *)malloc((size_t)3 * n * sizeof(double));
    double *alpha = (double *)malloc((size_t)3 * n * sizeof(double));
    nbuf_t b = {0, 0};
    for (int64_t k = 0; k < n_sub; k++) {
        int64_t i = idx[k];
        sub[i] = 1; need[i] = 1;
        int64_t cnt = neighbours(p, &c, n, x, i, 0, &b);
        for (int64_t q = 0; q < cnt; q++) need[b.ids[q]] = 1;
    }
    /* with the filter, the subset's neighbours need filtered pressures, which need the
     * densities of their own neighbours: one more ring */
    uint8_t *need2 = NULL;
    double *Pf = NULL;
    if (p->pressure_filter) {
        need2 = (uint8_t *)malloc((size_t)n);
        Pf = (double *)malloc((size_t)n * sizeof(double));
        memcpy(need2, need, (size_t)n);
        for (int64_t i = 0; i < n; i++) {
            if (!need[i]) continue;
            int64_t cnt = neighbours(p, &c, n, x, i, 0, &b);
            for (int64_t q = 0; q < cnt; q++) need2[b.ids[q]] = 1;
        }
    }
    free(b.ids);
    st = density_impl(p, &c, n, x, species, kind, 0, need2 ? need2 : need, rho, P, S);
    if (!st && p->pressure_filter) {
        st = filter_impl(p, &c, n, x, species, kind, rho, P, 0, need, Pf);
        for (int64_t i = 0; i < n && !st; i++)
            if (need[i]) P[i] = Pf[i];
    }
    free(need2); free(Pf);
    if (!st) st = forces_impl(p, &c, n, x, v, w, species, kind, rho, P, S, 0, sub, acc, alpha);
    for (int64_t k = 0; k < n_sub && !st; k++) {
        int64_t i = idx[k];
        rho_s[k] = rho[i]; P_s[k] = P[i]; S_s[k] = S[i];
        for (int a = 0; a < 3; a++) {
            acc_s[a * n_sub + k] = acc[a * n + i];
            alpha_s[a * n_sub + k] = alpha[a * n + i];
        }
    }
    free(need); free(sub); free(rho); free(P); free(S); free(acc); free(alpha);
    cells_free(&c);
    return st;
}

/* ------------------------------------------------------------------------------------
 * Velocity Verlet (kick-drift-kick).  On entry acc/alpha hold the accelerations at the
 * current positions (from or_evaluate or a previous step).  Per step:
 *   fluid: v += dt/2 a, w += dt/2 alpha, x += dt v, wrap periodic axes into [lo, hi);
 *   walls: (x, y) rotated by Omega dt about the z axis, v = Omega z x r, w = Omega z;
 *   the collision step on the half-step velocities at the new positions (when enabled);
 *   density, EOS, pressure filter (when enabled) and forces at the new positions with
 *   the half-step v and w;
 *   fluid: v += dt/2 a, w += dt/2 alpha.
 * ---------------------------------------------------------------------------------- */
int or_step(const or_params *p, int64_t n, double *x, double *v, double *w,
            const uint8_t *species, const uint8_t *kind, double *rho, double *P, double *S,
            double *acc, double *alpha, double dt, double Omega, int32_t nsteps, int brute)
{
    grid_t g;
    int st = make_grid(p, &g);
    if (st) return st;
    double cs = cos(Omega * dt), sn = sin(Omega * dt);
    double half = 0.5 * dt;
    for (int s = 0; s < nsteps; s++) {
        for (int64_t i = 0; i < n; i++) {
            if (kind[i] == OR_FLUID) {
                for (int a = 0; a < 3; a++) {
                    v[a * n + i] = v[a * n + i] + half * acc[a * n + i];
                    w[a * n + i] = w[a * n + i] + half * alpha[a * n + i];
                    double xn = x[a * n + i] + dt * v[a * n + i];
                    if (g.periodic[a]) {
                        if (xn >= p->hi[a]) xn -= g.L[a];
                        else if (xn < p->lo[a]) xn += g.L[a];
                    }
                    x[a * n + i] = xn;
                }
            } else {
                double x0 = x[i], y0 = x[n + i];
                double xr = cs * x0 - sn * y0;
                double yr = sn * x0 + cs * y0;
                x[i] = xr; x[n + i] = yr;
                v[i] = -Omega * yr; v[n + i] = Omega * xr; v[2 * n + i] = 0.0;
                w[i] = 0.0; w[n + i] = 0.0; w[2 * n + i] = Omega;
            }
        }
        if (p->coll_alpha > 0.0) {
            double *vn = (double *)malloc((size_t)3 * (n > 0 ? n : 1) * sizeof(double));
            if (!vn) return OR_E_INVALID;
            st = or_collide(p, n, x, v, species, kind, brute, vn);
            if (!st) memcpy(v, vn, (size_t)3 * n * sizeof(double));
            free(vn);
            if (st) return st;
        }
        st = or_evaluate(p, n, x, v, w, species, kind, brute, rho, P, S, acc, alpha);
        if (st) return st;
        for (int64_t i = 0; i < n; i++) {
            if (kind[i] != OR_FLUID) continue;
            for (int a = 0; a < 3; a++) {
                v[a * n + i] = v[a * n + i] + half * acc[a * n + i];
                w[a * n + i] = w[a * n + i] + half * alpha[a * n + i];
            }
        }
    }
    return OR_OK;
}

/* Global sums over fluid particles, FP64 with Neumaier compensation, ascending id:
 * out = [P_lin(3), J_tot(3) = sum m x × v + I w, E = sum m|v|^2/2 + I|w|^2/2]. */
static void nsum(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

int or_diagnostics(const or_params *p, int64_t n, const double *x, const double *v,
                   const double *w, const uint8_t *species, const uint8_t *kind, double out[7])
{
    double m[2];
    particle_masses(p, m);
    double s[7] = {0}, c[7] = {0};
    for (int64_t i = 0; i < n; i++) {
        if (kind[i] != OR_FLUID) continue;
        double mi = m[species[i]];
        double I = p->kappa_I * mi * p->dx * p->dx;
        double xi[3] = {x[i], x[n + i], x[2 * n + i]};
        double vi[3] = {v[i], v[n + i], v[2 * n + i]};
        double wi[3] = {w[i], w[n + i], w[2 * n + i]};
        double L[3];
        cross(xi, vi, L);
        for (int a = 0; a < 3; a++) {
            nsum(&s[a], &c[a], mi * vi[a]);
            nsum(&s[3 + a], &c[3 + a], mi * L[a] + I * wi[a]);
        }
        nsum(&s[6], &c[6], 0.5 * mi * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2])
                           + 0.5 * I * (wi[0] * wi[0] + wi[1] * wi[1] + wi[2] * wi[2]));
    }
    for (int k = 0; k < 7; k++) out[k] = s[k] + c[k];
    return OR_OK;
}

/* ------------------------------------------------------------------------------------
 * Rotational-force intensity (the diagnostic the paper renders and counts vortices on,
 * Sec. 3 with Figs. of the z = 0 section): the fifth term of Eq. 2, 2 eta_r curl(omega_0),
 * in the model's own discretisation.  The spin part of the viscous pair force is
 * 2 eta V_i V_j F_ij (w_i + w_j) x r_ij (viscous pairs), so per unit volume of particle i
 *     s_i = sum over viscous neighbours j of 2 eta V_j F_ij (w_i + w_j) x r_ij,
 * and the intensity is |s_i|.  It is evaluated at every fluid particle (the paper colours
 * both components by it), always from the viscous neighbours (walls included, as in the
 * pair forces); other particles get 0.  rho is the density of the same state; with a
 * mask (NULL: all particles) only the masked particles are evaluated, and rho is read only
 * for their viscous neighbours.
 * ---------------------------------------------------------------------------------- */
int or_rot_intensity(const or_params *p, int64_t n, const double *x, const double *w,
                     const uint8_t *species, const uint8_t *kind, const double *rho,
                     const uint8_t *mask, double *out)
{
    cells_t c;
    int st = cells_build(p, n, x, &c);
    if (st) return st;
    double m[2];
    particle_masses(p, m);
    int err = 0;
#pragma omp parallel
    {
        nbuf_t b = {0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            out[i] = 0.0;
            if (kind[i] != OR_FLUID || (mask && !mask[i])) continue;
            double s[3] = {0, 0, 0};
            int64_t cnt = neighbours(p, &c, n, x, i, 0, &b);
            for (int64_t k = 0; k < cnt; k++) {
                int64_t j = b.ids[k];
                if (species[j] != 1) continue;
                double r[3];
                within(p, &c.g, n, x, i, j, r);
                double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double Fij = kernel_F(p->kernel, p->h, rr);
                double Vj = m[species[j]] / rho[j];
                double ws[3], t[3];
                for (int a = 0; a < 3; a++) ws[a] = w[a * n + i] + w[a * n + j];
                cross(ws, r, t);
                double g = 2.0 * p->eta * Vj * Fij;
                for (int a = 0; a < 3; a++) s[a] += g * t[a];
            }
            out[i] = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
            if (!isfinite(out[i])) err = 1;
        }
        free(b.ids);
    }
    cells_free(&c);
    return err ? OR_E_NONFINITE : OR_OK;
}

int or_default_mass(const or_params *p, double m_out[2])
{
    particle_masses(p, m_out);
    return OR_OK;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
