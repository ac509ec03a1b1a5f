/*
 * FP64 CPU oracle: plain, slow, literal.  TEST INFRASTRUCTURE ONLY (see lks_oracle.h for who may
 * call it and for the passages of the paper each function follows).
 *
 * Every step is written in the order and notation of the paper's Algorithm 1 (Sec. 2.3) and the
 * reverse steps are the literal transposes of those forward steps, taken in reverse order:
 *   - the gradient operator is stored as explicit rows and its transpose scatters the same rows;
 *   - the boundary conditions are applied face by face, and their transpose walks the faces in
 *     the opposite order;
 *   - the transfer is a scatter from each design point, and its transpose is the gather back to
 *     the same design point.
 * Per-node loops that write only their own node carry an OpenMP pragma; every scatter and every
 * sum runs serially in a fixed order.
 */
#include "lks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------------
 * Velocity sets (Sec. 2.2: D2Q9 in 2D and D3Q15 in 3D; D3Q19 is the other standard 3D set of
 * the lattice Boltzmann literature the paper cites).  Weights w_i, velocities c_i.
 * ------------------------------------------------------------------------------------------ */
static const int C_D2Q9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W_D2Q9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int C_D3Q15[15][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1},
    {-1, -1, -1}};
static const double W_D3Q15[15] = {2.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                   1.0 / 9, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72,
                                   1.0 / 72, 1.0 / 72, 1.0 / 72};

static const int C_D3Q19[19][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1}, {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W_D3Q19[19] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36};

typedef struct {
    int q;
    const int (*c)[3];
    const double *w;
} lat_t;

static int get_lattice(const or_desc *d, lat_t *L) {
    if (d->lattice == OR_D2Q9 && d->dim == 2) {
        L->q = 9; L->c = C_D2Q9; L->w = W_D2Q9; return 0;
    }
    if (d->lattice == OR_D3Q15 && d->dim == 3) {
        L->q = 15; L->c = C_D3Q15; L->w = W_D3Q15; return 0;
    }
    if (d->lattice == OR_D3Q19 && d->dim == 3) {
        L->q = 19; L->c = C_D3Q19; L->w = W_D3Q19; return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------------------------
 * Grid helpers
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int dim;
    int n[3];
    int per[3];
    long nc;
} grid_t;

static void make_grid(const or_desc *d, grid_t *g) {
    g->dim = d->dim;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = d->n[a];
        g->per[a] = (a >= d->dim) ? 1 : (d->bc_kind[2 * a] == OR_BC_PERIODIC);
    }
    g->nc = (long)d->n[0] * d->n[1] * d->n[2];
}

static long node_index(const grid_t *g, const int x[3]) {
    return x[0] + (long)g->n[0] * (x[1] + (long)g->n[1] * x[2]);
}

static void node_coords(const grid_t *g, long idx, int x[3]) {
    x[0] = (int)(idx % g->n[0]);
    x[1] = (int)((idx / g->n[0]) % g->n[1]);
    x[2] = (int)(idx / ((long)g->n[0] * g->n[1]));
}

/* index of x + s*off, wrapping periodic axes; -1 if it leaves the domain */
static long neighbour(const grid_t *g, const int x[3], const int off[3], int s) {
    int y[3];
    for (int a = 0; a < 3; ++a) {
        int v = x[a] + s * off[a];
        if (v < 0 || v >= g->n[a]) {
            if (!g->per[a]) return -1;
            v %= g->n[a];
            if (v < 0) v += g->n[a];
        }
        y[a] = v;
    }
    return node_index(g, y);
}

/* a node lies on a face when it sits on the first or last plane of a non-periodic axis */
static int is_boundary(const grid_t *g, const int x[3]) {
    for (int a = 0; a < g->dim; ++a)
        if (!g->per[a] && (x[a] == 0 || x[a] == g->n[a] - 1)) return 1;
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Difference operator D_a used for du_alpha/dx_beta inside the equilibrium (Sec. 2.2 does not
 * say how the gradient is discretised; reading: second-order central differences, and at a
 * node on a non-periodic face the second-order one-sided difference pointing inward).
 * The operator is held as explicit rows so that its transpose is the same rows scattered.
 * ------------------------------------------------------------------------------------------ */
static int drow(const grid_t *g, const int x[3], int a, long cols[3], double coef[3]) {
    int e[3] = {0, 0, 0};
    e[a] = 1;
    int n = g->n[a];
    if (g->per[a] || (x[a] > 0 && x[a] < n - 1)) {
        cols[0] = neighbour(g, x, e, +1); coef[0] = 0.5;
        cols[1] = neighbour(g, x, e, -1); coef[1] = -0.5;
        return 2;
    }
    if (x[a] == 0) {
        cols[0] = node_index(g, x);       coef[0] = -1.5;
        cols[1] = neighbour(g, x, e, 1);  coef[1] = 2.0;
        cols[2] = neighbour(g, x, e, 2);  coef[2] = -0.5;
    } else {
        cols[0] = node_index(g, x);       coef[0] = 1.5;
        cols[1] = neighbour(g, x, e, -1); coef[1] = -2.0;
        cols[2] = neighbour(g, x, e, -2); coef[2] = 0.5;
    }
    return 3;
}

/* ------------------------------------------------------------------------------------------
 * Validation
 * ------------------------------------------------------------------------------------------ */
int or_validate(const or_desc *d) {
    lat_t L;
    if (!d) return -1;
    if (d->dim != 2 && d->dim != 3) return -2;
    if (get_lattice(d, &L)) return -3;
    for (int a = 0; a < 3; ++a) {
        if (a >= d->dim) {
            if (d->n[a] != 1 || d->nd[a] != 1) return -4;
            continue;
        }
        if (d->nd[a] < 1) return -5;
        int pm = d->bc_kind[2 * a] == OR_BC_PERIODIC, pp = d->bc_kind[2 * a + 1] == OR_BC_PERIODIC;
        if (pm != pp) return -6;
        if (d->n[a] < (pm ? 3 : 4)) return -7;
        for (int s = 0; s < 2; ++s) {
            int k = d->bc_kind[2 * a + s];
            if (k < OR_BC_PERIODIC || k > OR_BC_NOSLIP) return -8;
        }
    }
    if (!(d->nu > 0.0)) return -9;
    if (d->nsteps < 0 || !d->motion) return -10;
    if (d->obj_kind != OR_OBJ_NONE) {
        if (d->obj_kind < OR_OBJ_POWER || d->obj_kind > OR_OBJ_MASS) return -11;
        if (d->obj_n0 < 1 || d->obj_n1 > d->nsteps || d->obj_n0 > d->obj_n1) return -12;
    }
    if (d->weight != OR_W_COS4 && d->weight != OR_W_LIN) return -13;
    if (d->interp != OR_INTERP_PAPER && d->interp != OR_INTERP_FLUID_ONE) return -14;
    if (d->adj_form != OR_ADJ_EXACT && d->adj_form != OR_ADJ_PAPER) return -15;
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Brinkman interpolation (Sec. 2.3).  PAPER: gamma = 1 is solid,
 *   kappa_ref = kappa_max * q * gamma / ((1 - gamma) + q).
 * FLUID_ONE: the mirror form used when gamma = 1 is fluid,
 *   kappa_ref = kappa_max * q * (1 - gamma) / (q + gamma).
 * ------------------------------------------------------------------------------------------ */
int or_interp(const or_desc *d, const double *gamma, double *kref, double *kprime) {
    long nd = (long)d->nd[0] * d->nd[1] * d->nd[2];
    for (long i = 0; i < nd; ++i) {
        double g = gamma[i], km = d->kappa_max, q = d->q;
        if (d->interp == OR_INTERP_PAPER) {
            double den = (1.0 - g) + q;
            kref[i] = km * q * g / den;
            if (kprime) kprime[i] = km * q * (1.0 + q) / (den * den);
        } else {
            double den = q + g;
            kref[i] = km * q * (1.0 - g) / den;
            if (kprime) kprime[i] = -km * q * (1.0 + q) / (den * den);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Transfer weight (Sec. 2.3).  W = prod_alpha w(x_alpha - x_ref_alpha).
 * COS4: Peskin's four-point cosine kernel w(r) = (1 + cos(pi r / 2)) / 4 for |r| <= 2 (the
 *       printed "1 - cos" is read as a sign slip: it vanishes at r = 0 and jumps at |r| = 2).
 * LIN:  the hat w(r) = max(0, 1 - |r|).
 * ------------------------------------------------------------------------------------------ */
static double wfun(int kind, double r) {
    double a = fabs(r);
    if (kind == OR_W_LIN) return a < 1.0 ? 1.0 - a : 0.0;
    return a < 2.0 ? 0.25 * (1.0 + cos(M_PI * r / 2.0)) : 0.0;
}

static double wsupport(int kind) { return kind == OR_W_LIN ? 1.0 : 2.0; }

/* rigid-body map of a design point at step n (Eqs. rigid_body_position and rigid_body_velocity,
 * written for a general rotation R with angular velocity Omega: u_ref = Omega x (R (xi - xi_G))
 * + u_G, which reduces to the paper's 2D matrix form). */
static void rigid_map(const or_desc *d, int n, const double xi[3], double xr[3], double ur[3]) {
    const double *m = d->motion + 18L * n;
    const double *R = m, *Om = m + 9, *xG = m + 12, *uG = m + 15;
    double dxi[3], r[3];
    for (int a = 0; a < 3; ++a) dxi[a] = xi[a] - d->xi_G[a];
    for (int a = 0; a < 3; ++a) r[a] = R[3 * a + 0] * dxi[0] + R[3 * a + 1] * dxi[1] + R[3 * a + 2] * dxi[2];
    for (int a = 0; a < 3; ++a) xr[a] = r[a] + xG[a];
    ur[0] = Om[1] * r[2] - Om[2] * r[1] + uG[0];
    ur[1] = Om[2] * r[0] - Om[0] * r[2] + uG[1];
    ur[2] = Om[0] * r[1] - Om[1] * r[0] + uG[2];
    if (d->dim == 2) ur[2] = 0.0;
}

/* visit every (analysis node, weight) pair a design point spreads to; returns -1 if a pair
 * falls outside a non-periodic axis */
typedef void (*pair_fn)(void *ctx, long xi_idx, long x_idx, double W, const double ur[3]);

static int for_each_pair(const or_desc *d, int n, pair_fn fn, void *ctx) {
    grid_t g;
    make_grid(d, &g);
    double s = wsupport(d->weight);
    for (int k = 0; k < d->nd[2]; ++k)
        for (int j = 0; j < d->nd[1]; ++j)
            for (int i = 0; i < d->nd[0]; ++i) {
                long xi_idx = i + (long)d->nd[0] * (j + (long)d->nd[1] * k);
                double xi[3] = {i, j, k}, xr[3], ur[3];
                rigid_map(d, n, xi, xr, ur);
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                for (int a = 0; a < d->dim; ++a) {
                    lo[a] = (int)ceil(xr[a] - s);
                    hi[a] = (int)floor(xr[a] + s);
                }
                for (int z = lo[2]; z <= hi[2]; ++z)
                    for (int y = lo[1]; y <= hi[1]; ++y)
                        for (int x = lo[0]; x <= hi[0]; ++x) {
                            int p[3] = {x, y, z};
                            double W = 1.0;
                            for (int a = 0; a < d->dim; ++a) W *= wfun(d->weight, p[a] - xr[a]);
                            if (W == 0.0) continue;
                            int zero[3] = {0, 0, 0};
                            long idx = neighbour(&g, p, zero, 0);
                            if (idx < 0) return -1;
                            fn(ctx, xi_idx, idx, W, ur);
                        }
            }
    return 0;
}

typedef struct {
    const double *kref;
    double *kappa, *uS;
    long nc;
    int dim;
} spread_ctx;

static void spread_pair(void *vc, long xi_idx, long x_idx, double W, const double ur[3]) {
    spread_ctx *c = (spread_ctx *)vc;
    c->kappa[x_idx] += W * c->kref[xi_idx];
    for (int a = 0; a < c->dim; ++a) c->uS[a * c->nc + x_idx] += W * ur[a];
}

int or_transfer(const or_desc *d, int n, const double *kref, double *kappa, double *uS) {
    grid_t g;
    make_grid(d, &g);
    memset(kappa, 0, sizeof(double) * g.nc);
    memset(uS, 0, sizeof(double) * 3 * g.nc);
    spread_ctx c = {kref, kappa, uS, g.nc, d->dim};
    return for_each_pair(d, n, spread_pair, &c);
}

typedef struct {
    const double *kbar;
    double *G;
} gather_ctx;

static void gather_pair(void *vc, long xi_idx, long x_idx, double W, const double ur[3]) {
    (void)ur;
    gather_ctx *c = (gather_ctx *)vc;
    c->G[xi_idx] += W * c->kbar[x_idx];
}

int or_transfer_T(const or_desc *d, int n, const double *kbar, double *G) {
    gather_ctx c = {kbar, G};
    return for_each_pair(d, n, gather_pair, &c);
}

/* ------------------------------------------------------------------------------------------
 * Boundary conditions (Sec. 2.2, Eqs. bc_rho and bc_u: the macroscopic values are prescribed
 * directly).  Faces are applied in the order x-, x+, y-, y+, z-, z+, so a later face wins at
 * shared edges and corners.  On each face node p, with s = the next node inward:
 *   VELOCITY / NOSLIP: u = u_bar, rho = rho(s)
 *   ZERO_GRADIENT    : rho = rho_bar, u = u(s)   (outflow: zero normal gradient of u with the
 *                      pressure level held by Eq. bc_rho; copying rho too leaves the mean
 *                      pressure free and a channel then gains mass every step)
 *   PRESSURE         : rho = rho_bar, normal u = normal u(s), tangential u = u_bar tangential
 * ------------------------------------------------------------------------------------------ */
static void face_nodes_apply(const or_desc *d, const grid_t *g, int f, double *rho, double *u,
                             int transpose) {
    int a = f / 2, side = f % 2;
    int kind = d->bc_kind[f];
    for (long idx = 0; idx < g->nc; ++idx) {
        int p[3];
        node_coords(g, idx, p);
        if (p[a] != (side ? g->n[a] - 1 : 0)) continue;
        int s[3] = {p[0], p[1], p[2]};
        s[a] += side ? -1 : 1;
        long si = node_index(g, s);
        if (!transpose) {
            switch (kind) {
            case OR_BC_VELOCITY:
            case OR_BC_NOSLIP:
                rho[idx] = rho[si];
                for (int b = 0; b < g->dim; ++b) u[b * g->nc + idx] = d->bc_u[f][b];
                break;
            case OR_BC_ZERO_GRADIENT:
                rho[idx] = d->bc_rho[f];
                for (int b = 0; b < g->dim; ++b) u[b * g->nc + idx] = u[b * g->nc + si];
                break;
            case OR_BC_PRESSURE:
                rho[idx] = d->bc_rho[f];
                for (int b = 0; b < g->dim; ++b)
                    u[b * g->nc + idx] = (b == a) ? u[b * g->nc + si] : d->bc_u[f][b];
                break;
            }
        } else {
            /* transpose: a copied value sends its seed back to the source; every overwritten
             * value has zero derivative w.r.t. what it held before */
            switch (kind) {
            case OR_BC_VELOCITY:
            case OR_BC_NOSLIP:
                rho[si] += rho[idx];
                break;
            case OR_BC_ZERO_GRADIENT:
                for (int b = 0; b < g->dim; ++b) u[b * g->nc + si] += u[b * g->nc + idx];
                break;
            case OR_BC_PRESSURE:
                u[a * g->nc + si] += u[a * g->nc + idx];
                break;
            }
            rho[idx] = 0.0;
            for (int b = 0; b < g->dim; ++b) u[b * g->nc + idx] = 0.0;
        }
    }
}

int or_apply_bc(const or_desc *d, double *rho, double *u) {
    grid_t g;
    make_grid(d, &g);
    for (int f = 0; f < 2 * d->dim; ++f)
        if (d->bc_kind[f] != OR_BC_PERIODIC) face_nodes_apply(d, &g, f, rho, u, 0);
    return 0;
}

static void apply_bc_T(const or_desc *d, const grid_t *g, double *P, double *V) {
    for (int f = 2 * d->dim - 1; f >= 0; --f)
        if (d->bc_kind[f] != OR_BC_PERIODIC) face_nodes_apply(d, g, f, P, V, 1);
}

/* A from nu = (1/6 - 2A/9) (Sec. 2.2, lattice units) */
static double param_A(const or_desc *d) { return 4.5 * (1.0 / 6.0 - d->nu); }

/* ------------------------------------------------------------------------------------------
 * Forward step (Algorithm 1 body after the transfer)
 * ------------------------------------------------------------------------------------------ */
int or_step(const or_desc *d, const double *kappa, const double *uS, const double *rho,
            const double *u, double *rho_out, double *u_out) {
    grid_t g;
    lat_t L;
    make_grid(d, &g);
    if (get_lattice(d, &L)) return -1;
    const int D = d->dim;
    const long nc = g.nc;
    const double A = param_A(d);
    double *S = (double *)malloc(sizeof(double) * 9 * nc);
    double *E = (double *)malloc(sizeof(double) * L.q * nc);
    if (!S || !E) { free(S); free(E); return -2; }

    /* strain S_ab = du_a/dx_b + du_b/dx_a at every node */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nc; ++idx) {
        int x[3];
        node_coords(&g, idx, x);
        double du[3][3] = {{0}};
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                long cols[3]; double coef[3];
                int m = drow(&g, x, b, cols, coef);
                double v = 0.0;
                for (int t = 0; t < m; ++t) v += coef[t] * u[a * nc + cols[t]];
                du[a][b] = v;
            }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                S[(a * 3 + b) * nc + idx] = (a < D && b < D) ? du[a][b] + du[b][a] : 0.0;
    }

    /* equilibrium with the viscous A-term at every node */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nc; ++idx) {
        double uu = 0.0;
        for (int a = 0; a < D; ++a) uu += u[a * nc + idx] * u[a * nc + idx];
        for (int i = 0; i < L.q; ++i) {
            double cu = 0.0, cSc = 0.0;
            for (int a = 0; a < D; ++a) cu += L.c[i][a] * u[a * nc + idx];
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) cSc += L.c[i][a] * L.c[i][b] * S[(a * 3 + b) * nc + idx];
            E[i * nc + idx] = L.w[i] * (rho[idx] + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu + A * cSc);
        }
    }

    /* pull (Eqs. rho, u with tau = 1) and force update (Eqs. rho_ex, u_ex_2) at interior nodes;
     * face nodes are left NaN here and must all be overwritten by the boundary conditions */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nc; ++idx) {
        int x[3];
        node_coords(&g, idx, x);
        if (is_boundary(&g, x)) {
            rho_out[idx] = NAN;
            for (int a = 0; a < D; ++a) u_out[a * nc + idx] = NAN;
            continue;
        }
        double rs = 0.0, ms[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; ++i) {
            long y = neighbour(&g, x, L.c[i], -1);
            rs += E[i * nc + y];
            for (int a = 0; a < D; ++a) ms[a] += L.c[i][a] * E[i * nc + y];
        }
        double k = kappa[idx], ks = d->kappa_static ? d->kappa_static[idx] : 0.0;
        rho_out[idx] = rs;
        for (int a = 0; a < D; ++a)
            u_out[a * nc + idx] = (ms[a] + k * uS[a * nc + idx] + d->g[a]) / (1.0 + k + ks);
    }
    for (int a = D; a < 3; ++a) memset(u_out + a * nc, 0, sizeof(double) * nc);

    or_apply_bc(d, rho_out, u_out);
    free(S);
    free(E);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Reverse of one forward step: the exact transpose of or_step, steps in reverse order.
 * ------------------------------------------------------------------------------------------ */
static int step_T_core(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
                       const double *u_cur, const double *P, const double *V, const double *U3,
                       double *P_out, double *V_out, double *U3_out, double *kbar_out);

int or_step_T(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
              const double *u_cur, const double *P, const double *V, double *P_out,
              double *V_out, double *kbar_out) {
    return step_T_core(d, kappa, uS, u_prev, u_cur, P, V, NULL, P_out, V_out, NULL, kbar_out);
}

int or_step_T_paper(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
                    const double *u_cur, const double *P, const double *V, const double *U3,
                    double *P_out, double *V_out, double *U3_out, double *kbar_out) {
    return step_T_core(d, kappa, uS, u_prev, u_cur, P, V, U3, P_out, V_out, U3_out, kbar_out);
}

/* U3 == NULL: the exact transpose.  Otherwise the paper's form of Sec. 2.4: U3 carries 3 u~ of
 * the level being left (plus the objective's u-seed); only that part is divided by (1 + kappa)
 * and only that part forms the kappa seed, and U3_out receives 3 u~ of the new level. */
static int step_T_core(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
                       const double *u_cur, const double *P, const double *V, const double *U3,
                       double *P_out, double *V_out, double *U3_out, double *kbar_out) {
    grid_t g;
    lat_t L;
    make_grid(d, &g);
    if (get_lattice(d, &L)) return -1;
    const int D = d->dim;
    const long nc = g.nc;
    const double A = param_A(d);
    double *lp = (double *)malloc(sizeof(double) * nc);
    double *lv = (double *)malloc(sizeof(double) * 3 * nc);
    double *Ps = (double *)malloc(sizeof(double) * nc);
    double *Vs = (double *)malloc(sizeof(double) * 3 * nc);
    double *st = (double *)malloc(sizeof(double) * 9 * nc);
    if (!lp || !lv || !Ps || !Vs || !st) {
        free(lp); free(lv); free(Ps); free(Vs); free(st);
        return -2;
    }
    memcpy(lp, P, sizeof(double) * nc);
    memcpy(lv, V, sizeof(double) * 3 * nc);

    /* transpose of the boundary conditions, faces in reverse order */
    apply_bc_T(d, &g, lp, lv);

    /* transpose of the force update: V* = V / (1 + kappa + kappa_s), P* = P, and the kappa
     * seed -V*.(u - u_S); nothing flows through face nodes */
    for (long idx = 0; idx < nc; ++idx) {
        int x[3];
        node_coords(&g, idx, x);
        kbar_out[idx] = 0.0;
        if (is_boundary(&g, x)) {
            Ps[idx] = 0.0;
            for (int a = 0; a < 3; ++a) Vs[a * nc + idx] = 0.0;
            continue;
        }
        double k = kappa[idx], ks = d->kappa_static ? d->kappa_static[idx] : 0.0;
        Ps[idx] = lp[idx];
        double kb = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            if (a < D && !U3) {
                v = lv[a * nc + idx] / (1.0 + k + ks);
                kb -= v * (u_cur[a * nc + idx] - uS[a * nc + idx]);
            } else if (a < D) {
                /* Eq. au_ex: u~ (1 + kappa) = u~* - seed; the rest of the adjoint velocity passes */
                const double q = U3[a * nc + idx] / (1.0 + k + ks);
                v = q + (lv[a * nc + idx] - U3[a * nc + idx]);
                kb -= q * (u_cur[a * nc + idx] - uS[a * nc + idx]);
            }
            Vs[a * nc + idx] = v;
        }
        kbar_out[idx] = kb;
    }

    /* transpose of the pull: the seed of E_i(y) is P*(y + c_i) + c_i . V*(y + c_i); then the
     * w-weighted moments of the paper's adjoint (Eqs. arho, au, as) and the transpose of the
     * equilibrium (the structure of the paper's adjoint equilibrium) */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nc; ++idx) {
        int x[3];
        node_coords(&g, idx, x);
        double rt = 0.0, ut[3] = {0, 0, 0}, s[3][3] = {{0}};
        for (int i = 0; i < L.q; ++i) {
            long y = neighbour(&g, x, L.c[i], +1);
            double eb = 0.0;
            if (y >= 0) {
                eb = Ps[y];
                for (int a = 0; a < D; ++a) eb += L.c[i][a] * Vs[a * nc + y];
            }
            rt += L.w[i] * eb;
            for (int a = 0; a < D; ++a) {
                ut[a] += L.w[i] * L.c[i][a] * eb;
                for (int b = 0; b < D; ++b) s[a][b] += L.w[i] * L.c[i][a] * L.c[i][b] * eb;
            }
        }
        P_out[idx] = rt;
        for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            if (a < D) {
                v = 3.0 * ut[a] - 3.0 * rt * u_prev[a * nc + idx];
                for (int b = 0; b < D; ++b) v += 9.0 * s[a][b] * u_prev[b * nc + idx];
            }
            V_out[a * nc + idx] = v;
            if (U3_out) U3_out[a * nc + idx] = (a < D) ? 3.0 * ut[a] : 0.0;
            for (int b = 0; b < 3; ++b) st[(a * 3 + b) * nc + idx] = s[a][b];
        }
    }

    /* transpose of the strain: S_ab(y) = D_b u_a(y) + D_a u_b(y) with seed A * s~_ab(y) */
    for (long idx = 0; idx < nc; ++idx) {
        int x[3];
        node_coords(&g, idx, x);
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                double sb = A * st[(a * 3 + b) * nc + idx];
                long cols[3]; double coef[3];
                int m = drow(&g, x, b, cols, coef);
                for (int t = 0; t < m; ++t) V_out[a * nc + cols[t]] += coef[t] * sb;
                m = drow(&g, x, a, cols, coef);
                for (int t = 0; t < m; ++t) V_out[b * nc + cols[t]] += coef[t] * sb;
            }
    }

    free(lp); free(lv); free(Ps); free(Vs); free(st);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Objectives (Sec. 2.5 for J1 and J2; the body-force objectives use the reaction of the VPM
 * force F = -kappa (u - u_S) on the fluid, i.e. F_b = kappa (u - u_S) on the body):
 *   DRAG   : F_b . dir           POWER : F_b . u_S
 *   TORQUE : dir . ((x - centre) x F_b)
 *   J1     : -rho / 3 (pressure p = rho/3)     J2: -dir . u     MASS: rho
 * ------------------------------------------------------------------------------------------ */
static double obj_density(const or_desc *d, const grid_t *g, long idx, const double *kappa,
                          const double *uS, const double *rho, const double *u) {
    const long nc = g->nc;
    int x[3];
    node_coords(g, idx, x);
    double vel[3] = {0, 0, 0}, us[3] = {0, 0, 0};
    for (int a = 0; a < d->dim; ++a) {
        vel[a] = u[a * nc + idx];
        us[a] = uS[a * nc + idx];
    }
    double k = kappa[idx];
    double Fb[3] = {k * (vel[0] - us[0]), k * (vel[1] - us[1]), k * (vel[2] - us[2])};
    double r[3] = {x[0] - d->obj_centre[0], x[1] - d->obj_centre[1], x[2] - d->obj_centre[2]};
    const double *n = d->obj_dir;
    switch (d->obj_kind) {
    case OR_OBJ_DRAG: return Fb[0] * n[0] + Fb[1] * n[1] + Fb[2] * n[2];
    case OR_OBJ_POWER: return Fb[0] * us[0] + Fb[1] * us[1] + Fb[2] * us[2];
    case OR_OBJ_TORQUE: {
        double t0 = r[1] * Fb[2] - r[2] * Fb[1];
        double t1 = r[2] * Fb[0] - r[0] * Fb[2];
        double t2 = r[0] * Fb[1] - r[1] * Fb[0];
        return n[0] * t0 + n[1] * t1 + n[2] * t2;
    }
    case OR_OBJ_J1: return -rho[idx] / 3.0;
    case OR_OBJ_J2: return -(n[0] * vel[0] + n[1] * vel[1] + n[2] * vel[2]);
    case OR_OBJ_MASS: return rho[idx];
    }
    return 0.0;
}

double or_objective_step(const or_desc *d, const double *kappa, const double *uS,
                         const double *rho, const double *u) {
    grid_t g;
    make_grid(d, &g);
    double j = 0.0;
    for (long idx = 0; idx < g.nc; ++idx) {
        if (d->obj_mask && !d->obj_mask[idx]) continue;
        j += obj_density(d, &g, idx, kappa, uS, rho, u);
    }
    return j;
}

int or_objective_partials(const or_desc *d, const double *kappa, const double *uS,
                          const double *rho, const double *u, double *dP, double *dV,
                          double *dK) {
    grid_t g;
    make_grid(d, &g);
    const long nc = g.nc;
    (void)rho;
    for (long idx = 0; idx < nc; ++idx) {
        double p = 0.0, v[3] = {0, 0, 0}, kb = 0.0;
        int on = !(d->obj_mask && !d->obj_mask[idx]);
        if (on) {
            int x[3];
            node_coords(&g, idx, x);
            double vel[3] = {0, 0, 0}, us[3] = {0, 0, 0};
            for (int a = 0; a < d->dim; ++a) {
                vel[a] = u[a * nc + idx];
                us[a] = uS[a * nc + idx];
            }
            double k = kappa[idx];
            double r[3] = {x[0] - d->obj_centre[0], x[1] - d->obj_centre[1], x[2] - d->obj_centre[2]};
            const double *n = d->obj_dir;
            switch (d->obj_kind) {
            case OR_OBJ_DRAG:
                for (int a = 0; a < 3; ++a) v[a] = k * n[a];
                for (int a = 0; a < 3; ++a) kb += (vel[a] - us[a]) * n[a];
                break;
            case OR_OBJ_POWER:
                for (int a = 0; a < 3; ++a) v[a] = k * us[a];
                for (int a = 0; a < 3; ++a) kb += (vel[a] - us[a]) * us[a];
                break;
            case OR_OBJ_TORQUE: {
                /* dir . (r x F) = F . (dir x r) */
                double m[3] = {n[1] * r[2] - n[2] * r[1], n[2] * r[0] - n[0] * r[2],
                               n[0] * r[1] - n[1] * r[0]};
                for (int a = 0; a < 3; ++a) v[a] = k * m[a];
                for (int a = 0; a < 3; ++a) kb += (vel[a] - us[a]) * m[a];
                break;
            }
            case OR_OBJ_J1: p = -1.0 / 3.0; break;
            case OR_OBJ_J2:
                for (int a = 0; a < 3; ++a) v[a] = -n[a];
                break;
            case OR_OBJ_MASS: p = 1.0; break;
            }
        }
        if (dP) dP[idx] = p;
        if (dV)
            for (int a = 0; a < 3; ++a) dV[a * nc + idx] = (a < d->dim) ? v[a] : 0.0;
        if (dK) dK[idx] = kb;
    }
    return 0;
}

static double obj_scale(const or_desc *d, long nc) {
    double s = 1.0;
    if (d->obj_norm & OR_NORM_TIME) s /= (double)(d->obj_n1 - d->obj_n0 + 1);
    if (d->obj_norm & OR_NORM_MASK) {
        long cnt = 0;
        for (long i = 0; i < nc; ++i) cnt += d->obj_mask ? (d->obj_mask[i] != 0) : 1;
        s /= (double)(cnt > 0 ? cnt : 1);
    }
    return s;
}

/* ------------------------------------------------------------------------------------------
 * Full solve: Algorithm 1 then (if grad) Algorithm 2 as the exact reverse sweep
 * ------------------------------------------------------------------------------------------ */
int or_solve(const or_desc *d, const double *gamma, double *J, double *jn, double *grad,
             double *rho_final, double *u_final, double *rho_traj, double *u_traj) {
    int rc = or_validate(d);
    if (rc) return rc;
    grid_t g;
    make_grid(d, &g);
    const long nc = g.nc;
    const int N = d->nsteps;
    const long ndn = (long)d->nd[0] * d->nd[1] * d->nd[2];
    const int D = d->dim;

    double *kref = (double *)malloc(sizeof(double) * ndn);
    double *kpr = (double *)malloc(sizeof(double) * ndn);
    double *kappa = (double *)malloc(sizeof(double) * nc);
    double *uS = (double *)malloc(sizeof(double) * 3 * nc);
    double *rho_t = (double *)malloc(sizeof(double) * (size_t)(N + 1) * nc);
    double *u_t = (double *)malloc(sizeof(double) * (size_t)(N + 1) * 3 * nc);
    if (!kref || !kpr || !kappa || !uS || !rho_t || !u_t) { rc = -100; goto done; }
    or_interp(d, gamma, kref, kpr);

    /* initial state with the boundary conditions applied */
    for (long i = 0; i < nc; ++i) {
        rho_t[i] = d->rho_init ? d->rho_init[i] : d->rho0;
        for (int a = 0; a < 3; ++a)
            u_t[a * nc + i] = (a < D) ? (d->u_init ? d->u_init[a * nc + i] : d->u0[a]) : 0.0;
    }
    or_apply_bc(d, rho_t, u_t);

    const double sc = (d->obj_kind != OR_OBJ_NONE) ? obj_scale(d, nc) : 0.0;
    double Jacc = 0.0;
    if (jn) jn[0] = 0.0;
    for (int n = 1; n <= N; ++n) {
        double *r0 = rho_t + (size_t)(n - 1) * nc, *u0 = u_t + (size_t)(n - 1) * 3 * nc;
        double *r1 = rho_t + (size_t)n * nc, *u1 = u_t + (size_t)n * 3 * nc;
        if (or_transfer(d, n, kref, kappa, uS)) { rc = -101; goto done; }
        or_step(d, kappa, uS, r0, u0, r1, u1);
        double jv = 0.0;
        if (d->obj_kind != OR_OBJ_NONE && n >= d->obj_n0 && n <= d->obj_n1)
            jv = sc * or_objective_step(d, kappa, uS, r1, u1);
        if (jn) jn[n] = jv;
        Jacc += jv;
    }
    if (J) *J = Jacc;
    if (rho_final) memcpy(rho_final, rho_t + (size_t)N * nc, sizeof(double) * nc);
    if (u_final) memcpy(u_final, u_t + (size_t)N * 3 * nc, sizeof(double) * 3 * nc);
    if (rho_traj) memcpy(rho_traj, rho_t, sizeof(double) * (size_t)(N + 1) * nc);
    if (u_traj) memcpy(u_traj, u_t, sizeof(double) * (size_t)(N + 1) * 3 * nc);

    if (grad) {
        double *P = (double *)calloc(nc, sizeof(double));
        double *V = (double *)calloc(3 * nc, sizeof(double));
        double *P2 = (double *)malloc(sizeof(double) * nc);
        double *V2 = (double *)malloc(sizeof(double) * 3 * nc);
        double *kb = (double *)malloc(sizeof(double) * nc);
        double *dP = (double *)malloc(sizeof(double) * nc);
        double *dV = (double *)malloc(sizeof(double) * 3 * nc);
        double *dK = (double *)malloc(sizeof(double) * nc);
        double *G = (double *)calloc(ndn, sizeof(double));
        const int paper = d->adj_form == OR_ADJ_PAPER;
        double *U3 = paper ? (double *)calloc(3 * nc, sizeof(double)) : NULL;
        double *U32 = paper ? (double *)malloc(sizeof(double) * 3 * nc) : NULL;
        if (!P || !V || !P2 || !V2 || !kb || !dP || !dV || !dK || !G || (paper && (!U3 || !U32))) {
            rc = -102;
        } else {
            for (int n = N; n >= 1; --n) {
                double *r1 = rho_t + (size_t)n * nc;
                double *u0 = u_t + (size_t)(n - 1) * 3 * nc, *u1 = u_t + (size_t)n * 3 * nc;
                or_transfer(d, n, kref, kappa, uS);
                int inwin = d->obj_kind != OR_OBJ_NONE && n >= d->obj_n0 && n <= d->obj_n1;
                if (inwin) {
                    or_objective_partials(d, kappa, uS, r1, u1, dP, dV, dK);
                    for (long i = 0; i < nc; ++i) P[i] += sc * dP[i];
                    for (long i = 0; i < 3 * nc; ++i) V[i] += sc * dV[i];
                    if (paper)  /* Eq. au_ex: the u-seed joins u~ before the division */
                        for (long i = 0; i < 3 * nc; ++i) U3[i] += sc * dV[i];
                }
                if (paper) {
                    or_step_T_paper(d, kappa, uS, u0, u1, P, V, U3, P2, V2, U32, kb);
                    memcpy(U3, U32, sizeof(double) * 3 * nc);
                } else {
                    or_step_T(d, kappa, uS, u0, u1, P, V, P2, V2, kb);
                }
                if (inwin)
                    for (long i = 0; i < nc; ++i) kb[i] += sc * dK[i];
                or_transfer_T(d, n, kb, G);
                memcpy(P, P2, sizeof(double) * nc);
                memcpy(V, V2, sizeof(double) * 3 * nc);
            }
            for (long i = 0; i < ndn; ++i) grad[i] = kpr[i] * G[i];
        }
        free(P); free(V); free(P2); free(V2); free(kb); free(dP); free(dV); free(dK); free(G);
        free(U3); free(U32);
    }
done:
    free(kref); free(kpr); free(kappa); free(uS); free(rho_t); free(u_t);
    return rc;
}

/* threads the OpenMP loops of this library use (1 without OpenMP) */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
