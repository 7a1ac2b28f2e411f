/*
 * Whole-domain FP64 lattice Boltzmann solver: collide, then pull-stream
 * between two arrays (Sec. 2.1, eq. (1), and its split into a cell-local
 * collision and a streaming step).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Boundary readings (the paper's validation domain is fully periodic,
 * Sec. 4.1; the other boundaries are used by the single-turbine and wall
 * cases):
 *   y        periodic;
 *   z sides  periodic, halfway bounce-back (wall half a cell outside the
 *            first/last layer) or free-slip (specular reflection of c_z);
 *   x        periodic, or inflow/outflow: a source cell at x = -1 holds the
 *            equilibrium at density 1 and the inlet velocity of its (y,z);
 *            a source at x = nx copies the post-collision state of x = nx-1
 *            (zero gradient).
 *   A source outside in z is resolved first; the reflected or wrapped
 *   source is then checked in y and x.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_rotor_state; /* defined in orc_alm.c */

struct orc_grid {
    orc_params p;
    size_t n;
    double *f, *ft;      /* [27][n]: pre-collision / post-collision */
    double *fext;        /* [3][n]: body force + user force field */
    double *frot;        /* [3][n]: force spread by the rotors */
    double *uin;         /* [3][ny*nz] inlet velocity */
    double mlp[ORC_MLP_NBLOB];
    int has_mlp;
    long t;
    void *rotors[ORC_MAX_ROTORS];
    void *turbines[ORC_MAX_ROTORS];
};

/* accessors shared with orc_alm.c */
double *orc__pops(orc_grid *g) { return g->f; }
double *orc__frot(orc_grid *g) { return g->frot; }
double *orc__fext(orc_grid *g) { return g->fext; }
void **orc__rotors(orc_grid *g) { return g->rotors; }
const orc_params *orc__params(const orc_grid *g) { return &g->p; }
const double *orc__cpops(const orc_grid *g) { return g->f; }
const double *orc__cfrot(const orc_grid *g) { return g->frot; }
const double *orc__cfext(const orc_grid *g) { return g->fext; }
void *const *orc__crotors(const orc_grid *g) { return g->rotors; }
void **orc__turbines(orc_grid *g) { return g->turbines; }
void *const *orc__cturbines(const orc_grid *g) { return g->turbines; }
void orc__free_rotor(void *r);
void orc__free_turbine(void *t);

static inline size_t cell(const orc_grid *g, int x, int y, int z)
{
    return (size_t)x + (size_t)g->p.nx * ((size_t)y + (size_t)g->p.ny * (size_t)z);
}
static inline int wrap(int v, int n) { return (v % n + n) % n; }
static inline int cx_(int i) { return i % 3 - 1; }
static inline int cy_(int i) { return (i / 3) % 3 - 1; }
static inline int cz_(int i) { return i / 9 - 1; }

orc_grid *orc_create(const orc_params *p)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return NULL;
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    g->p = *p;
    g->n = (size_t)p->nx * p->ny * p->nz;
    g->f = (double *)calloc(ORC_Q * g->n, sizeof(double));
    g->ft = (double *)calloc(ORC_Q * g->n, sizeof(double));
    g->fext = (double *)calloc(3 * g->n, sizeof(double));
    g->frot = (double *)calloc(3 * g->n, sizeof(double));
    g->uin = (double *)calloc(3 * (size_t)p->ny * p->nz, sizeof(double));
    if (!g->f || !g->ft || !g->fext || !g->frot || !g->uin) {
        orc_destroy(g);
        return NULL;
    }
    for (int d = 0; d < 3; ++d) {
        for (size_t c = 0; c < g->n; ++c)
            g->fext[d * g->n + c] = p->body_force[d];
        for (size_t c = 0; c < (size_t)p->ny * p->nz; ++c)
            g->uin[d * (size_t)p->ny * p->nz + c] = p->u_in[d];
    }
    return g;
}

void orc_destroy(orc_grid *g)
{
    if (!g)
        return;
    for (int r = 0; r < ORC_MAX_ROTORS; ++r) {
        orc__free_rotor(g->rotors[r]);
        orc__free_turbine(g->turbines[r]);
    }
    free(g->f);
    free(g->ft);
    free(g->fext);
    free(g->frot);
    free(g->uin);
    free(g);
}

size_t orc_cells(const orc_grid *g) { return g->n; }
long orc_time(const orc_grid *g) { return g->t; }

/* f = f_eq(rho, u) in every cell; rho has n entries, u is [3][n] */
void orc_init_fields(orc_grid *g, const double *rho, const double *u)
{
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)g->n; ++c) {
        double uc[3] = {u[c], u[g->n + c], u[2 * g->n + c]};
        double fe[ORC_Q];
        orc_feq(rho[c], uc, fe);
        for (int i = 0; i < ORC_Q; ++i)
            g->f[i * g->n + c] = fe[i];
    }
    memset(g->frot, 0, 3 * g->n * sizeof(double));
    g->t = 0;
}

void orc_set_pops(orc_grid *g, const double *f)
{
    memcpy(g->f, f, ORC_Q * g->n * sizeof(double));
}
void orc_get_pops(const orc_grid *g, double *f)
{
    memcpy(f, g->f, ORC_Q * g->n * sizeof(double));
}

/* external force field [3][n]; replaces the uniform body force */
void orc_set_force_field(orc_grid *g, const double *F)
{
    memcpy(g->fext, F, 3 * g->n * sizeof(double));
}

void orc_set_inlet_plane(orc_grid *g, const double *u)
{
    memcpy(g->uin, u, 3 * (size_t)g->p.ny * g->p.nz * sizeof(double));
}

void orc_set_mlp(orc_grid *g, const double *blob)
{
    memcpy(g->mlp, blob, sizeof(g->mlp));
    g->has_mlp = 1;
}

void orc_get_force(const orc_grid *g, double *F)
{
    for (size_t k = 0; k < 3 * g->n; ++k)
        F[k] = g->fext[k] + g->frot[k];
}

/* Post-streaming population i at (x,y,z): the post-collision value at the
 * source x - c_i, with the boundary readings listed at the top of the file. */
static double pull(const orc_grid *g, int i, int x, int y, int z)
{
    const orc_params *p = &g->p;
    int ii = i;
    int sx = x - cx_(i), sy = y - cy_(i), sz = z - cz_(i);
    if (sz < 0 || sz >= p->nz) {
        int bc = sz < 0 ? p->bc_zlo : p->bc_zhi;
        if (bc == ORC_NOSLIP)
            return g->ft[(size_t)(26 - i) * g->n + cell(g, x, y, z)];
        if (bc == ORC_FREESLIP) {
            ii = i - 18 * cz_(i); /* reflect c_z */
            sz = z;
        } else {
            sz = wrap(sz, p->nz);
        }
    }
    sy = wrap(sy, p->ny);
    if (sx < 0 || sx >= p->nx) {
        if (p->bc_x == ORC_PERIODIC) {
            sx = wrap(sx, p->nx);
        } else if (sx < 0) {
            size_t pl = (size_t)p->ny * p->nz, q = (size_t)sy + (size_t)p->ny * sz;
            double uin[3] = {g->uin[q], g->uin[pl + q], g->uin[2 * pl + q]};
            double fe[ORC_Q];
            orc_feq(1.0, uin, fe);
            return fe[ii];
        } else {
            sx = p->nx - 1;
        }
    }
    return g->ft[(size_t)ii * g->n + cell(g, sx, sy, sz)];
}

static double cell_omega1(const orc_grid *g, const double kappa[ORC_Q])
{
    const orc_params *p = &g->p;
    if (p->closure == ORC_CLOSURE_SMAG)
        return orc_smagorinsky_omega(kappa, p->omega[0], p->cs);
    if (p->closure == ORC_CLOSURE_MLP && g->has_mlp)
        return orc_mlp_omega(g->mlp, kappa, p->omega[0], p->mlp_emulate_bf16);
    return p->omega[0];
}

/* collision of one cell, with the closure choosing omega_1 from the
 * pre-collision central moments */
static void collide_cell(const orc_grid *g, size_t c, double fout[ORC_Q])
{
    double f[ORC_Q], F[3];
    for (int i = 0; i < ORC_Q; ++i)
        f[i] = g->f[(size_t)i * g->n + c];
    for (int d = 0; d < 3; ++d)
        F[d] = g->fext[d * g->n + c] + g->frot[d * g->n + c];
    double omega[10];
    memcpy(omega, g->p.omega, sizeof(omega));
    if (g->p.closure != ORC_CLOSURE_NONE) {
        double rho = 0.0, j[3] = {0, 0, 0}, u[3], kappa[ORC_Q];
        for (int i = 0; i < ORC_Q; ++i) {
            rho += f[i];
            j[0] += cx_(i) * f[i];
            j[1] += cy_(i) * f[i];
            j[2] += cz_(i) * f[i];
        }
        for (int d = 0; d < 3; ++d)
            u[d] = (j[d] + 0.5 * F[d]) / rho;
        orc_central_moments(f, u, kappa);
        omega[0] = cell_omega1(g, kappa);
    }
    orc_collide(f, F, omega, fout);
}

void orc_step(orc_grid *g, int nsteps)
{
    const orc_params *p = &g->p;
    for (int s = 0; s < nsteps; ++s) {
        int any_rotor = 0;
        for (int r = 0; r < ORC_MAX_ROTORS; ++r)
            any_rotor |= g->rotors[r] != NULL || g->turbines[r] != NULL;
        if (any_rotor)
            orc_alm_step(g);

#pragma omp parallel for schedule(static)
        for (long c = 0; c < (long)g->n; ++c) {
            double fo[ORC_Q];
            collide_cell(g, (size_t)c, fo);
            for (int i = 0; i < ORC_Q; ++i)
                g->ft[(size_t)i * g->n + c] = fo[i];
        }

#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    size_t c = cell(g, x, y, z);
                    for (int i = 0; i < ORC_Q; ++i)
                        g->f[(size_t)i * g->n + c] = pull(g, i, x, y, z);
                }
        g->t += 1;
    }
}

/* rho = sum f and u = (sum c f + F/2)/rho with the force of the last step */
void orc_get_fields(const orc_grid *g, double *rho, double *u)
{
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)g->n; ++c) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < ORC_Q; ++i) {
            double fi = g->f[(size_t)i * g->n + c];
            r += fi;
            j[0] += cx_(i) * fi;
            j[1] += cy_(i) * fi;
            j[2] += cz_(i) * fi;
        }
        rho[c] = r;
        for (int d = 0; d < 3; ++d)
            u[d * g->n + c] =
                (j[d] + 0.5 * (g->fext[d * g->n + c] + g->frot[d * g->n + c])) / r;
    }
}

/* Neumaier-compensated running sum, so that the FP64 totals below are exact
 * to a few ulp whatever the cell count */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

/* mass = sum rho, momentum = sum rho u, kinetic energy = 1/2 sum rho |u|^2 */
void orc_global_moments(const orc_grid *g, double *mass, double mom[3], double *ke)
{
    double *rho = (double *)malloc(g->n * sizeof(double));
    double *u = (double *)malloc(3 * g->n * sizeof(double));
    orc_get_fields(g, rho, u);
    ksum m = {0, 0}, px = {0, 0}, py = {0, 0}, pz = {0, 0}, e = {0, 0};
    for (size_t c = 0; c < g->n; ++c) {
        double ux = u[c], uy = u[g->n + c], uz = u[2 * g->n + c];
        kadd(&m, rho[c]);
        kadd(&px, rho[c] * ux);
        kadd(&py, rho[c] * uy);
        kadd(&pz, rho[c] * uz);
        kadd(&e, 0.5 * rho[c] * (ux * ux + uy * uy + uz * uz));
    }
    *mass = m.s + m.c;
    mom[0] = px.s + px.c;
    mom[1] = py.s + py.c;
    mom[2] = pz.s + pz.c;
    *ke = e.s + e.c;
    free(rho);
    free(u);
}
