/*
 * Actuator line model, FP64 (Sec. 2.2: nodes sample density and velocity by
 * trilinear interpolation, blade-element forces from tabulated lift and drag,
 * projection back onto the lattice by convolution with a regularisation
 * kernel; Sec. 3.3, Alg. 2 for the rotation-matrix pose update of the line
 * nodes, here in its closed form for a rigid rotor turning about +x).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Readings:
 *   cell centres sit at integer coordinates;
 *   each step runs: kinematics -> sample -> blade element -> spread, then
 *   the collision uses the new force; the sampled velocity includes half the
 *   force of the previous step;
 *   blade b of B is at azimuth theta0 + Omega t + 2 pi b / B, measured from
 *   +y towards +z (right-handed about +x);
 *   the relative velocity is the in-plane (axial, tangential) part of
 *   u - Omega r e_theta; the radial part is ignored;
 *   the regularisation kernel is the Gaussian
 *   exp(-|d|^2/eps^2) / (eps^3 pi^(3/2)) on the 13^3 nodes round(x_p) +- 6,
 *   renormalised to unit sum per node, so that the total force is conserved
 *   exactly (the property the paper values in its discrete kernel), or the
 *   paper's own choice, the 3-point discrete delta of Roma, Peskin and Berger
 *   (1999) as a product of 1-D factors in lattice units;
 *   the optional "Glauert type" tip-loss correction (Sec. 2.2, Sec. 4) is
 *   Prandtl's factor F = 2/pi arccos(exp(-B (R - r) / (2 r |sin phi|))),
 *   phi the inflow angle between the relative wind and the rotor plane,
 *   multiplying the whole blade-element force (lift and drag).
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SUPPORT 6
#define PI 3.14159265358979323846

typedef struct {
    orc_rotor_desc d; /* array pointers below point into own storage */
    double *r, *chord, *twist, *dl, *alpha, *cl, *cd;
    double *pos;   /* [npts][3] positions at the last step */
    double *force; /* [npts][3] force on the blade at the last step */
    double loads[3];
} rotor_t;

double *orc__pops(orc_grid *g);
double *orc__frot(orc_grid *g);
double *orc__fext(orc_grid *g);
void **orc__rotors(orc_grid *g);
void **orc__turbines(orc_grid *g);
void orc__free_turbine(void *t);
const orc_params *orc__params(const orc_grid *g);
const double *orc__cpops(const orc_grid *g);
const double *orc__cfrot(const orc_grid *g);
const double *orc__cfext(const orc_grid *g);
void *const *orc__crotors(const orc_grid *g);
long orc_time(const orc_grid *g);

static double *dupd(const double *src, int n)
{
    double *p = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(p, src, sizeof(double) * n);
    return p;
}

void orc__free_rotor(void *vr)
{
    rotor_t *r = (rotor_t *)vr;
    if (!r)
        return;
    free(r->r);
    free(r->chord);
    free(r->twist);
    free(r->dl);
    free(r->alpha);
    free(r->cl);
    free(r->cd);
    free(r->pos);
    free(r->force);
    free(r);
}

int orc_set_rotor(orc_grid *g, int id, const orc_rotor_desc *d)
{
    if (id < 0 || id >= ORC_MAX_ROTORS || d->n_blades < 1 || d->n_points < 1 ||
        d->n_polar < 2)
        return -1;
    void **rs = orc__rotors(g);
    orc__free_rotor(rs[id]);
    /* a slot holds a rotor or a turbine */
    void **ts = orc__turbines(g);
    orc__free_turbine(ts[id]);
    ts[id] = NULL;
    rotor_t *r = (rotor_t *)calloc(1, sizeof(rotor_t));
    r->d = *d;
    int np = d->n_points, npts = d->n_blades * d->n_points;
    r->r = dupd(d->r, np);
    r->chord = dupd(d->chord, np);
    r->twist = dupd(d->twist_deg, np);
    r->dl = dupd(d->dl, np);
    r->alpha = dupd(d->alpha_deg, d->n_polar);
    r->cl = dupd(d->cl, d->n_polar);
    r->cd = dupd(d->cd, d->n_polar);
    r->pos = (double *)calloc(3 * npts, sizeof(double));
    r->force = (double *)calloc(3 * npts, sizeof(double));
    rs[id] = r;
    return 0;
}

/* Trilinear interpolation of a cell-centred field [ncomp][n] at x; indices
 * wrap periodically (callers keep points inside non-periodic directions). */
void orc_trilinear(const orc_grid *g, const double *field, int ncomp,
                   const double x[3], double *out)
{
    const orc_params *p = orc__params(g);
    int dims[3] = {p->nx, p->ny, p->nz};
    int i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(x[a]);
        i0[a] = (int)fl;
        fr[a] = x[a] - fl;
    }
    size_t n = (size_t)p->nx * p->ny * p->nz;
    for (int k = 0; k < ncomp; ++k)
        out[k] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int ix = ((i0[0] + dx) % dims[0] + dims[0]) % dims[0];
                int iy = ((i0[1] + dy) % dims[1] + dims[1]) % dims[1];
                int iz = ((i0[2] + dz) % dims[2] + dims[2]) % dims[2];
                double w = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) *
                           (dz ? fr[2] : 1.0 - fr[2]);
                size_t c = (size_t)ix + (size_t)p->nx * ((size_t)iy + (size_t)p->ny * iz);
                for (int k = 0; k < ncomp; ++k)
                    out[k] += w * field[(size_t)k * n + c];
            }
}

/* Linear interpolation in a polar table on a uniform angle grid; angles
 * outside the table take the end values. */
static double polar(double a, int n, const double *alpha, const double *v)
{
    double da = (alpha[n - 1] - alpha[0]) / (n - 1);
    double s = (a - alpha[0]) / da;
    if (!(s > 0.0)) /* also NaN */
        return v[0];
    if (s >= n - 1)
        return v[n - 1];
    int k = (int)floor(s);
    if (k > n - 2)
        k = n - 2;
    double t = s - k;
    return v[k] * (1.0 - t) + v[k + 1] * t;
}

/* Blade-element force (Sec. 2.2, the force equation of the actuator line):
 * F = 1/2 rho |W|^2 c l (C_L e_L + C_D e_D), with e_D along the in-plane
 * relative wind W = W_n e_x - W_t e_theta and e_L normal to it in the
 * (e_x, e_theta) plane. The inflow angle is phi = atan2(W_n, W_t), the angle
 * of attack alpha = phi - twist - pitch (degrees, wrapped to [-180, 180)).
 * Returns the axial (Fn) and tangential (Ft, along e_theta) force on the
 * blade element. */
void orc_blade_element(double rho, double wn, double wt, double chord,
                       double dl, double twist_deg, double pitch_deg, int n_polar,
                       const double *alpha_deg, const double *cl,
                       const double *cd, double *Fn, double *Ft, double *alpha_out)
{
    double phi = atan2(wn, wt) * 180.0 / PI;
    double a = phi - twist_deg - pitch_deg;
    while (a >= 180.0)
        a -= 360.0;
    while (a < -180.0)
        a += 360.0;
    double CL = polar(a, n_polar, alpha_deg, cl);
    double CD = polar(a, n_polar, alpha_deg, cd);
    double w2 = wn * wn + wt * wt;
    double wm = sqrt(w2);
    double q = 0.5 * rho * w2 * chord * dl;
    /* e_L = (W_t e_x + W_n e_theta)/|W|, e_D = (W_n e_x - W_t e_theta)/|W| */
    double fn = 0.0, ft = 0.0;
    if (wm > 0.0) {
        fn = q * (CL * wt + CD * wn) / wm;
        ft = q * (CL * wn - CD * wt) / wm;
    }
    *Fn = fn;
    *Ft = ft;
    if (alpha_out)
        *alpha_out = a;
}

/* Add -Fp eta(x - xp), normalised over the support, to the force field F
 * [3][n] (the fluid receives the reaction of the force on the blade). */
void orc_spread_point(const orc_grid *g, const double xp[3], const double Fp[3],
                      double eps, double *F)
{
    const orc_params *p = orc__params(g);
    int dims[3] = {p->nx, p->ny, p->nz};
    size_t n = (size_t)p->nx * p->ny * p->nz;
    int c0[3];
    for (int a = 0; a < 3; ++a)
        c0[a] = (int)floor(xp[a] + 0.5);
    double norm = 1.0 / (eps * eps * eps * pow(PI, 1.5));
    double wsum = 0.0;
    for (int dz = -SUPPORT; dz <= SUPPORT; ++dz)
        for (int dy = -SUPPORT; dy <= SUPPORT; ++dy)
            for (int dx = -SUPPORT; dx <= SUPPORT; ++dx) {
                double ex = c0[0] + dx - xp[0], ey = c0[1] + dy - xp[1],
                       ez = c0[2] + dz - xp[2];
                wsum += norm * exp(-(ex * ex + ey * ey + ez * ez) / (eps * eps));
            }
    for (int dz = -SUPPORT; dz <= SUPPORT; ++dz)
        for (int dy = -SUPPORT; dy <= SUPPORT; ++dy)
            for (int dx = -SUPPORT; dx <= SUPPORT; ++dx) {
                double ex = c0[0] + dx - xp[0], ey = c0[1] + dy - xp[1],
                       ez = c0[2] + dz - xp[2];
                double w = norm * exp(-(ex * ex + ey * ey + ez * ez) / (eps * eps)) / wsum;
                int ix = ((c0[0] + dx) % dims[0] + dims[0]) % dims[0];
                int iy = ((c0[1] + dy) % dims[1] + dims[1]) % dims[1];
                int iz = ((c0[2] + dz) % dims[2] + dims[2]) % dims[2];
                size_t c = (size_t)ix + (size_t)p->nx * ((size_t)iy + (size_t)p->ny * iz);
                for (int k = 0; k < 3; ++k)
                    F[(size_t)k * n + c] -= w * Fp[k];
            }
}

/* Roma et al. 3-point discrete delta in one dimension (lattice units): the
 * unique function with support |r| < 3/2 whose shifts sum to one, have zero
 * first moment and sum of squares 1/2 at every r. */
double orc_roma_phi(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a < 1.5) {
        double b = 1.0 - a;
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * b * b)) / 6.0;
    }
    return 0.0;
}

/* Add -Fp delta(x - xp) with the 3-point delta (27 nodes, weights sum to 1
 * by construction, no renormalisation). */
void orc_spread_point_roma(const orc_grid *g, const double xp[3], const double Fp[3],
                           double *F)
{
    const orc_params *p = orc__params(g);
    int dims[3] = {p->nx, p->ny, p->nz};
    size_t n = (size_t)p->nx * p->ny * p->nz;
    int lo[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = (int)floor(xp[a]) - 1; /* nodes lo .. lo + 3 cover |x - xp| < 3/2 */
    for (int kz = 0; kz < 4; ++kz)
        for (int ky = 0; ky < 4; ++ky)
            for (int kx = 0; kx < 4; ++kx) {
                double w = orc_roma_phi(lo[0] + kx - xp[0]) * orc_roma_phi(lo[1] + ky - xp[1]) *
                           orc_roma_phi(lo[2] + kz - xp[2]);
                if (w == 0.0)
                    continue;
                int ix = ((lo[0] + kx) % dims[0] + dims[0]) % dims[0];
                int iy = ((lo[1] + ky) % dims[1] + dims[1]) % dims[1];
                int iz = ((lo[2] + kz) % dims[2] + dims[2]) % dims[2];
                size_t c = (size_t)ix + (size_t)p->nx * ((size_t)iy + (size_t)p->ny * iz);
                for (int k = 0; k < 3; ++k)
                    F[(size_t)k * n + c] -= w * Fp[k];
            }
}

/* Prandtl tip-loss factor for a blade element at radius r of a rotor of
 * radius R with B blades, inflow angle phi (radians); 0 at and beyond the
 * tip, 1 where the relative wind lies in the rotor plane. */
double orc_tip_loss(int n_blades, double radius, double r, double phi_rad)
{
    if (!(r < radius))
        return 0.0;
    double s = fabs(sin(phi_rad));
    if (s == 0.0)
        return 1.0;
    double f = 0.5 * n_blades * (radius - r) / (r * s);
    return 2.0 / PI * acos(exp(-f));
}

/* One ALM update: kinematics, sampling, blade elements, spreading, loads. */
void orc_alm_step(orc_grid *g)
{
    const orc_params *p = orc__params(g);
    size_t n = (size_t)p->nx * p->ny * p->nz;
    const double *f = orc__cpops(g);
    double *frot = orc__frot(g);
    const double *fext = orc__cfext(g);

    /* macroscopic fields of the current (pre-collision) state with half the
     * force of the previous step */
    double *fld = (double *)malloc(4 * n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < ORC_Q; ++i) {
            double fi = f[(size_t)i * n + c];
            r += fi;
            j[0] += (i % 3 - 1) * fi;
            j[1] += ((i / 3) % 3 - 1) * fi;
            j[2] += (i / 9 - 1) * fi;
        }
        fld[c] = r;
        for (int d = 0; d < 3; ++d)
            fld[(size_t)(d + 1) * n + c] =
                (j[d] + 0.5 * (fext[d * n + c] + frot[d * n + c])) / r;
    }
    memset(frot, 0, 3 * n * sizeof(double));

    double t = (double)orc_time(g);
    void **rs = orc__rotors(g);
    for (int id = 0; id < ORC_MAX_ROTORS; ++id) {
        rotor_t *R = (rotor_t *)rs[id];
        if (!R)
            continue;
        const orc_rotor_desc *d = &R->d;
        double T = 0.0, Q = 0.0;
        for (int b = 0; b < d->n_blades; ++b) {
            double th = d->azimuth0 + d->omega_rot * t + 2.0 * PI * b / d->n_blades;
            double er[3] = {0.0, cos(th), sin(th)};
            double et[3] = {0.0, -sin(th), cos(th)};
            for (int k = 0; k < d->n_points; ++k) {
                int pidx = b * d->n_points + k;
                double rr = R->r[k];
                double xp[3];
                for (int a = 0; a < 3; ++a)
                    xp[a] = d->hub[a] + rr * er[a];
                double s[4];
                orc_trilinear(g, fld, 4, xp, s);
                double rho = s[0];
                double u[3] = {s[1], s[2], s[3]};
                double ut = u[0] * et[0] + u[1] * et[1] + u[2] * et[2];
                double wn = u[0];                 /* axial: axis is +x */
                double wt = -(ut - d->omega_rot * rr);
                double Fn, Ft;
                orc_blade_element(rho, wn, wt, R->chord[k], R->dl[k], R->twist[k],
                                  d->pitch_deg, d->n_polar, R->alpha, R->cl, R->cd,
                                  &Fn, &Ft, NULL);
                if (d->tip_loss) {
                    double Fl = orc_tip_loss(d->n_blades, d->radius, rr, atan2(wn, wt));
                    Fn *= Fl;
                    Ft *= Fl;
                }
                double Fp[3];
                for (int a = 0; a < 3; ++a)
                    Fp[a] = Fn * (a == 0 ? 1.0 : 0.0) + Ft * et[a];
                for (int a = 0; a < 3; ++a) {
                    R->pos[3 * pidx + a] = xp[a];
                    R->force[3 * pidx + a] = Fp[a];
                }
                T += Fn;
                Q += rr * Ft;
                if (d->kernel == ORC_KERNEL_ROMA3)
                    orc_spread_point_roma(g, xp, Fp, frot);
                else
                    orc_spread_point(g, xp, Fp, d->eps, frot);
            }
        }
        R->loads[0] = T;
        R->loads[1] = Q;
        R->loads[2] = Q * d->omega_rot;
    }
    orc__turbines_step(g, fld);
    free(fld);
}

/* thrust, torque, power of the last step; optional per-point force [npts][3] */
void orc_rotor_loads(const orc_grid *g, int id, double out[3], double *pt_force)
{
    rotor_t *R = (rotor_t *)orc__crotors(g)[id];
    if (!R) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    memcpy(out, R->loads, 3 * sizeof(double));
    if (pt_force)
        memcpy(pt_force, R->force, 3 * sizeof(double) * R->d.n_blades * R->d.n_points);
}

void orc_rotor_points(const orc_grid *g, int id, double *pos)
{
    rotor_t *R = (rotor_t *)orc__crotors(g)[id];
    if (R)
        memcpy(pos, R->pos, 3 * sizeof(double) * R->d.n_blades * R->d.n_points);
}
