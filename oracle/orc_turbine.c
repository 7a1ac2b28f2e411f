/*
 * Turbine topology tree, FP64 (Sec. 3.3 of the waLBerla-wind paper: a
 * turbine is a parent-child hierarchy of components, each defined in its own
 * frame by its position and orientation relative to its parent; Alg. 1
 * updates a node's discretisation and then recurses into its children;
 * Alg. 2 gives the pose update of disks and lines, T_c = T_p T_r R and
 * p_c = p_p + T_p p_r). The force models of the components are those the
 * paper lists for its framework (actuator lines with or without tip loss,
 * disks) plus cross-flow drag for towers.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Readings (the paper gives the pose update, not the motion laws or the force
 * models of the non-blade components):
 *   R is the rotation about a fixed unit axis, given in the frame T_p T_r, by
 *   angle0 + omega t + amp sin(freq t + phase); the node origin may
 *   oscillate, p_r = pos + disp sin(freq t + phase);
 *   the points of a rigid line share the pose of the line's start and sit at
 *   s_k dir in its frame; disk points sit on rings of radius s_j in the
 *   node's y-z plane at angles 2 pi k / n_azimuth from +y towards +z, each
 *   standing for the area 2 pi s_j width_j / n_azimuth;
 *   a point moves with the time derivative of its position, written with
 *   angular velocities: w_c = w_p + T_p T_r (dtheta/dt) axis and
 *   v(o_c) = v(o_p) + w_p x (T_p p_r) + T_p dp_r/dt, v(x) = v(o_c) + w_c x (x - o_c);
 *   blade elements use the actuator-line formula of orc_blade_element in the
 *   plane of e_n = T_c normal and e_t = e_n x e_s (e_s = T_c dir), which for
 *   a rotor about +x is the axial / tangential pair of orc_alm.c;
 *   line drag is the cross-flow drag of a cylinder,
 *   1/2 rho C_D d l |W_p| W_p with W_p the part of W normal to the line;
 *   disk drag is the normal force 1/2 rho C A |W.n| (W.n) n; with C = C_T'
 *   (a thrust coefficient on the local normal velocity) it is the actuator
 *   disk;
 *   W = u - v is the sampled velocity relative to the moving point.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

typedef struct {
    double T[9];  /* world orientation, row-major */
    double o[3];  /* world origin */
    double w[3];  /* world angular velocity */
    double vo[3]; /* velocity of the origin */
} pose_t;

typedef struct {
    orc_turbine_desc d;
    orc_node *nodes; /* own copies; array pointers below */
    double *arrays;  /* all per-node arrays back to back */
    double *alpha, *cl, *cd;
    int npts;
    double *pts;        /* [npts][9]: x, v, F at the last step */
    double *node_loads; /* [n_nodes][7]: F, M about the node origin, P */
} turbine_t;

void **orc__turbines(orc_grid *g);
void **orc__rotors(orc_grid *g);
void orc__free_rotor(void *r);
void *const *orc__cturbines(const orc_grid *g);
double *orc__frot(orc_grid *g);
long orc_time(const orc_grid *g);

static void matmul(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

static void matvec(const double A[9], const double x[3], double y[3])
{
    for (int i = 0; i < 3; ++i)
        y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* rotation by th about the unit vector a (Rodrigues' formula) */
static void axis_rotation(const double a[3], double th, double R[9])
{
    double c = cos(th), s = sin(th), k = 1.0 - c;
    R[0] = c + k * a[0] * a[0];
    R[1] = k * a[0] * a[1] - s * a[2];
    R[2] = k * a[0] * a[2] + s * a[1];
    R[3] = k * a[1] * a[0] + s * a[2];
    R[4] = c + k * a[1] * a[1];
    R[5] = k * a[1] * a[2] - s * a[0];
    R[6] = k * a[2] * a[0] - s * a[1];
    R[7] = k * a[2] * a[1] + s * a[0];
    R[8] = c + k * a[2] * a[2];
}

/* Alg. 2 for one node, given its parent's pose */
static void update_node(const orc_node *nd, const pose_t *par, double t, pose_t *out)
{
    double ph = nd->freq * t + nd->phase;
    double th = nd->angle0 + nd->omega * t + nd->amp * sin(ph);
    double dth = nd->omega + nd->amp * nd->freq * cos(ph);
    double R[9], TrR[9], TpTr[9], pr[3], dpr[3], Tpr[3], Tdpr[3], wa[3], wx[3];
    axis_rotation(nd->axis, th, R);
    matmul(nd->rot, R, TrR);
    matmul(par->T, TrR, out->T); /* T_c = T_p T_r R */
    for (int a = 0; a < 3; ++a) {
        pr[a] = nd->pos[a] + nd->disp[a] * sin(ph);
        dpr[a] = nd->disp[a] * nd->freq * cos(ph);
    }
    matvec(par->T, pr, Tpr);
    for (int a = 0; a < 3; ++a)
        out->o[a] = par->o[a] + Tpr[a]; /* p_c = p_p + T_p p_r */
    matmul(par->T, nd->rot, TpTr);
    matvec(TpTr, nd->axis, wa);
    cross(par->w, Tpr, wx);
    matvec(par->T, dpr, Tdpr);
    for (int a = 0; a < 3; ++a) {
        out->w[a] = par->w[a] + dth * wa[a];
        out->vo[a] = par->vo[a] + wx[a] + Tdpr[a];
    }
}

/* Alg. 1: update this node's discretisation, then every child's */
static void update_tree(const orc_turbine_desc *d, int node, const pose_t *par, double t,
                        pose_t *poses)
{
    update_node(&d->nodes[node], par, t, &poses[node]);
    for (int c = node + 1; c < d->n_nodes; ++c)
        if (d->nodes[c].parent == node)
            update_tree(d, c, &poses[node], t, poses);
}

static void update_all(const orc_turbine_desc *d, double t, pose_t *poses)
{
    pose_t world;
    memset(&world, 0, sizeof(world));
    world.T[0] = world.T[4] = world.T[8] = 1.0;
    for (int r = 0; r < d->n_nodes; ++r)
        if (d->nodes[r].parent < 0)
            update_tree(d, r, &world, t, poses);
}

static int node_points(const orc_node *nd)
{
    if (nd->kind == ORC_NODE_LINE)
        return nd->n_points;
    if (nd->kind == ORC_NODE_DISK)
        return nd->n_points * nd->n_azimuth;
    return 0;
}

int orc_turbine_npoints(const orc_turbine_desc *d)
{
    int n = 0;
    for (int k = 0; k < d->n_nodes; ++k)
        n += node_points(&d->nodes[k]);
    return n;
}

/* offset of point m of a node in its own frame, and the area (disk) or
 * length (line) it stands for */
static void point_offset(const orc_node *nd, int m, double q[3], double *measure)
{
    if (nd->kind == ORC_NODE_LINE) {
        for (int a = 0; a < 3; ++a)
            q[a] = nd->s[m] * nd->dir[a];
        *measure = nd->width[m];
    } else {
        int j = m / nd->n_azimuth, k = m % nd->n_azimuth;
        double phi = 2.0 * PI * k / nd->n_azimuth;
        q[0] = 0.0;
        q[1] = nd->s[j] * cos(phi);
        q[2] = nd->s[j] * sin(phi);
        *measure = 2.0 * PI * nd->s[j] * nd->width[j] / nd->n_azimuth;
    }
}

static int check_desc(const orc_turbine_desc *d)
{
    if (d->n_nodes < 1 || d->n_nodes > ORC_MAX_NODES)
        return -1;
    int blade = 0;
    for (int k = 0; k < d->n_nodes; ++k) {
        const orc_node *nd = &d->nodes[k];
        if (nd->parent >= k || nd->parent < -1)
            return -1;
        if (nd->kind == ORC_NODE_LINE || nd->kind == ORC_NODE_DISK) {
            if (nd->n_points < 1 || !nd->s || !nd->width)
                return -1;
            if (nd->kind == ORC_NODE_DISK && nd->n_azimuth < 1)
                return -1;
        }
        if (nd->force == ORC_FORCE_BLADE) {
            if (nd->kind != ORC_NODE_LINE || !nd->chord || !nd->twist)
                return -1;
            blade = 1;
        }
        if (nd->force == ORC_FORCE_DRAG && nd->kind == ORC_NODE_LINE && !nd->chord)
            return -1;
    }
    if (blade && d->n_polar < 2)
        return -1;
    return orc_turbine_npoints(d) > 0 ? 0 : -1;
}

int orc_turbine_kinematics(const orc_turbine_desc *d, double t, double *x, double *v,
                           double *frames)
{
    if (check_desc(d))
        return -1;
    pose_t *poses = (pose_t *)calloc(d->n_nodes, sizeof(pose_t));
    update_all(d, t, poses);
    int p = 0;
    for (int k = 0; k < d->n_nodes; ++k) {
        const orc_node *nd = &d->nodes[k];
        const pose_t *P = &poses[k];
        if (frames) {
            memcpy(frames + 15 * k, P->T, 9 * sizeof(double));
            memcpy(frames + 15 * k + 9, P->o, 3 * sizeof(double));
            memcpy(frames + 15 * k + 12, P->w, 3 * sizeof(double));
        }
        for (int m = 0; m < node_points(nd); ++m, ++p) {
            double q[3], Tq[3], wq[3], meas;
            point_offset(nd, m, q, &meas);
            matvec(P->T, q, Tq);
            cross(P->w, Tq, wq);
            for (int a = 0; a < 3; ++a) {
                if (x)
                    x[3 * p + a] = P->o[a] + Tq[a];
                if (v)
                    v[3 * p + a] = P->vo[a] + wq[a];
            }
        }
    }
    free(poses);
    return 0;
}

void orc__free_turbine(void *vt)
{
    turbine_t *tb = (turbine_t *)vt;
    if (!tb)
        return;
    free(tb->nodes);
    free(tb->arrays);
    free(tb->alpha);
    free(tb->cl);
    free(tb->cd);
    free(tb->pts);
    free(tb->node_loads);
    free(tb);
}

static double *copy_into(double **dst, const double *src, int n)
{
    if (!src)
        return NULL;
    double *p = *dst;
    memcpy(p, src, n * sizeof(double));
    *dst += n;
    return p;
}

int orc_set_turbine(orc_grid *g, int id, const orc_turbine_desc *d)
{
    if (id < 0 || id >= ORC_MAX_ROTORS || check_desc(d))
        return -1;
    turbine_t *tb = (turbine_t *)calloc(1, sizeof(turbine_t));
    tb->d = *d;
    tb->nodes = (orc_node *)malloc(d->n_nodes * sizeof(orc_node));
    memcpy(tb->nodes, d->nodes, d->n_nodes * sizeof(orc_node));
    size_t total = 0;
    for (int k = 0; k < d->n_nodes; ++k)
        total += 4 * (size_t)d->nodes[k].n_points;
    tb->arrays = (double *)malloc((total > 0 ? total : 1) * sizeof(double));
    double *cur = tb->arrays;
    for (int k = 0; k < d->n_nodes; ++k) {
        orc_node *nd = &tb->nodes[k];
        int np = d->nodes[k].kind == ORC_NODE_FRAME ? 0 : d->nodes[k].n_points;
        nd->s = copy_into(&cur, d->nodes[k].s, np);
        nd->width = copy_into(&cur, d->nodes[k].width, np);
        nd->chord = copy_into(&cur, d->nodes[k].chord, np);
        nd->twist = copy_into(&cur, d->nodes[k].twist, np);
    }
    tb->d.nodes = tb->nodes;
    int npol = d->n_polar > 0 ? d->n_polar : 1;
    tb->alpha = (double *)calloc(npol, sizeof(double));
    tb->cl = (double *)calloc(npol, sizeof(double));
    tb->cd = (double *)calloc(npol, sizeof(double));
    if (d->n_polar > 0) {
        memcpy(tb->alpha, d->alpha_deg, d->n_polar * sizeof(double));
        memcpy(tb->cl, d->cl, d->n_polar * sizeof(double));
        memcpy(tb->cd, d->cd, d->n_polar * sizeof(double));
    }
    tb->d.alpha_deg = tb->alpha;
    tb->d.cl = tb->cl;
    tb->d.cd = tb->cd;
    tb->npts = orc_turbine_npoints(d);
    tb->pts = (double *)calloc(9 * (size_t)tb->npts, sizeof(double));
    tb->node_loads = (double *)calloc(7 * (size_t)d->n_nodes, sizeof(double));
    /* a slot holds a rotor or a turbine */
    void **rs = orc__rotors(g);
    orc__free_rotor(rs[id]);
    rs[id] = NULL;
    void **ts = orc__turbines(g);
    orc__free_turbine(ts[id]);
    ts[id] = tb;
    return 0;
}

/* Force on the structure at one point from the sampled density rho and the
 * relative velocity W (world frame). */
static void point_force(const orc_turbine_desc *d, const orc_node *nd, const pose_t *P, int m,
                        double rho, const double W[3], double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    double q[3], meas;
    point_offset(nd, m, q, &meas);
    if (nd->force == ORC_FORCE_BLADE) {
        double es[3], en[3], et[3];
        matvec(P->T, nd->dir, es);
        matvec(P->T, nd->normal, en);
        cross(en, es, et);
        double wn = dot(W, en), wt = -dot(W, et);
        double Fn, Ft;
        orc_blade_element(rho, wn, wt, nd->chord[m], nd->width[m], nd->twist[m], nd->pitch_deg,
                          d->n_polar, d->alpha_deg, d->cl, d->cd, &Fn, &Ft, NULL);
        if (nd->tip_loss) {
            double Fl = orc_tip_loss(d->n_blades, d->radius, nd->s[m], atan2(wn, wt));
            Fn *= Fl;
            Ft *= Fl;
        }
        for (int a = 0; a < 3; ++a)
            F[a] = Fn * en[a] + Ft * et[a];
    } else if (nd->force == ORC_FORCE_DRAG && nd->kind == ORC_NODE_LINE) {
        double es[3], Wp[3];
        matvec(P->T, nd->dir, es);
        double ws = dot(W, es);
        for (int a = 0; a < 3; ++a)
            Wp[a] = W[a] - ws * es[a];
        double c = 0.5 * rho * nd->coef * nd->chord[m] * meas * sqrt(dot(Wp, Wp));
        for (int a = 0; a < 3; ++a)
            F[a] = c * Wp[a];
    } else if (nd->force == ORC_FORCE_DRAG) {
        const double ex[3] = {1.0, 0.0, 0.0};
        double n[3];
        matvec(P->T, ex, n);
        double wn = dot(W, n);
        double c = 0.5 * rho * nd->coef * meas * fabs(wn) * wn;
        for (int a = 0; a < 3; ++a)
            F[a] = c * n[a];
    }
}

/* One step of every turbine: poses (Alg. 1, 2), sampling of the fields fld
 * [4][n] (rho, u) at each point, force models, spreading into the rotor
 * force field, loads. Called by orc_alm_step after the rotors. */
void orc__turbines_step(orc_grid *g, const double *fld)
{
    double t = (double)orc_time(g);
    double *frot = orc__frot(g);
    void **ts = orc__turbines(g);
    for (int id = 0; id < ORC_MAX_ROTORS; ++id) {
        turbine_t *tb = (turbine_t *)ts[id];
        if (!tb)
            continue;
        const orc_turbine_desc *d = &tb->d;
        pose_t *poses = (pose_t *)calloc(d->n_nodes, sizeof(pose_t));
        update_all(d, t, poses);
        memset(tb->node_loads, 0, 7 * sizeof(double) * d->n_nodes);
        int p = 0;
        for (int k = 0; k < d->n_nodes; ++k) {
            const orc_node *nd = &tb->nodes[k];
            const pose_t *P = &poses[k];
            double *L = tb->node_loads + 7 * k;
            for (int m = 0; m < node_points(nd); ++m, ++p) {
                double q[3], Tq[3], wq[3], x[3], v[3], meas;
                point_offset(nd, m, q, &meas);
                matvec(P->T, q, Tq);
                cross(P->w, Tq, wq);
                for (int a = 0; a < 3; ++a) {
                    x[a] = P->o[a] + Tq[a];
                    v[a] = P->vo[a] + wq[a];
                }
                double s[4];
                orc_trilinear(g, fld, 4, x, s);
                double W[3] = {s[1] - v[0], s[2] - v[1], s[3] - v[2]};
                double F[3], Mx[3];
                point_force(d, nd, P, m, s[0], W, F);
                cross(Tq, F, Mx); /* (x - o_c) x F */
                for (int a = 0; a < 3; ++a) {
                    tb->pts[9 * p + a] = x[a];
                    tb->pts[9 * p + 3 + a] = v[a];
                    tb->pts[9 * p + 6 + a] = F[a];
                    L[a] += F[a];
                    L[3 + a] += Mx[a];
                }
                L[6] += dot(F, v);
                if (nd->force == ORC_FORCE_NONE)
                    continue;
                if (d->kernel == ORC_KERNEL_ROMA3)
                    orc_spread_point_roma(g, x, F, frot);
                else
                    orc_spread_point(g, x, F, d->eps, frot);
            }
        }
        free(poses);
    }
}

void orc_turbine_loads(const orc_grid *g, int id, double *node_loads, double *pts)
{
    turbine_t *tb = (turbine_t *)orc__cturbines(g)[id];
    if (!tb)
        return;
    if (node_loads)
        memcpy(node_loads, tb->node_loads, 7 * sizeof(double) * tb->d.n_nodes);
    if (pts)
        memcpy(pts, tb->pts, 9 * sizeof(double) * tb->npts);
}
