/*
 * FP64 CPU oracle for the D3Q27 cumulant lattice-Boltzmann method with
 * actuator-line coupling (Sec. 2.1 and Sec. 2.2 of the waLBerla-wind paper,
 * arXiv 2402.13171).
 *
 * TEST INFRASTRUCTURE ONLY. This code is plain, slow and written to be read
 * against the paper; it shares no source with the HIP library and is only
 * ever loaded by the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark.
 *
 * Conventions
 *   velocity index   i = (cx+1) + 3(cy+1) + 9(cz+1), c in {-1,0,1}^3
 *   opposite         ibar = 26 - i
 *   moment index     m = a + 3b + 9c for the moment of order (a,b,c),
 *                    a,b,c in {0,1,2}
 *   population array f[i*n + cell], cell = x + nx*(y + ny*z) (x fastest)
 *   lattice units    dx = dt = 1, c_s^2 = 1/3
 */
#ifndef ORC_H
#define ORC_H
#include <stddef.h>

#define ORC_Q 27

/* boundary kinds (x: periodic or inflow/outflow; z sides: periodic,
 * halfway bounce-back, free-slip; y is always periodic) */
enum { ORC_PERIODIC = 0, ORC_INOUT = 1, ORC_NOSLIP = 2, ORC_FREESLIP = 3 };
enum { ORC_CLOSURE_NONE = 0, ORC_CLOSURE_SMAG = 1, ORC_CLOSURE_MLP = 2 };

/* ---- single-cell building blocks (orc_lattice.c) ---- */
void   orc_lattice(int c[ORC_Q][3], double w[ORC_Q]);
void   orc_feq(double rho, const double u[3], double f[ORC_Q]);
void   orc_central_moments_direct(const double f[ORC_Q], const double u[3],
                                  double kappa[ORC_Q]);
void   orc_central_moments(const double f[ORC_Q], const double u[3],
                           double kappa[ORC_Q]);
void   orc_central_to_pops(const double kappa[ORC_Q], const double u[3],
                           double f[ORC_Q]);
void   orc_cumulants(const double kappa[ORC_Q], double C[ORC_Q]);
void   orc_cumulants_inverse(const double C[ORC_Q], double kappa[ORC_Q]);
void   orc_relax(const double C[ORC_Q], const double omega[10],
                 double Cs[ORC_Q]);
void   orc_collide(const double f[ORC_Q], const double F[3],
                   const double omega[10], double fout[ORC_Q]);
double orc_smagorinsky_omega(const double kappa[ORC_Q], double omega0,
                             double cs);
void   orc_closure_features(const double kappa[ORC_Q], double omega0,
                            double feat[6]);

/* ---- learned closure network (orc_mlp.c) ---- */
#define ORC_MLP_NPARAM 1313
#define ORC_MLP_NBLOB  (ORC_MLP_NPARAM + 13)
double orc_mlp_nu_t(const double *blob, const double feat[6], int emulate_bf16);
double orc_mlp_omega(const double *blob, const double kappa[ORC_Q],
                     double omega0, int emulate_bf16);
double orc_bf16_round(double x);

/* ---- whole-domain solver (orc_solver.c) ---- */
typedef struct {
    int nx, ny, nz;
    double omega[10];      /* omega[0] = shear rate; omega[1..9] higher */
    int closure;           /* ORC_CLOSURE_* */
    double cs;             /* Smagorinsky constant */
    int bc_x;              /* ORC_PERIODIC or ORC_INOUT */
    int bc_zlo, bc_zhi;    /* ORC_PERIODIC, ORC_NOSLIP or ORC_FREESLIP */
    double u_in[3];        /* uniform inlet velocity */
    double body_force[3];  /* uniform body force */
    int mlp_emulate_bf16;  /* closure network arithmetic: 0 FP64, 1 BF16 emulation */
} orc_params;

typedef struct orc_grid orc_grid;

orc_grid *orc_create(const orc_params *p);
void   orc_destroy(orc_grid *g);
size_t orc_cells(const orc_grid *g);
void   orc_init_fields(orc_grid *g, const double *rho, const double *u);
void   orc_set_pops(orc_grid *g, const double *f);
void   orc_get_pops(const orc_grid *g, double *f);
void   orc_set_force_field(orc_grid *g, const double *F);
void   orc_set_inlet_plane(orc_grid *g, const double *u);
void   orc_set_mlp(orc_grid *g, const double *blob);
void   orc_step(orc_grid *g, int nsteps);
void   orc_get_fields(const orc_grid *g, double *rho, double *u);
void   orc_global_moments(const orc_grid *g, double *mass, double mom[3],
                          double *ke);
long   orc_time(const orc_grid *g);
void   orc_get_force(const orc_grid *g, double *F);

/* ---- actuator line (orc_alm.c) ---- */
#define ORC_MAX_ROTORS 8
typedef struct {
    double hub[3];
    double radius, omega_rot, azimuth0, eps, pitch_deg;
    int n_blades, n_points;
    const double *r, *chord, *twist_deg, *dl;  /* n_points each */
    int n_polar;
    const double *alpha_deg, *cl, *cd;          /* uniform alpha grid */
    int kernel;    /* ORC_KERNEL_GAUSS or ORC_KERNEL_ROMA3 */
    int tip_loss;  /* 1: blade-element force times the tip-loss factor */
} orc_rotor_desc;
#define ORC_KERNEL_GAUSS 0
#define ORC_KERNEL_ROMA3 1

int  orc_set_rotor(orc_grid *g, int id, const orc_rotor_desc *d);
void orc_rotor_loads(const orc_grid *g, int id, double out[3], double *pt_force);
void orc_rotor_points(const orc_grid *g, int id, double *pos);

/* single-point helpers exposed for the unit pins */
void orc_trilinear(const orc_grid *g, const double *field, int ncomp,
                   const double x[3], double *out);
void orc_blade_element(double rho, const double urel_axial,
                       const double urel_tan, double chord, double dl,
                       double twist_deg, double pitch_deg, int n_polar,
                       const double *alpha_deg, const double *cl,
                       const double *cd, double *Fn, double *Ft,
                       double *alpha_out);
void orc_spread_point(const orc_grid *g, const double xp[3],
                      const double Fp[3], double eps, double *F);
double orc_roma_phi(double r);
void orc_spread_point_roma(const orc_grid *g, const double xp[3],
                           const double Fp[3], double *F);
double orc_tip_loss(int n_blades, double radius, double r, double phi_rad);

/* ---- turbine topology tree (orc_turbine.c) ---- */
#define ORC_MAX_NODES 32
enum { ORC_NODE_FRAME = 0, ORC_NODE_LINE = 1, ORC_NODE_DISK = 2 };
enum { ORC_FORCE_NONE = 0, ORC_FORCE_BLADE = 1, ORC_FORCE_DRAG = 2 };
typedef struct {
    int parent;            /* parent index (< own index), -1 for a root */
    int kind;              /* ORC_NODE_* */
    int force;             /* ORC_FORCE_* */
    int n_points;          /* line points / disk rings */
    int n_azimuth;         /* disk points per ring */
    int tip_loss;
    double pos[3];         /* p_r, parent frame */
    double rot[9];         /* T_r, row-major */
    double axis[3];        /* rotation axis of R, frame T_p T_r */
    double omega, angle0;
    double amp, freq, phase;
    double disp[3];
    double dir[3];         /* line direction, node frame */
    double normal[3];      /* blade-element normal, node frame */
    double coef;           /* drag / thrust coefficient */
    double pitch_deg;
    const double *s, *width, *chord, *twist;
} orc_node;
typedef struct {
    int n_nodes;
    const orc_node *nodes;
    int kernel;
    double eps;
    int n_blades;
    double radius;
    int n_polar;
    const double *alpha_deg, *cl, *cd;
} orc_turbine_desc;

int  orc_set_turbine(orc_grid *g, int id, const orc_turbine_desc *d);
int  orc_turbine_npoints(const orc_turbine_desc *d);
/* positions x[npts][3] and velocities v[npts][3] of every point at time t,
 * and per node (nullable) frames[n_nodes][15]: T[9], origin[3], angular
 * velocity[3]; no grid involved */
int  orc_turbine_kinematics(const orc_turbine_desc *d, double t, double *x,
                            double *v, double *frames);
/* per node [n_nodes][7]: F[3], moment about the node origin[3], power;
 * per point [npts][9]: x, v, F (both nullable) */
void orc_turbine_loads(const orc_grid *g, int id, double *node_loads,
                       double *pts);
void orc__turbines_step(orc_grid *g, const double *fld);

/* internal: the ALM sub-steps of one time step, called by orc_step */
void orc_alm_step(orc_grid *g);

#endif
