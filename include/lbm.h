/*
 * lbm.h - C ABI of the MI355X D3Q27 cumulant lattice-Boltzmann solver with
 * actuator-line rotor coupling (after the waLBerla-wind method of
 * arXiv 2402.13171).
 *
 * What the library computes
 *   One time step is eq. (1) of Sec. 2.1: the cumulant collision (Sec. 2.1,
 *   Geier et al. 2015) with a Guo-type force, followed by streaming on the
 *   D3Q27 lattice. When rotors are set, each step first runs the actuator
 *   line of Sec. 2.2: rotor kinematics (Alg. 2 in closed form), trilinear
 *   sampling of density and velocity at the blade points, blade-element
 *   forces from tabulated lift/drag polars (the force equation of
 *   Sec. 2.2), and projection of the reaction force onto the lattice with a
 *   normalised Gaussian kernel. Optional eddy-viscosity closures set the
 *   shear rate per cell (Smagorinsky, or a learned per-cell network).
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3. Cell (x,y,z) sits at integer
 *     coordinates; x is the fastest index; cell = x + nx*(y + ny*z).
 *   - Velocity index i = (cx+1) + 3(cy+1) + 9(cz+1); opposite is 26 - i.
 *   - Host field arrays are FP64: rho[n], u[3][n] (ux block, uy block, uz
 *     block), F[3][n]; populations f[27][n].
 *   - Every function returns an lbm_status (0 = LBM_OK, < 0 = error). No
 *     function throws or aborts; after an error, lbm_last_error(ctx) gives a
 *     message. Arguments are validated before any device work.
 *   - Device memory for the populations and the small auxiliary area is
 *     owned by the caller (e.g. PyTorch) and handed over with lbm_attach; it
 *     must stay valid until lbm_destroy. Rotor, closure and staging buffers
 *     are owned by the context. Host arrays passed in are copied before the
 *     call returns; host output buffers are owned by the caller.
 *   - Work is enqueued on the stream given in lbm_config (NULL: the library
 *     creates one). Calls that return host data synchronise that stream.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* invalid argument or configuration */
    LBM_ENOMEM = -2,      /* a device or host allocation failed */
    LBM_EHIP = -3,        /* a HIP runtime call failed */
    LBM_EUNSTABLE = -4,   /* the mass / NaN check of lbm_step fired */
    LBM_ESTATE = -5       /* call out of order (e.g. before lbm_attach) */
} lbm_status;

typedef enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2 } lbm_storage;
typedef enum { LBM_CLOSURE_NONE = 0, LBM_CLOSURE_SMAG = 1, LBM_CLOSURE_MLP = 2 } lbm_closure;
typedef enum {
    LBM_BC_PERIODIC = 0,
    LBM_BC_INFLOW_OUTFLOW = 1, /* x only: equilibrium inlet at x=-1 (density 1,
                                  inlet velocity), zero-gradient outlet at x=nx */
    LBM_BC_NOSLIP = 2,         /* z sides: halfway bounce-back */
    LBM_BC_FREESLIP = 3        /* z sides: specular reflection */
} lbm_bc;

typedef struct {
    int nx, ny, nz;        /* cells; each >= 2, nx*ny*nz < 2^32 */
    double omega;          /* shear relaxation rate omega_1, 0 < omega < 2 */
    double omega_hi[9];    /* omega_2..omega_10 (bulk, 3rd..6th order); an
                              entry of 0 means the default 1.0. With all of
                              omega_3..omega_10 at 1 the collision takes a
                              shorter exact form (higher cumulants vanish) */
    int storage;           /* lbm_storage: populations are stored as the
                              deviation f_i - w_i in this type */
    int closure;           /* lbm_closure */
    double cs_smag;        /* Smagorinsky constant for LBM_CLOSURE_SMAG */
    int bc_x;              /* LBM_BC_PERIODIC or LBM_BC_INFLOW_OUTFLOW */
    int bc_z_lo, bc_z_hi;  /* LBM_BC_PERIODIC (both), NOSLIP or FREESLIP */
    double u_in[3];        /* uniform inlet velocity (bc_x inflow/outflow) */
    double body_force[3];  /* uniform body force per cell */
    int check_every;       /* FP64 mass/NaN check period in steps; 0 = off */
    void *stream;          /* hipStream_t, or NULL */
    int general_path;      /* 0: the library picks the stream-collide path
                              (32-bit-offset fast path with per-lane
                              inflow/outflow rules where offsets fit); 1: the
                              64-bit general boundary path on every cell, for
                              validation. Results agree to rounding. */
    int rounding;          /* 16-bit storage: how the stepping kernels round
                              the stored deviations. LBM_ROUND_STOCHASTIC
                              (0, default): to one of the two neighbouring
                              representable values with probability by
                              distance (expected value exact), so that a
                              steady flow does not accumulate the same
                              rounding step after step; LBM_ROUND_NEAREST
                              (1): to nearest even. Initialisation rounds to
                              nearest either way. No effect on FP32. */
} lbm_config;
typedef enum { LBM_ROUND_STOCHASTIC = 0, LBM_ROUND_NEAREST = 1 } lbm_rounding;

/* Create a context (validates cfg; no device memory is touched yet). */
int lbm_create(const lbm_config *cfg, lbm_ctx **out);
int lbm_destroy(lbm_ctx *ctx);

/* Bytes of caller-owned device memory lbm_attach needs: the population
 * store (blocked layout: each x row cut into blocks of W cells, W = 32 for
 * FP32 storage and 64 for 16-bit storage, rows padded to whole blocks, a
 * block's 27 directions stored one after the other, W values of the storage
 * type each; nz * ny * ceil(nx / W) * 27 W values, rounded up to 256 bytes) and the auxiliary area (outflow ghost plane, inlet
 * plane, reduction partials and flags). */
int lbm_required_bytes(const lbm_ctx *ctx, size_t *pop_bytes, size_t *aux_bytes);

/* Hand over device buffers of at least the required sizes, 256-byte aligned. */
int lbm_attach(lbm_ctx *ctx, void *d_pops, void *d_aux);

/* Taylor-Green vortex u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz,
 * w = 0, density rho0, populations at equilibrium; resets time to 0. */
int lbm_init_tgv(lbm_ctx *ctx, double u0, double k, double rho0);

/* Equilibrium populations from host FP64 density rho[n] and velocity u[3][n];
 * resets time to 0. */
int lbm_init_fields(lbm_ctx *ctx, const double *rho, const double *u);

/* Actuator-line rotor: rigid blades turning about the +x axis through hub.
 * r, chord, twist_deg, dl: n_points values per blade (element centre radius,
 * chord, twist in degrees, element length). Polars: n_polar >= 2 values of
 * C_L and C_D on a uniform grid alpha_deg[] (ascending), interpolated
 * linearly, end values outside. Blade b sits at azimuth
 * azimuth0 + omega_rot * t + 2 pi b / n_blades, measured from +y towards +z.
 * kernel selects the regularisation of the spread force (Sec. 2.2):
 * LBM_KERNEL_GAUSS, the Gaussian of width eps (> 0) on 13 nodes per axis
 * around the nearest node, renormalised to unit sum; or LBM_KERNEL_ROMA3, the
 * 3-point discrete delta of Roma et al. (27 nodes, unit sum by construction;
 * eps ignored). tip_loss = 1 multiplies each blade-element force by the
 * Prandtl tip-loss factor 2/pi arccos(exp(-B (radius - r) / (2 r |sin phi|))),
 * phi the inflow angle (the paper's Glauert-type correction, Sec. 2.2, 4).
 * Zero-initialised trailing fields give the Gaussian without tip loss.
 * All arrays are copied. rotor_id in [0, 8). The rotor's spreading box must
 * lie inside the domain. */
enum { LBM_KERNEL_GAUSS = 0, LBM_KERNEL_ROMA3 = 1 };
typedef struct {
    double hub[3];
    double axis[3];        /* must be (1, 0, 0) */
    double radius, omega_rot, azimuth0, eps, pitch_deg;
    int n_blades, n_points;
    const double *r, *chord, *twist_deg, *dl;
    int n_polar;
    const double *alpha_deg, *cl, *cd;
    int kernel;            /* LBM_KERNEL_GAUSS or LBM_KERNEL_ROMA3 */
    int tip_loss;          /* 0 or 1 */
} lbm_rotor;
int lbm_set_rotor(lbm_ctx *ctx, int rotor_id, const lbm_rotor *rotor);

/* Time-dependent inlet for bc_x inflow/outflow: the inlet velocity of cell
 * (y,z) at step t is mean[q] + turbulence taken from a frozen periodic box
 * convected through the inlet (Taylor's hypothesis): with s = advect * t
 * (mod lt), the box slice at s, linearly interpolated between slices
 * floor(s) and floor(s)+1. q = y + ny*z. Host FP64 arrays mean[3][ny*nz]
 * and box[3][lt][ny*nz] (box may be NULL: steady mean inlet). Copied. */
int lbm_set_inflow(lbm_ctx *ctx, const double *mean, const double *box, int lt, double advect);

/* Enqueue n time steps. With check_every > 0, an FP64 check runs every
 * check_every steps and at the end: it fails if any cell has a NaN, rho <= 0
 * or |u| > 1, or, in a domain closed in x (periodic), if the total mass
 * drifts from its value at the first checked call by more than 1e-6 (FP32
 * storage; 1e-5 FP16, 1e-4 BF16) relative. The call then synchronises and
 * returns LBM_EUNSTABLE if a check failed. */
int lbm_step(lbm_ctx *ctx, int n);

/* Density and velocity at the current time, u = (sum c f + F/2)/rho with
 * the force of the last step, into host rho[n] and u[3][n]. Synchronises. */
int lbm_get_fields(lbm_ctx *ctx, double *rho, double *u);

/* Thrust (axial force on the blades), torque about the axis and power
 * (torque * omega_rot) of the last step; pt_force (nullable) receives the
 * force on each blade point, [n_blades*n_points][3]. Synchronises. */
int lbm_rotor_loads(lbm_ctx *ctx, int rotor_id, double out[3], double *pt_force);

/* ---- turbine topology tree (Sec. 3.3, Alg. 1 and Alg. 2) ----
 * A turbine is a tree of components (tower, nacelle, hub, blades, disks),
 * each placed and oriented relative to its parent. Nodes are given in an
 * order where every parent precedes its children. At step t, node c with
 * parent p gets the world orientation and origin
 *   T_c = T_p T_r R(t),   o_c = o_p + T_p (pos + disp sin(freq t + phase)),
 * T_p = identity and o_p = 0 for the root; R(t) is the rotation about the
 * unit vector axis (in the frame T_p T_r) by the angle
 *   angle0 + omega t + amp sin(freq t + phase)
 * (omega: constant rotor or yaw rate; amp/freq/phase and disp: a prescribed
 * oscillation such as a floating platform's pitch and surge). A point with
 * node-frame offset q sits at x = o_c + T_c q and moves with the velocity
 * that this motion implies (the sum over the node and its ancestors of each
 * rotation rate times axis, crossed with the lever arm, plus the rates of
 * the displacements). Discretisations (Alg. 2):
 *   LBM_NODE_FRAME  no points (a joint: hub, nacelle frame, platform);
 *   LBM_NODE_LINE   n_points points q_k = s[k] dir (a blade, a tower);
 *   LBM_NODE_DISK   n_points rings of n_azimuth points, ring j at radius
 *                   s[j] in the node's y-z plane, point k at angle
 *                   2 pi k / n_azimuth from +y towards +z; the disk normal
 *                   is the node's x axis; a point stands for the area
 *                   2 pi s[j] width[j] / n_azimuth.
 * Force models (force on the structure; the fluid receives its reaction,
 * W = u - v is the sampled velocity relative to the moving point):
 *   LBM_FORCE_BLADE (lines only) blade element as in lbm_set_rotor, in the
 *     plane of e_n = T_c normal and e_t = e_n x e_s, e_s = T_c dir:
 *     W_n = W.e_n, W_t = -W.e_t, angle of attack
 *     atan2(W_n, W_t) - twist[k] - pitch_deg, force
 *     1/2 rho (W_n^2 + W_t^2) chord[k] width[k] (C_L e_L + C_D e_D) in that
 *     plane; tip_loss = 1 applies the Prandtl factor with the turbine's
 *     n_blades and radius at r = s[k];
 *   LBM_FORCE_DRAG on a line: cross-flow drag of a cylinder of diameter
 *     chord[k] and length width[k], 1/2 rho coef chord[k] width[k] |W_p| W_p
 *     with W_p = W - (W.e_s) e_s;
 *   LBM_FORCE_DRAG on a disk: normal force 1/2 rho coef A |W.n| (W.n) n,
 *     n the disk normal, A the point's area; with coef = C_T' (thrust
 *     coefficient on the local normal velocity) this is the actuator disk.
 *   LBM_FORCE_NONE: points that only sample (probes).
 * Spreading as for rotors (kernel, eps). At most 32 nodes, depth 16, 512
 * points per turbine. A turbine takes one of the 8 rotor slots (set_rotor
 * and set_turbine replace whatever the slot held; arguments are checked
 * before the slot is touched, and a device error while uploading leaves the
 * slot empty). The spreading box covers
 * every point's reach over all times (from the rotation and oscillation
 * amplitudes) and must lie inside the domain. All arrays are copied. */
enum { LBM_NODE_FRAME = 0, LBM_NODE_LINE = 1, LBM_NODE_DISK = 2 };
enum { LBM_FORCE_NONE = 0, LBM_FORCE_BLADE = 1, LBM_FORCE_DRAG = 2 };
typedef struct {
    int parent;            /* index of the parent node (smaller than own); -1: root */
    int kind;              /* LBM_NODE_* */
    int force;             /* LBM_FORCE_* */
    int n_points;          /* LINE: points; DISK: rings */
    int n_azimuth;         /* DISK: points per ring */
    int tip_loss;          /* BLADE: 0 or 1 */
    double pos[3];         /* origin relative to the parent's, parent frame */
    double rot[9];         /* T_r, row-major, orthonormal with determinant +1 */
    double axis[3];        /* unit rotation axis (need not be set if static) */
    double omega, angle0;  /* rad/step, rad */
    double amp, freq, phase;
    double disp[3];        /* oscillating origin displacement, parent frame */
    double dir[3];         /* LINE: unit direction, node frame */
    double normal[3];      /* BLADE: unit vector normal to dir, node frame */
    double coef;           /* DRAG: drag or thrust coefficient */
    double pitch_deg;      /* BLADE */
    const double *s;       /* [n_points] LINE distance along dir / DISK ring radius */
    const double *width;   /* [n_points] LINE element length / DISK ring width */
    const double *chord;   /* [n_points] BLADE chord / line DRAG diameter; NULL otherwise */
    const double *twist;   /* [n_points] BLADE twist, degrees; NULL otherwise */
} lbm_node;
typedef struct {
    int n_nodes;
    const lbm_node *nodes;
    int kernel;            /* LBM_KERNEL_GAUSS or LBM_KERNEL_ROMA3 */
    double eps;            /* Gaussian width */
    int n_blades;          /* tip-loss factor: blades and tip radius */
    double radius;
    int n_polar;           /* polars of every BLADE node (>= 2 if any) */
    const double *alpha_deg, *cl, *cd;
} lbm_turbine;
int lbm_set_turbine(lbm_ctx *ctx, int turbine_id, const lbm_turbine *turbine);

/* Loads of a turbine at the last step, per node (node_loads[n_nodes][7]:
 * total force on the node's points F[3], moment about the node's origin
 * sum (x - o_c) x F [3], power sum F.v) and, if pts is not NULL, per point
 * (pts[n_points_total][9]: position x[3], velocity v[3], force F[3]; points
 * in node order, rings before azimuth on disks). Synchronises. */
int lbm_turbine_loads(lbm_ctx *ctx, int turbine_id, double *node_loads, double *pts);
/* Spreading box of a turbine: the inclusive lattice-node range lo..hi per
 * axis that holds the spreading support of every point at every time (the
 * box lbm_set_turbine allocates and requires inside the domain). Checks the
 * turbine like lbm_set_turbine; needs no context and no device. */
int lbm_turbine_box(const lbm_turbine *turbine, int lo[3], int hi[3]);

/* Number of points of the turbine in slot turbine_id (size of pts above). */
int lbm_turbine_points(const lbm_ctx *ctx, int turbine_id, int *n_points_total);

/* FP64 totals over the domain: mass sum rho, momentum sum rho u, kinetic
 * energy 1/2 sum rho |u|^2. Synchronises. */
int lbm_global_moments(lbm_ctx *ctx, double *mass, double mom[3], double *kin_energy);

/* Populations f_i (not shifted) at the current time in natural layout, host
 * FP64 f[27][n]. Synchronises. */
int lbm_get_pops(lbm_ctx *ctx, double *f);

/* Populations f_i (not shifted) of m chosen cells (linear indices
 * cells[k] < n, host array) into host f[m][27]. For spot checks of large
 * lattices. Synchronises. */
int lbm_sample_pops(lbm_ctx *ctx, const size_t *cells, size_t m, double *f);

/* Box-filtered fields on the coarse grid of w^3-cell blocks (nx, ny, nz
 * divisible by w): out[10][nc], nc = n / w^3, holding the block means of
 * rho, ux, uy, uz, ux ux, uy uy, uz uz, ux uy, ux uz, uy uz (u as in
 * lbm_get_fields). Used to build training data for the learned closure.
 * Synchronises. */
int lbm_get_filtered(lbm_ctx *ctx, int w, double *out);

/* Number of completed steps. */
int lbm_time(const lbm_ctx *ctx, long *t);

/* Dense body-force field, host FP64 F[3][n], added to body_force in every
 * cell (e.g. Kolmogorov forcing); NULL removes it. */
int lbm_set_force_field(lbm_ctx *ctx, const double *F);

/* Closure network parameters (1326 floats: W1[32][6] b1[32] W2[32][32]
 * b2[32] w3[32] b3 mu[6] sigma[6] nu_scale); the matrix weights are used in
 * bfloat16 on the matrix cores, the rest in float32. */
int lbm_set_closure_weights(lbm_ctx *ctx, const float *w, size_t n);

/* ---- learned closure training (device-resident batches) ----
 * A trainer holds FP32 master parameters, Adam moments and the bfloat16
 * matrix-core copy of the closure network (same 1326-float layout as
 * lbm_set_closure_weights). Feature batches are device arrays d_feat[m][6]
 * (the six closure inputs per cell) with scaled targets d_target[m] =
 * nu_t / nu_scale; the loss is mean((softplus(z) - target)^2). */
typedef struct lbm_mlp lbm_mlp;
int lbm_mlp_create(void *stream, lbm_mlp **out);
int lbm_mlp_destroy(lbm_mlp *m);
/* Set all parameters (host blob) and reset the Adam state. */
int lbm_mlp_set_params(lbm_mlp *m, const float *blob, size_t n);
/* Current parameters into a host blob of 1326 floats. Synchronises. */
int lbm_mlp_get_params(lbm_mlp *m, float *blob, size_t n);
/* Eddy viscosity nu_t for m cells: device d_feat[m][6] -> device d_nu[m]. */
int lbm_mlp_forward(lbm_mlp *m, const float *d_feat, size_t count, float *d_nu);
/* Loss and gradient of one batch (kept on the device for lbm_mlp_adam_step;
 * copied to host grad[1313] when grad is not NULL, which synchronises). The
 * batch loss is added to an accumulator read by lbm_mlp_take_loss. */
int lbm_mlp_loss_grad(lbm_mlp *m, const float *d_feat, const float *d_target, size_t count, float *grad);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the same
 * loss and gradient as lbm_mlp_loss_grad, bit for bit, with the per-wave
 * partials in a static device array of the library instead of a buffer the
 * trainer allocates as batches grow. Calls no hipMalloc or hipFree. At most
 * 65536 samples per call (5.4 MB of scratch per device, held until the
 * process ends); larger batches return LBM_EINVAL before any device work, as
 * does a current device other than the one the trainer was created on.
 * Every call on one device shares that device's scratch: calls that overlap
 * in time on one device (two trainers on different streams) race and must be
 * ordered by the caller. */
int lbm_mlp_loss_grad_noalloc(lbm_mlp *m, const float *d_feat, const float *d_target, size_t count, float *grad);
/* One Adam update (Kingma and Ba 2015) with the last gradient. */
int lbm_mlp_adam_step(lbm_mlp *m, float lr, float beta1, float beta2, float eps);
/* Mean loss over the batches since the last call; resets. Synchronises. */
int lbm_mlp_take_loss(lbm_mlp *m, double *mean_loss);
const char *lbm_mlp_last_error(const lbm_mlp *m);

/* Checkpoint: raw population store, outflow ghost plane, time, layout
 * parity and the force boxes of the rotor and turbine slots (the spread
 * force of the last step, half of which the next step's sampled velocity
 * includes), behind a header that records the grid shape and storage type.
 * lbm_state_bytes gives the size. Restore into a context with the same
 * configuration and the same rotors and turbines set: a state of another
 * grid shape (even with the same cell count), another storage type or other
 * force boxes gives LBM_EINVAL, checked before any device work; so does a
 * state written by a library version with another population layout (the
 * header's first word names the layout). Synchronises. */
int lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
int lbm_get_state(lbm_ctx *ctx, void *host_buf, size_t bytes);
int lbm_set_state(lbm_ctx *ctx, const void *host_buf, size_t bytes);

/* Device-to-device copy of `bytes` (multiple of 16, 16-byte aligned device
 * pointers) with a plain streaming kernel (one 16-byte element per thread,
 * 256-thread groups), enqueued on `stream` (hipStream_t or NULL). It measures
 * achievable HBM bandwidth, the reference the paper takes from the STREAM
 * copy kernel (Sec. 4.3), and calibrates hardware traffic counters against a
 * kernel of known traffic. Null pointers, a size that is not a multiple of 16
 * or unaligned pointers give LBM_EINVAL before any device work; bytes = 0
 * launches nothing. The regions must not overlap. */
int lbm_copy_probe(const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Access-pattern probe (measurement, Sec. 4.3's roofline): enqueue on the
 * context's stream one pass of the stream-collide kernel's memory traffic
 * for the given AA parity (0: read and write the own cell's 27 slots; 1: the
 * neighbours' slots, periodic wrap) with the same tiling and addressing and
 * no collision. Moves 27 * 2 * sizeof(storage) bytes per cell. The
 * populations are left permuted: initialise again before stepping. Needs the
 * 32-bit offsets of the fast path (one z plane of the store, ny * ceil(nx/W)
 * blocks of 27 * W values, W as in lbm_required_bytes, below 4 GiB);
 * otherwise LBM_EINVAL. */
int lbm_pattern_probe(lbm_ctx *ctx, int parity);

const char *lbm_strerror(int code);
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
