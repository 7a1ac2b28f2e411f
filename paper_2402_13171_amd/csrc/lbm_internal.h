// Internal declarations shared by the kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

constexpr int MAX_ROTORS = 8;
constexpr int SUPPORT = 6;          // Gaussian support half-width (nodes)
constexpr int MLP_NBLOB = 1326;

enum Bc { BC_PERIODIC = 0, BC_INOUT = 1, BC_NOSLIP = 2, BC_FREESLIP = 3 };

// Cells per block of the blocked population layout (lbm_access.h) for an
// element size in bytes: 32 for FP32 storage (a direction's run in a block is
// one 128-byte line), 64 for 16-bit storage.
__host__ __device__ constexpr int blk_width(int esize) { return esize == 4 ? 32 : 64; }

// 32-bit finaliser of MurmurHash3 (Appleby): the random words of the
// stochastic rounding of 16-bit stores (per-step seed on the host, per cell
// on the device) and SR_WEYL, the golden-ratio Weyl increment between them.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
constexpr uint32_t SR_WEYL = 0x9e3779b9u;

// Force box of one rotor: [3][bnx*bny*bnz] FP32, x fastest.
struct ForceBox {
    int x0, y0, z0, bnx, bny, bnz;
    const float *F;
};

// Closure network in device memory: bf16 matrices in the matrix-core
// operand order plus float32 vectors.
struct MlpDev {
    uint16_t W1[32 * 8];    // [out][in], inputs padded 6 -> 8 with zeros
    uint16_t W2[32 * 32];   // [out][in]
    uint16_t W2T[32 * 32];  // [in][out] (backward pass)
    alignas(16) float b1[32];  // 16-byte aligned: read as float4 by the kernels
    alignas(16) float b2[32];
    alignas(16) float w3[32];
    float b3;
    float mu[8], inv_sigma[8];
    float nu_scale;
};
constexpr int MLP_NPARAM = 1313;
// host: closure parameter blob (1326 floats) -> device layout
void mlp_pack(const float *blob, MlpDev *out);

// Everything a lattice kernel needs, passed by value.
struct Geo {
    void *pops;          // population store (storage type), blocked layout (lbm_access.h)
    int nbx;             // blocks per x row (nx rounded up to blk_width cells)
    int nx, ny, nz;
    int bc_x, bc_zlo, bc_zhi;
    const float *uin_rd; // inlet velocity plane [3][ny*nz] of the streaming a swapped-layout read completes
    const float *uin_wr; // inlet velocity plane of the current step (odd-step inlet writes)
    void *ghost;         // outflow ghost plane [9][ny*nz] (storage type)
    // z planes 0 / nz-1 that a fast-path launch leaves to the boundary-cell
    // kernel (0 outside that split)
    int skip_zlo, skip_zhi;
};


struct Physics {
    float omega, omega2, tau0, smag_c;  // smag_c = 18 sqrt(2) Cs^2
    float nu0;
    float omega_hi[8];                  // omega_3 .. omega_10 (general-rate collision)
    float bf[3];                        // uniform body force
    const float *ffield;                // dense force [3][n] or null
    int nbox;
    ForceBox box[MAX_ROTORS];
    const MlpDev *mlp;
    uint32_t sr_seed;                   // stochastic rounding of 16-bit stores: per-step seed
};

// Turbine topology tree (Sec. 3.3): one node as the point kernel reads it.
constexpr int TREE_MAX_NODES = 32;
constexpr int TREE_MAX_DEPTH = 16;
struct NodeDev {
    int parent, kind, force, tip_loss;
    double pos[3], rot[9], axis[3];
    double omega, angle0, amp, freq, phase;
    double disp[3], dir[3], normal[3];
    double coef, pitch_deg;
};
// One point of a turbine: its node, its offset q in the node frame and its
// element data (line: length; disk: area).
struct TreePointDev {
    int node;
    int pad_;
    double q[3];
    double s, measure, chord, twist;
};
constexpr int TREE_PT_OUT = 12;  // per point out: x[3], v[3], F[3], (x - o_node) x F [3]

// Per-rotor device description used by the actuator-line kernels. A slot
// holds either a rigid rotor about +x (closed-form kinematics) or a turbine
// tree (nodes != nullptr).
struct RotorDev {
    double hub[3];
    double omega_rot, azimuth0, pitch_deg, eps, radius;
    int n_blades, n_points, n_polar;
    int kernel;    // LBM_KERNEL_GAUSS / LBM_KERNEL_ROMA3
    int tip_loss;  // multiply blade-element forces by the Prandtl factor
    int half;      // spreading support: nodes nearest(x_p) +- half per axis
    int npts;      // points of the slot (rotor: n_blades * n_points)
    int n_nodes;   // turbine tree nodes (0 for a rotor)
    const NodeDev *nodes;       // turbine tree, or nullptr for a rotor
    const TreePointDev *tpts;   // [npts] turbine points
    double alpha0, dalpha;
    float alpha0_f, inv_dalpha_f;  // the polar grid for the FP32 lookup
    const double *r, *chord, *twist, *dl;     // n_points
    const double *blade_cs;                   // rotor: cos, sin of 2 pi b / n_blades per blade
    double cos_az, sin_az;                    // rotor: cos, sin of azimuth0 + omega t (set per launch)
    const float *cl, *cd;                     // n_polar
    // outputs
    float *pts;        // per point: x - c0 [3], -F [3] (reaction on the flow), c0 [3] (nearest node, as float)
    double *pt_force;  // per point: F[3] in FP64 (turbine: TREE_PT_OUT values)
    double *loads;     // T, Q, P, then per batch of 32 points: partial T, Q
    // spreading box
    ForceBox box;
    float *Fbox;
};

constexpr int PT_STRIDE = 10;

// Kernel launchers (defined in the .hip files).
// mode: SC_FAST (periodic box, 32-bit offsets), SC_GENERAL (boundary rules
// everywhere), SC_SPLIT (boundary rules, 32-bit offsets valid: the fast path
// with the x inflow/outflow rules applied per lane, on all cells in even
// steps and on all cells off the z walls in odd steps, whose wall planes take
// the general path)
enum { SC_FAST = 0, SC_GENERAL = 1, SC_SPLIT = 2 };
// stochastic != 0: 16-bit stores round stochastically (lbm_config.rounding)
int launch_stream_collide(int storage, int stochastic, int parity, int closure, int mode, bool force,
                          bool general_rates, const Geo &g, const Physics &ph, hipStream_t s);
int launch_init_tgv(int storage, const Geo &g, double u0, double k, double rho0, hipStream_t s);
int launch_pattern_probe(int storage, int parity, const Geo &g, hipStream_t s);
int launch_init_eq(int storage, const Geo &g, const double *rho, const double *u, size_t cell0,
                   size_t ncell, hipStream_t s);
int launch_fields(int storage, int parity, const Geo &g, const Physics &ph, double *rho, double *u,
                  size_t cell0, size_t ncell, hipStream_t s);
int launch_pops(int storage, int parity, const Geo &g, double *f, size_t cell0, size_t ncell,
                hipStream_t s);
int launch_sample_pops(int storage, int parity, const Geo &g, const size_t *cells, size_t m, double *f,
                       hipStream_t s);
int launch_filtered(int storage, int parity, const Geo &g, const Physics &ph, int w, double *out, size_t cc0,
                    size_t ncc, hipStream_t s);
int launch_inflow(float *uin, const float *mean, const float *box, int lt, int plane, double s_pos,
                  hipStream_t s);
int launch_moments(int storage, int parity, const Geo &g, const Physics &ph, double *partials,
                   int nblocks, double *out, hipStream_t s);
int launch_check(int storage, int parity, const Geo &g, const Physics &ph, double *partials,
                 int nblocks, double mass0, double tol, int *flag, hipStream_t s);
int launch_alm(int storage, int parity, const Geo &g, const Physics &ph, const RotorDev *h_rots, int nrot,
               long t, hipStream_t s);
constexpr int ALM_MAX_POINTS = 512;
constexpr int ALM_BATCH_PTS = 32;  // actuator points per workgroup of k_alm_points
constexpr int ALM_LOADS_LEN = 3 + 2 * (ALM_MAX_POINTS / ALM_BATCH_PTS);
constexpr int RED_NBLOCKS = 1024;   // reduction grid (fixed: deterministic sums)
constexpr int RED_NMOM = 6;

}  // namespace lbm
