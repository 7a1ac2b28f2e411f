// Actuator-line kernels (Sec. 2.2 of the waLBerla-wind paper): per step, one
// workgroup per 32 blade points computes their kinematics, stages the density and
// velocity of the 8 cells around every point in LDS, interpolates them
// trilinearly, evaluates the blade-element force and reduces thrust and
// torque per batch of points in FP64 (the host adds the batch partials when
// the loads are read); a second kernel spreads the reaction force onto the
// rotor's box of cells in gather form (no atomics, deterministic).
#include "../../include/lbm.h"
#include "lbm_access.h"

namespace lbm {

constexpr int ALM_BLOCK = 256;
constexpr int ALM_MAX_PTS = ALM_MAX_POINTS;  // points per slot (checked on the host)
constexpr double PI_D = 3.14159265358979323846;

// Lift and drag by linear interpolation in the polar tables on the uniform
// grid alpha0 + k dalpha (degrees), clamped to their ends (s <= 0 or NaN: the
// first entry, s >= n - 1: the last one, both exactly); FP32, like the
// tables. One index for both tables and no branch, so that the four loads
// are in flight together.
__device__ __forceinline__ void polar_pair(float a, const RotorDev &R, const float *cl, const float *cd, float &CL,
                                           float &CD) {
    const float last = (float)(R.n_polar - 1);
    float s = (a - R.alpha0_f) * R.inv_dalpha_f;
    s = s > 0.0f ? fminf(s, last) : 0.0f;
    const int k = min((int)floorf(s), R.n_polar - 2);
    const float t = fminf(s - (float)k, 1.0f);
    const float l0 = cl[k], l1 = cl[k + 1], d0 = cd[k], d1 = cd[k + 1];
    CL = l0 * (1.0f - t) + l1 * t;
    CD = d0 * (1.0f - t) + d1 * t;
}

__device__ __forceinline__ int wrap_any(int v, int n) { return ((v % n) + n) % n; }

// 1-D factor of the 3-point discrete delta of Roma, Peskin and Berger (1999),
// lattice units: support |r| < 3/2, shifts summing to one.
__device__ __forceinline__ float roma_phi(float r) {
    const float a = fabsf(r);
    if (a <= 0.5f) return (1.0f + sqrtf(1.0f - 3.0f * a * a)) * (1.0f / 3.0f);
    if (a < 1.5f) {
        const float b = 1.0f - a;
        return (5.0f - 3.0f * a - sqrtf(1.0f - 3.0f * b * b)) * (1.0f / 6.0f);
    }
    return 0.0f;
}

// Prandtl tip-loss factor 2/pi arccos(exp(-f)), f = B (R - r) / (2 r |sin phi|):
// zero at and beyond the tip, one for wind in the rotor plane.
__device__ __forceinline__ float tip_loss_factor(int B, float R, float r, float phi) {
    if (!(r < R)) return 0.0f;
    const float s = fabsf(sinf(phi));
    if (s == 0.0f) return 1.0f;
    return (float)(2.0 / PI_D) * acosf(expf(-0.5f * (float)B * (R - r) / (r * s)));
}

// ------------------------------------------------------------ turbine tree
// World pose of a node (Sec. 3.3, Alg. 2): composed from the root down,
// T_c = T_p T_r R(theta), o_c = o_p + T_p p_r, with theta = angle0 + omega t
// + amp sin(freq t + phase) about the node's axis and p_r = pos + disp
// sin(freq t + phase); alongside, the angular velocity w_c = w_p + T_p T_r
// (dtheta/dt) axis and the velocity of the origin v_c = v_p + w_p x (T_p p_r)
// + T_p dp_r/dt, so that a point x of the node moves with v_c + w_c x (x - o_c).
struct TreePose {
    double T[9], o[3], w[3], vo[3];
};

__device__ __forceinline__ void m3mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
__device__ __forceinline__ void m3vec(const double *A, const double *x, double *y) {
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}
__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static_assert(sizeof(NodeDev) % 8 == 0 && alignof(NodeDev) == 8, "node table copied as 8-byte words");

__device__ void tree_pose(const NodeDev *nodes, int node, double t, TreePose &P) {
    int chain[TREE_MAX_DEPTH];
    int d = 0;
    for (int k = node; k >= 0 && d < TREE_MAX_DEPTH; k = nodes[k].parent) chain[d++] = k;  // depth checked on the host
    for (int a = 0; a < 9; ++a) P.T[a] = (a % 4 == 0) ? 1.0 : 0.0;
    for (int a = 0; a < 3; ++a) P.o[a] = P.w[a] = P.vo[a] = 0.0;
    for (int i = d - 1; i >= 0; --i) {
        const NodeDev &N = nodes[chain[i]];
        double sph, cph, st, ct;
        sincos(N.freq * t + N.phase, &sph, &cph);
        const double th = N.angle0 + N.omega * t + N.amp * sph;
        const double dth = N.omega + N.amp * N.freq * cph;
        sincos(th, &st, &ct);
        const double *a = N.axis;
        const double k1 = 1.0 - ct;
        // rotation by th about the unit axis a (Rodrigues)
        const double R[9] = {ct + k1 * a[0] * a[0],        k1 * a[0] * a[1] - st * a[2], k1 * a[0] * a[2] + st * a[1],
                             k1 * a[1] * a[0] + st * a[2], ct + k1 * a[1] * a[1],        k1 * a[1] * a[2] - st * a[0],
                             k1 * a[2] * a[0] - st * a[1], k1 * a[2] * a[1] + st * a[0], ct + k1 * a[2] * a[2]};
        double TpTr[9], Tn[9], pr[3], dpr[3], Tpr[3], Tdpr[3], wa[3], wx[3];
        m3mul(P.T, N.rot, TpTr);
        m3mul(TpTr, R, Tn);
        for (int c = 0; c < 3; ++c) {
            pr[c] = N.pos[c] + N.disp[c] * sph;
            dpr[c] = N.disp[c] * N.freq * cph;
        }
        m3vec(P.T, pr, Tpr);
        m3vec(P.T, dpr, Tdpr);
        m3vec(TpTr, N.axis, wa);
        cross3(P.w, Tpr, wx);
        for (int c = 0; c < 3; ++c) {
            P.o[c] += Tpr[c];
            P.vo[c] += wx[c] + Tdpr[c];
            P.w[c] += dth * wa[c];
        }
        for (int c = 0; c < 9; ++c) P.T[c] = Tn[c];
    }
}

// cos and sin of blade b's azimuth azimuth0 + omega t + 2 pi b / n_blades at
// the launch's step, by angle addition from the step's cos, sin of
// azimuth0 + omega t (computed on the host in FP64 per launch) and the
// blade's offset (a table written when the rotor is set): no trigonometry on
// the device
__device__ __forceinline__ void blade_azimuth(const RotorDev &R, int b, double &ct, double &st) {
    const double cb = R.blade_cs[2 * b], sb = R.blade_cs[2 * b + 1];
    ct = R.cos_az * cb - R.sin_az * sb;
    st = R.sin_az * cb + R.cos_az * sb;
}

// Position (and, with v != nullptr, velocity and the node pose) of point p
// of slot R at time t: a rotor's blade element or a turbine point.
__device__ __forceinline__ void slot_point(const RotorDev &R, const TreePose *poses, int p, double t, double xp[3],
                                           double *v, TreePose *pose, double *Tq) {
    if (R.nodes) {
        const TreePointDev &tp = R.tpts[p];
        const TreePose &P = poses[tp.node];
        double q[3] = {tp.q[0], tp.q[1], tp.q[2]}, tq[3];
        m3vec(P.T, q, tq);
        for (int a = 0; a < 3; ++a) xp[a] = P.o[a] + tq[a];
        if (v) {
            double wq[3];
            cross3(P.w, tq, wq);
            for (int a = 0; a < 3; ++a) {
                v[a] = P.vo[a] + wq[a];
                Tq[a] = tq[a];
            }
            *pose = P;
        }
    } else {
        const int b = p / R.n_points, k = p % R.n_points;
        const double rr = R.r[k];
        double ct, st;
        blade_azimuth(R, b, ct, st);
        xp[0] = R.hub[0];
        xp[1] = R.hub[1] + rr * ct;
        xp[2] = R.hub[2] + rr * st;
    }
}

// Blade-element force (Sec. 2.2) from the in-plane relative wind: W_n along
// the rotor normal, W_t against the blade's motion; Fn, Ft along e_n, e_t.
// Evaluated in FP32 (the sampled velocity comes from FP32 or 16-bit
// populations and the polars are FP32 tables); the load sums stay FP64.
__device__ __forceinline__ void blade_element(const RotorDev &R, const float *cl, const float *cd, double rho_d,
                                              double wn_d, double wt_d, double chord, double dl, double twist,
                                              double pitch, int tip_loss, double r, double &Fn_d, double &Ft_d) {
    const float rho = (float)rho_d, wn = (float)wn_d, wt = (float)wt_d;
    const float phi = atan2f(wn, wt);
    float a = phi * (float)(180.0 / PI_D) - (float)twist - (float)pitch;
    // |phi| <= 180 and |twist + pitch| < 180: one correction wraps to [-180, 180)
    if (a >= 180.0f) a -= 360.0f;
    else if (a < -180.0f) a += 360.0f;
    float CL, CD;
    polar_pair(a, R, cl, cd, CL, CD);
    const float w2 = wn * wn + wt * wt, wm = sqrtf(w2);
    const float q = 0.5f * rho * w2 * (float)chord * (float)dl;
    float Fn = 0.0f, Ft = 0.0f;
    if (wm > 0.0f) {
        Fn = q * (CL * wt + CD * wn) / wm;
        Ft = q * (CL * wn - CD * wt) / wm;
    }
    if (tip_loss) {
        const float Fl = tip_loss_factor(R.n_blades, (float)R.radius, (float)r, phi);
        Fn *= Fl;
        Ft *= Fl;
    }
    Fn_d = Fn;
    Ft_d = Ft;
}

// Points are processed in batches of 32: workgroup (b, r) handles points
// 32b .. 32b+31 of slot r. Its 256 threads first stage the density and
// velocity of the 8 cells around each of the 32 points in LDS (thread ->
// point, corner), then 32 threads interpolate and evaluate the force model.
// A rotor leaves FP64 partial thrust and torque per workgroup (the host adds
// the partials in batch order when the loads are read); a turbine leaves
// per point x, v, F and the moment (x - o_node) x F, which the host sums
// per node.
constexpr int ALM_BATCH = ALM_BLOCK / 8;
static_assert(ALM_BATCH == ALM_BATCH_PTS, "batch size shared with the host-side load sum");
constexpr int ALM_MAX_BATCHES = ALM_MAX_PTS / ALM_BATCH;

struct PointsLds {
    double corner[ALM_BLOCK][4];     // rho, u of one corner cell per work item
    TreePose pose[TREE_MAX_NODES];   // turbine: every node's pose at this step
    NodeDev nodes[TREE_MAX_NODES];   // turbine: the node table
};

// batch bx of slot by
template <typename T, int PAR>
__device__ __forceinline__ void alm_points_wg(const Geo &g, const Physics &ph, const RotorDev *rots, long t, int bx,
                                              int by, PointsLds &L) {
    const RotorDev &R = rots[by];
    const int npts = R.npts;
    const int base = bx * ALM_BATCH;
    if (base >= npts) return;  // uniform across the workgroup
    double(*s_corner)[4] = L.corner;
    TreePose *s_pose = L.pose;
    NodeDev *s_nodes = L.nodes;
    // the blade data of the batch's points into registers, in flight with
    // the sampling
    double pre_r = 0.0, pre_chord = 0.0, pre_dl = 0.0, pre_twist = 0.0, pre_ct = 0.0, pre_st = 0.0;
    if (!R.nodes && threadIdx.x < ALM_BATCH && base + (int)threadIdx.x < npts) {
        const int k = (base + (int)threadIdx.x) % R.n_points, b = (base + (int)threadIdx.x) / R.n_points;
        pre_r = R.r[k];
        pre_chord = R.chord[k];
        pre_dl = R.dl[k];
        pre_twist = R.twist[k];
        blade_azimuth(R, b, pre_ct, pre_st);
    }
    if (R.nodes) {
        // one coalesced copy of the node table, so that the pose recursion
        // walks the parent chain in LDS rather than through one dependent
        // global load per level (n_nodes <= TREE_MAX_NODES, checked on the host)
        constexpr int NW = (int)(sizeof(NodeDev) / 8);
        const unsigned long long *src = (const unsigned long long *)R.nodes;
        unsigned long long *dst = (unsigned long long *)s_nodes;
        for (int q = threadIdx.x; q < R.n_nodes * NW; q += ALM_BLOCK) dst[q] = src[q];
        __syncthreads();
        if (threadIdx.x < R.n_nodes) tree_pose(s_nodes, threadIdx.x, (double)t, s_pose[threadIdx.x]);
        __syncthreads();
    }
    {
        const int p = base + threadIdx.x / 8, corner = threadIdx.x % 8;
        if (p < npts) {
            double xp[3];
            slot_point(R, s_pose, p, (double)t, xp, nullptr, nullptr, nullptr);
            const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
            const int cx = wrap_any((int)floor(xp[0]) + dx, g.nx);
            const int cy = wrap_any((int)floor(xp[1]) + dy, g.ny);
            const int cz = wrap_any((int)floor(xp[2]) + dz, g.nz);
            double r, ux, uy, uz;
            cell_macro<T, PAR>(g, ph, ((size_t)cz * g.ny + cy) * g.nx + cx, cx, cy, cz, r, ux, uy, uz);
            s_corner[threadIdx.x][0] = r;
            s_corner[threadIdx.x][1] = ux;
            s_corner[threadIdx.x][2] = uy;
            s_corner[threadIdx.x][3] = uz;
        }
    }
    __syncthreads();
    if (threadIdx.x < ALM_BATCH) {
        const float *pcl = R.cl, *pcd = R.cd;
        double accT = 0.0, accQ = 0.0;
        const int p = base + threadIdx.x;
        if (p < npts) {
            double xp[3], vp[3] = {0, 0, 0}, Tq[3] = {0, 0, 0};
            TreePose P;
            double ct = 0.0, st = 0.0;  // rotor: cos, sin of the blade's azimuth
            if (!R.nodes) {
                // slot_point's arithmetic, with the radius and azimuth loaded at the start
                ct = pre_ct;
                st = pre_st;
                xp[0] = R.hub[0];
                xp[1] = R.hub[1] + pre_r * ct;
                xp[2] = R.hub[2] + pre_r * st;
            } else {
                slot_point(R, s_pose, p, (double)t, xp, vp, &P, Tq);
            }
            double fr[3];
            for (int a = 0; a < 3; ++a) fr[a] = xp[a] - floor(xp[a]);
            double sm[4] = {0, 0, 0, 0};
            for (int c = 0; c < 8; ++c) {
                const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
                const double w = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) * (dz ? fr[2] : 1.0 - fr[2]);
                for (int q = 0; q < 4; ++q) sm[q] += w * s_corner[threadIdx.x * 8 + c][q];
            }
            const double rho = sm[0];
            double Fp[3] = {0.0, 0.0, 0.0};
            if (!R.nodes) {
                const double rr = pre_r;  // R.r[k], R.chord[k], ... loaded at the start
                // e_theta = (0, -sin, cos); relative in-plane wind W = W_n e_x - W_t e_theta
                const double ut = -sm[2] * st + sm[3] * ct;
                const double wn = sm[1];
                const double wt = -(ut - R.omega_rot * rr);
                double Fn, Ft;
                blade_element(R, pcl, pcd, rho, wn, wt, pre_chord, pre_dl, pre_twist, R.pitch_deg, R.tip_loss, rr, Fn,
                              Ft);
                Fp[0] = Fn;
                Fp[1] = -Ft * st;
                Fp[2] = Ft * ct;
                accT = Fn;
                accQ = rr * Ft;
            } else {
                const TreePointDev &tp = R.tpts[p];
                const NodeDev &N = s_nodes[tp.node];
                const double W[3] = {sm[1] - vp[0], sm[2] - vp[1], sm[3] - vp[2]};
                if (N.force == LBM_FORCE_BLADE) {
                    double es[3], en[3], et[3];
                    m3vec(P.T, N.dir, es);
                    m3vec(P.T, N.normal, en);
                    cross3(en, es, et);
                    const double wn = dot3(W, en), wt = -dot3(W, et);
                    double Fn, Ft;
                    blade_element(R, pcl, pcd, rho, wn, wt, tp.chord, tp.measure, tp.twist, N.pitch_deg, N.tip_loss,
                                  tp.s, Fn, Ft);
                    for (int a = 0; a < 3; ++a) Fp[a] = Fn * en[a] + Ft * et[a];
                } else if (N.force == LBM_FORCE_DRAG && N.kind == LBM_NODE_LINE) {
                    // cross-flow drag of a cylinder: the part of W normal to the line
                    double es[3], Wp[3];
                    m3vec(P.T, N.dir, es);
                    const double ws = dot3(W, es);
                    for (int a = 0; a < 3; ++a) Wp[a] = W[a] - ws * es[a];
                    const double c = 0.5 * rho * N.coef * tp.chord * tp.measure * sqrt(dot3(Wp, Wp));
                    for (int a = 0; a < 3; ++a) Fp[a] = c * Wp[a];
                } else if (N.force == LBM_FORCE_DRAG) {
                    // disk: force along the normal (the node's x axis) on the normal wind
                    const double n[3] = {P.T[0], P.T[3], P.T[6]};
                    const double wn = dot3(W, n);
                    const double c = 0.5 * rho * N.coef * tp.measure * fabs(wn) * wn;
                    for (int a = 0; a < 3; ++a) Fp[a] = c * n[a];
                }
                double m[3];
                cross3(Tq, Fp, m);
                double *o = R.pt_force + (size_t)TREE_PT_OUT * p;
                for (int a = 0; a < 3; ++a) {
                    o[a] = xp[a];
                    o[3 + a] = vp[a];
                    o[6 + a] = Fp[a];
                    o[9 + a] = m[a];
                }
            }
            // the record the spreading kernel reads (which also normalises the
            // Gaussian weights, from the per-axis tables it builds anyway)
            float *Pt = R.pts + (size_t)p * PT_STRIDE;
            for (int ax = 0; ax < 3; ++ax) {
                const int c0 = (int)floor(xp[ax] + 0.5);
                Pt[ax] = (float)(xp[ax] - c0);  // offset from the nearest node
                Pt[3 + ax] = (float)(-Fp[ax]);
                Pt[6 + ax] = (float)c0;
                if (!R.nodes) R.pt_force[3 * p + ax] = Fp[ax];
            }
        }
        // thrust and torque of the batch: the same pairwise tree in FP64 as
        // an LDS reduction (lane i adds lane i + s for s = 16, 8, 4, 2, 1), in
        // registers across the batch's 32 lanes of the first wave
        for (int s = ALM_BATCH / 2; s > 0; s >>= 1) {
            accT += __shfl_down(accT, s);
            accQ += __shfl_down(accQ, s);
        }
        if (threadIdx.x == 0) {
            R.loads[3 + 2 * bx] = accT;
            R.loads[4 + 2 * bx] = accQ;
        }
    }
}

// Gather-form spreading over one slot's box: F(X) = sum_p (-F_p) eta(X - x_p) / W_p.
// One workgroup per tile of SP_TX x SP_TY x SP_TZ box cells. The workgroup
// first keeps the points whose support reaches the tile, those of even index
// and then those of odd index, each in point order (a ballot compaction per
// wave, then the waves' counts in order). Both
// kernels are products of one factor per axis (the Gaussian's exponential
// splits, Roma's delta is defined that way), so the workgroup tabulates, for
// each kept point, the factor of every support offset on each axis in LDS
// (Gaussian: W_p, the sum of its weights over the support, is the product of
// the three table sums; the Roma delta's weights sum to one). The y and z
// factors, 1 / W_p and -F_p are then combined once per (point, (y, z) row of
// the tile), and each cell sums over the kept points g_x(X) times its row's
// vector. Two threads share a cell: one sums the points of even index, the
// other those of odd index, each in point order, and the cell's force is the
// even sum plus the odd sum: the same terms, each rounded the same way and
// grouped the same way wherever the tile boundaries fall, so the result does
// not depend on the tiling. Points are taken in chunks of SP_CHUNK.
constexpr int SP_TX = 16, SP_TY = 4, SP_TZ = 4;
constexpr int SP_CELLS = SP_TX * SP_TY * SP_TZ;
constexpr int SP_BLOCK = 2 * SP_CELLS;  // two threads per cell
constexpr int SP_CHUNK = 64;
constexpr int SP_UNROLL = 8;
constexpr int SP_ROWS = SP_TY * SP_TZ;  // (y, z) rows of SP_TX cells in a tile
// a kept point as the per-cell sum reads it (two 16-byte LDS reads): its
// nearest node minus the support half-width, 1 / W_p and -F_p
struct KeptPoint {
    int c[3];
    float inv_w;
    float f[3];
    float pad;
};
static_assert(sizeof(KeptPoint) == 32, "two 16-byte reads");
constexpr int SP_W = 2 * SUPPORT + 1;  // widest support (Gaussian), offsets -SUPPORT..SUPPORT

// One launch spreads every slot: workgroups [first[r], first[r+1]) take the
// tiles of slot r (tile counts per axis in tiles[r]).
// what the spreading workgroups read of each slot, passed by value (kernel
// arguments) so that a workgroup needs no load of the slot table first
struct SpreadSlot {
    const float *pts;
    float *Fbox;
    ForceBox box;
    int npts, half;
    int roma;   // Roma delta (else Gaussian)
    float ie2;  // Gaussian: 1 / eps^2
};
struct SpreadTiles {
    int nslots;
    int first[MAX_ROTORS + 1];
    int tx[MAX_ROTORS], ty[MAX_ROTORS];
    SpreadSlot slot[MAX_ROTORS];
};

struct SpreadLds {
    // the kept points' records, in point order: offset from the nearest node,
    // the nearest node minus the support half-width, -F and (per chunk) 1 / W_p
    float off[ALM_MAX_PTS][3];
    KeptPoint k[ALM_MAX_PTS];
    int wave[SP_BLOCK / 64];
    float part[SP_CELLS][3];         // the odd-index sums of each cell
    float g[SP_CHUNK][3][SP_W];      // per-axis factors of a chunk of kept points
    float sum[SP_CHUNK][3];          // and their sums over the support
    float4 row[SP_CHUNK][SP_ROWS];   // y, z factors x 1/W_p x (-F_p) per tile row
};

// the spreading workgroup blk of the launch (over all slots)
__device__ __forceinline__ void alm_spread_wg(const SpreadTiles &st, int blk_all, SpreadLds &L) {
    int rid = 0;
    while (rid + 1 < st.nslots && blk_all >= st.first[rid + 1]) ++rid;  // uniform per workgroup
    const int blk = blk_all - st.first[rid], tiles_x = st.tx[rid], tiles_y = st.ty[rid];
    const SpreadSlot &R = st.slot[rid];
    const int npts = R.npts;
    const ForceBox &B = R.box;
    const int half = R.half, W = 2 * half + 1;  // half <= SUPPORT (checked on the host)
    float(*s_off)[3] = L.off;
    KeptPoint *s_k = L.k;
    int *s_wave = L.wave;
    float(*s_g)[3][SP_W] = L.g;
    float(*s_sum)[3] = L.sum;
    float4(*s_row)[SP_ROWS] = L.row;
    const int tx = blk % tiles_x, ty = (blk / tiles_x) % tiles_y, tz = blk / (tiles_x * tiles_y);
    // tile extent in lattice coordinates (clipped to the box)
    const int X0 = B.x0 + tx * SP_TX, Y0 = B.y0 + ty * SP_TY, Z0 = B.z0 + tz * SP_TZ;
    const int X1 = min(X0 + SP_TX, B.x0 + B.bnx) - 1, Y1 = min(Y0 + SP_TY, B.y0 + B.bny) - 1,
              Z1 = min(Z0 + SP_TZ, B.z0 + B.bnz) - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // kept points: those of even index first, then those of odd index, each
    // group in point order
    int count = 0, n_even = 0;  // uniform across the workgroup
    for (int parity = 0; parity < 2; ++parity) {
        for (int k0 = 0; k0 < npts; k0 += SP_BLOCK) {
            const int p = k0 + threadIdx.x;
            bool reach = false;
            float rec[9];
            if (p < npts && (p & 1) == parity) {
                // the whole record in one round trip, kept in LDS if the point reaches the tile
                const float *P = R.pts + (size_t)p * PT_STRIDE;
#pragma unroll
                for (int q = 0; q < 9; ++q) rec[q] = P[q];
                const int cx = (int)rec[6], cy = (int)rec[7], cz = (int)rec[8];
                reach = cx - half <= X1 && cx + half >= X0 && cy - half <= Y1 && cy + half >= Y0 &&
                        cz - half <= Z1 && cz + half >= Z0;
            }
            const unsigned long long bal = __ballot(reach);
            if (lane == 0) s_wave[wave] = __popcll(bal);
            __syncthreads();
            int off = count;
            for (int w = 0; w < wave; ++w) off += s_wave[w];
            if (reach) {
                const int k = off + __popcll(bal & ((1ull << lane) - 1ull));
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    s_off[k][a] = rec[a];
                    s_k[k].f[a] = rec[3 + a];
                    s_k[k].c[a] = (int)rec[6 + a] - half;
                }
            }
            for (int w = 0; w < SP_BLOCK / 64; ++w) count += s_wave[w];
            __syncthreads();
        }
        if (parity == 0) n_even = count;
    }
    // two threads per cell: the first sums the kept points of even index, the
    // second those of odd index (each in point order), and F = F_even + F_odd
    const int cell = (int)threadIdx.x % SP_CELLS, grp = (int)threadIdx.x / SP_CELLS;
    const int lo = grp == 0 ? 0 : n_even, hi = grp == 0 ? n_even : count;
    const int X = X0 + cell % SP_TX, Y = Y0 + (cell / SP_TX) % SP_TY, Z = Z0 + cell / (SP_TX * SP_TY);
    const bool mine = X <= X1 && Y <= Y1 && Z <= Z1;  // threads past the box edge keep to the barriers
    const float ie2 = R.ie2;
    const bool roma = R.roma != 0;  // uniform over the grid
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    for (int c0 = 0; c0 < count; c0 += SP_CHUNK) {
        const int nk = min(SP_CHUNK, count - c0);
        // factors: e = d - (x_p - node) for d = -half..half on each axis, one
        // thread per (point, axis), which also sums its row
        for (int q = threadIdx.x; q < nk * 3; q += SP_BLOCK) {
            const int k = q / 3, ax = q % 3;
            const float o = s_off[c0 + k][ax];
            float sa = 0.0f;
            for (int d = 0; d < W; ++d) {
                const float e = (float)(d - half) - o;
                const float v = roma ? roma_phi(e) : expf(-e * e * ie2);
                s_g[k][ax][d] = v;
                sa += v;
            }
            s_sum[k][ax] = sa;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nk; q += SP_BLOCK) {
            double S = 1.0;
            if (!roma)
                for (int ax = 0; ax < 3; ++ax) S *= (double)s_sum[q][ax];
            s_k[c0 + q].inv_w = (float)(1.0 / S);
        }
        __syncthreads();
        // the y and z factors of each kept point for each (y, z) row of the
        // tile, times 1 / W_p and -F_p: one float4 per (point, row), with the
        // point's window start in x (zero where the row is outside its window)
        for (int q = threadIdx.x; q < nk * SP_ROWS; q += SP_BLOCK) {
            const int k = q / SP_ROWS, r = q % SP_ROWS;
            const KeptPoint &P = s_k[c0 + k];
            const int dy = Y0 + r % SP_TY - P.c[1], dz = Z0 + r / SP_TY - P.c[2];
            const bool in = (unsigned)dy < (unsigned)W && (unsigned)dz < (unsigned)W;
            const float a = in ? s_g[k][1][dy] * s_g[k][2][dz] * P.inv_w : 0.0f;
            s_row[k][r] = make_float4(a * P.f[0], a * P.f[1], a * P.f[2], __int_as_float(P.c[0]));
        }
        __syncthreads();
        // this thread's kept points within the chunk, as chunk positions
        const int k_lo = max(lo, c0) - c0, k_hi = min(hi, c0 + nk) - c0;
        if (mine && k_lo < k_hi) {
            // per cell: F += g_x(X) A(row); SP_UNROLL points at a time, so that
            // their LDS reads are in flight together, in point order
            const int r = cell / SP_TX;
            for (int k0 = k_lo; k0 < k_hi; k0 += SP_UNROLL) {
                float gx[SP_UNROLL];
                float4 A[SP_UNROLL];
                bool in[SP_UNROLL];
#pragma unroll
                for (int u = 0; u < SP_UNROLL; ++u) {
                    const int k = k0 + u < k_hi ? k0 + u : k0;  // past the end: a valid entry, not used
                    A[u] = s_row[k][r];
                    const int dx = X - __float_as_int(A[u].w);
                    in[u] = k0 + u < k_hi && (unsigned)dx < (unsigned)W;
                    gx[u] = s_g[k][0][in[u] ? dx : 0];
                }
#pragma unroll
                for (int u = 0; u < SP_UNROLL; ++u)
                    if (in[u]) {
                        Fx = fmaf(gx[u], A[u].x, Fx);
                        Fy = fmaf(gx[u], A[u].y, Fy);
                        Fz = fmaf(gx[u], A[u].z, Fz);
                    }
            }
        }
        __syncthreads();  // the next chunk overwrites the tables
    }
    // the odd-index sums to the threads of the even-index ones
    if (grp == 1) {
        L.part[cell][0] = Fx;
        L.part[cell][1] = Fy;
        L.part[cell][2] = Fz;
    }
    __syncthreads();
    if (grp == 1 || !mine) return;
    Fx += L.part[cell][0];
    Fy += L.part[cell][1];
    Fz += L.part[cell][2];
    const size_t nb = (size_t)B.bnx * B.bny * B.bnz;
    const size_t c = (size_t)(X - B.x0) + (size_t)B.bnx * ((size_t)(Y - B.y0) + (size_t)B.bny * (size_t)(Z - B.z0));
    R.Fbox[c] = Fx;
    R.Fbox[nb + c] = Fy;
    R.Fbox[2 * nb + c] = Fz;
}

// Two launches per step: the point batches, then the spreading tiles, which
// read every point's record. (Tried and dropped: one launch whose spreading
// workgroups wait on an arrival counter of the point workgroups; the
// device-scope fences and the wait cost more than the launch they save.)
// every slot's parameters, passed by value (kernel arguments) so that a
// workgroup needs no load of the slot table before its first dependent load
struct RotorSet {
    RotorDev r[MAX_ROTORS];
};
// kernel arguments are limited to 4 KiB
static_assert(sizeof(Geo) + sizeof(Physics) + sizeof(RotorSet) + sizeof(long) <= 4096, "points-kernel arguments");
static_assert(sizeof(SpreadTiles) <= 4096, "spreading-kernel arguments");

template <typename T, int PAR>
__global__ __launch_bounds__(ALM_BLOCK) void k_alm_points(Geo g, Physics ph, RotorSet rs, long t) {
    __shared__ PointsLds L;
    alm_points_wg<T, PAR>(g, ph, rs.r, t, (int)blockIdx.x, (int)blockIdx.y, L);
}

__global__ __launch_bounds__(SP_BLOCK) void k_alm_spread(SpreadTiles st) {
    __shared__ SpreadLds L;
    alm_spread_wg(st, (int)blockIdx.x, L);
}

template <typename T, int PAR>
static void alm_t(const Geo &g, const Physics &ph, const RotorDev *h_rots, int nrot, long t,
                  hipStream_t s) {
    int nb = 1;
    for (int r = 0; r < nrot; ++r) {
        const int b = (h_rots[r].npts + ALM_BATCH - 1) / ALM_BATCH;
        nb = b > nb ? b : nb;
    }
    RotorSet rs{};
    for (int r = 0; r < nrot; ++r) {
        rs.r[r] = h_rots[r];
        const double az = h_rots[r].azimuth0 + h_rots[r].omega_rot * (double)t;
        rs.r[r].cos_az = cos(az);
        rs.r[r].sin_az = sin(az);
    }
    k_alm_points<T, PAR><<<dim3(nb, nrot), ALM_BLOCK, 0, s>>>(g, ph, rs, t);
    SpreadTiles st{};
    st.nslots = nrot;
    for (int r = 0; r < nrot; ++r) {
        const ForceBox &B = h_rots[r].box;
        const int tx = (B.bnx + SP_TX - 1) / SP_TX, ty = (B.bny + SP_TY - 1) / SP_TY, tz = (B.bnz + SP_TZ - 1) / SP_TZ;
        st.tx[r] = tx;
        st.ty[r] = ty;
        st.first[r + 1] = st.first[r] + tx * ty * tz;
        const RotorDev &R = h_rots[r];
        SpreadSlot &S = st.slot[r];
        S.pts = R.pts;
        S.Fbox = R.Fbox;
        S.box = R.box;
        S.npts = R.npts;
        S.half = R.half;
        S.roma = R.kernel == LBM_KERNEL_ROMA3;
        S.ie2 = R.kernel == LBM_KERNEL_GAUSS ? (float)(1.0 / (R.eps * R.eps)) : 0.0f;
    }
    k_alm_spread<<<(unsigned)st.first[nrot], SP_BLOCK, 0, s>>>(st);
}

int launch_alm(int storage, int parity, const Geo &g, const Physics &ph, const RotorDev *h_rots, int nrot,
               long t, hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: alm_t<float, 0>(g, ph, h_rots, nrot, t, s); break;
        case 1: alm_t<float, 1>(g, ph, h_rots, nrot, t, s); break;
        case 2: alm_t<__half, 0>(g, ph, h_rots, nrot, t, s); break;
        case 3: alm_t<__half, 1>(g, ph, h_rots, nrot, t, s); break;
        case 4: alm_t<bf16_t, 0>(g, ph, h_rots, nrot, t, s); break;
        case 5: alm_t<bf16_t, 1>(g, ph, h_rots, nrot, t, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lbm
