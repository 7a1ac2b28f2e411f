// Host side of the C ABI declared in include/lbm.h: argument validation,
// device bookkeeping and the per-step kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

struct RotorHost {
    bool on = false;
    RotorDev dev{};  // host copy of the device description (device pointers inside)
    int npts = 0;
    double *d_r = nullptr, *d_chord = nullptr, *d_twist = nullptr, *d_dl = nullptr;
    float *d_cl = nullptr, *d_cd = nullptr, *d_pts = nullptr, *d_Fbox = nullptr;
    double *d_ptf = nullptr, *d_loads = nullptr;
    double *d_bcs = nullptr;             // rotor: cos, sin of each blade's azimuth offset 2 pi b / B
    size_t ptf_len = 0;                  // doubles in d_ptf
    // turbine tree (Sec. 3.3): device nodes and points, node of each point
    NodeDev *d_nodes = nullptr;
    TreePointDev *d_tpts = nullptr;
    int n_nodes = 0;
    std::vector<int> pt_node;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct lbm_ctx {
    lbm_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t n = 0, esize = 4;
    int nbx = 0;          // blocks of blk_width(esize) cells per x row
    size_t zplane = 0;    // elements per z plane of the blocked store
    size_t pop_bytes = 0, aux_bytes = 0;
    size_t off_ghost = 0, off_uin = 0, off_part = 0, off_flag = 0;
    void *pops = nullptr, *aux = nullptr;
    bool attached = false;
    long t = 0;
    int parity = 0;
    float omega2 = 1.0f;
    float omega_hi[8] = {1, 1, 1, 1, 1, 1, 1, 1};  // omega_3 .. omega_10
    bool general_rates = false;
    float *d_ffield = nullptr;
    RotorHost rot[MAX_ROTORS];
    std::vector<RotorDev> h_rots;
    MlpDev *d_mlp = nullptr;
    bool mlp_set = false;
    double mass0 = 0.0;
    bool mass0_set = false;
    double *d_stage = nullptr;
    size_t stage_bytes = 0;
    float *d_in_mean = nullptr, *d_in_box = nullptr;  // time-dependent inlet
    int in_lt = 0;
    double in_advect = 0.0;
    std::string err;
};

namespace {

int fail(lbm_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(ctx, LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// No exception crosses the C ABI: a failed host allocation inside an entry
// point (a staging vector, the error string) returns LBM_ENOMEM, anything
// else LBM_EINVAL, with the message kept when it can be stored.
template <typename F>
int guard(const lbm_ctx *cc, F &&body) noexcept {
    lbm_ctx *c = const_cast<lbm_ctx *>(cc);
    int code;
    const char *msg;
    try {
        return body();
    } catch (const std::bad_alloc &) {
        code = LBM_ENOMEM;
        msg = "host allocation failed";
    } catch (const std::length_error &) {
        code = LBM_ENOMEM;
        msg = "host allocation too large";
    } catch (...) {
        code = LBM_EINVAL;
        msg = "unexpected host error";
    }
    if (c) {
        try {
            c->err = msg;
        } catch (...) {
        }
    }
    return code;
}

// Two inlet planes alternate: plane[t % 2] holds the inlet velocity of step t.
// A swapped-layout read at time t completes the streaming of step t - 1 and
// so takes plane[(t + 1) % 2]; the inlet writes of an odd step t take plane[t % 2].
size_t plane_floats(const lbm_ctx *c) { return 3 * (size_t)c->cfg.ny * c->cfg.nz; }
float *uin_plane(const lbm_ctx *c, long t) {
    const size_t stride = (plane_floats(c) * sizeof(float) + 255) / 256 * 256;
    return (float *)((char *)c->aux + c->off_uin + (size_t)(t & 1) * stride);
}

Geo geo_of(const lbm_ctx *c) {
    Geo g{};
    g.pops = c->pops;
    g.nbx = c->nbx;
    g.nx = c->cfg.nx;
    g.ny = c->cfg.ny;
    g.nz = c->cfg.nz;
    g.bc_x = c->cfg.bc_x;
    g.bc_zlo = c->cfg.bc_z_lo;
    g.bc_zhi = c->cfg.bc_z_hi;
    g.uin_rd = uin_plane(c, c->t + 1);
    g.uin_wr = uin_plane(c, c->t);
    g.ghost = (char *)c->aux + c->off_ghost;
    return g;
}

bool has_force(const lbm_ctx *c) {
    return c->cfg.body_force[0] != 0.0 || c->cfg.body_force[1] != 0.0 || c->cfg.body_force[2] != 0.0 ||
           c->d_ffield != nullptr || !c->h_rots.empty();
}

Physics physics_of(const lbm_ctx *c) {
    Physics ph{};
    ph.omega = (float)c->cfg.omega;
    ph.omega2 = c->omega2;
    ph.tau0 = (float)(1.0 / c->cfg.omega);
    ph.smag_c = (float)(18.0 * std::sqrt(2.0) * c->cfg.cs_smag * c->cfg.cs_smag);
    ph.nu0 = (float)((1.0 / c->cfg.omega - 0.5) / 3.0);
    for (int k = 0; k < 8; ++k) ph.omega_hi[k] = c->omega_hi[k];
    for (int k = 0; k < 3; ++k) ph.bf[k] = (float)c->cfg.body_force[k];
    ph.ffield = c->d_ffield;
    ph.nbox = (int)c->h_rots.size();
    for (int r = 0; r < ph.nbox; ++r) ph.box[r] = c->h_rots[r].box;
    ph.mlp = c->d_mlp;
    return ph;
}

// The fast stream-collide path needs 32-bit byte offsets within one z plane
// of the blocked store; with them, a periodic box runs it everywhere and an
// open one on every cell off the z walls (odd steps). Otherwise: the general
// path.
bool fast_offsets_fit(const lbm_ctx *c) { return c->zplane * c->esize < ((size_t)1 << 32); }
bool general_bc(const lbm_ctx *c) {
    return c->cfg.bc_x != LBM_BC_PERIODIC || c->cfg.bc_z_lo != LBM_BC_PERIODIC || c->cfg.bc_z_hi != LBM_BC_PERIODIC ||
           !fast_offsets_fit(c);
}
static int sc_mode(const lbm_ctx *c) {
    if (c->cfg.general_path || !fast_offsets_fit(c)) return SC_GENERAL;
    return general_bc(c) ? SC_SPLIT : SC_FAST;
}

int ensure_stage(lbm_ctx *c, size_t bytes) {
    if (c->stage_bytes >= bytes) return LBM_OK;
    if (c->d_stage) (void)hipFree(c->d_stage);
    c->d_stage = nullptr;
    c->stage_bytes = 0;
    if (hipMalloc((void **)&c->d_stage, bytes) != hipSuccess) return fail(c, LBM_ENOMEM, "staging buffer of %zu bytes", bytes);
    c->stage_bytes = bytes;
    return LBM_OK;
}

// cells per host<->device chunk (keeps the staging buffer modest)
size_t chunk_cells(const lbm_ctx *c) {
    const size_t target = (size_t)1 << 22;
    return c->n < target ? c->n : target;
}

int ready(lbm_ctx *c) {
    if (!c) return LBM_EINVAL;
    if (!c->attached) return fail(c, LBM_ESTATE, "call lbm_attach first");
    return LBM_OK;
}

int refresh_rotor_table(lbm_ctx *c) {
    // the active slots in slot order; the actuator-line kernels take them by
    // value at each launch
    c->h_rots.clear();
    for (int r = 0; r < MAX_ROTORS; ++r)
        if (c->rot[r].on) c->h_rots.push_back(c->rot[r].dev);
    return LBM_OK;
}

void free_rotor(RotorHost &R) {
    void *ptrs[] = {R.d_bcs, R.d_r,   R.d_chord, R.d_twist, R.d_dl,    R.d_cl,   R.d_cd,
                    R.d_pts, R.d_Fbox,  R.d_ptf,   R.d_loads, R.d_nodes, R.d_tpts};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    R = RotorHost{};
}

int zero_rotor_boxes(lbm_ctx *c) {
    for (int r = 0; r < MAX_ROTORS; ++r) {
        RotorHost &R = c->rot[r];
        if (!R.on) continue;
        const size_t nb = (size_t)R.dev.box.bnx * R.dev.box.bny * R.dev.box.bnz;
        HIPCHK(c, hipMemsetAsync(R.d_Fbox, 0, 3 * nb * sizeof(float), c->stream));
        HIPCHK(c, hipMemsetAsync(R.d_loads, 0, ALM_LOADS_LEN * sizeof(double), c->stream));
        HIPCHK(c, hipMemsetAsync(R.d_ptf, 0, R.ptf_len * sizeof(double), c->stream));
    }
    return LBM_OK;
}

int after_init(lbm_ctx *c) {
    c->t = 0;
    c->parity = 0;
    c->mass0_set = false;
    int rc = zero_rotor_boxes(c);
    if (rc) return rc;
    HIPCHK(c, hipMemsetAsync((char *)c->aux + c->off_ghost, 0, c->off_uin - c->off_ghost, c->stream));
    return LBM_OK;
}

int moments_now(lbm_ctx *c, double out[RED_NMOM]) {
    Geo g = geo_of(c);
    Physics ph = physics_of(c);
    double *part = (double *)((char *)c->aux + c->off_part);
    double *res = part + (size_t)RED_NBLOCKS * RED_NMOM;
    if (launch_moments((int)c->cfg.storage, c->parity, g, ph, part, RED_NBLOCKS, res, c->stream))
        return fail(c, LBM_EHIP, "moment reduction launch failed");
    HIPCHK(c, hipMemcpyAsync(out, res, RED_NMOM * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "out of memory";
        case LBM_EHIP: return "HIP runtime error";
        case LBM_EUNSTABLE: return "simulation unstable (mass or NaN check failed)";
        case LBM_ESTATE: return "call out of order";
        default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int lbm_create(const lbm_config *cfg, lbm_ctx **out) {
    return guard(nullptr, [&]() -> int {
        if (!cfg || !out) return LBM_EINVAL;
        *out = nullptr;
        const lbm_config &c = *cfg;
        if (c.nx < 2 || c.ny < 2 || c.nz < 2) return LBM_EINVAL;
        const size_t n = (size_t)c.nx * c.ny * c.nz;
        if (n >= ((size_t)1 << 32)) return LBM_EINVAL;
        if (!(c.omega > 0.0 && c.omega < 2.0)) return LBM_EINVAL;
        for (int k = 0; k < 9; ++k)
            if (!(c.omega_hi[k] >= 0.0 && c.omega_hi[k] < 2.0)) return LBM_EINVAL;
        if (c.storage < LBM_F32 || c.storage > LBM_BF16) return LBM_EINVAL;
        if (c.closure < LBM_CLOSURE_NONE || c.closure > LBM_CLOSURE_MLP) return LBM_EINVAL;
        if (c.closure == LBM_CLOSURE_SMAG && !(c.cs_smag >= 0.0)) return LBM_EINVAL;
        if (c.bc_x != LBM_BC_PERIODIC && c.bc_x != LBM_BC_INFLOW_OUTFLOW) return LBM_EINVAL;
        for (int b : {c.bc_z_lo, c.bc_z_hi})
            if (b != LBM_BC_PERIODIC && b != LBM_BC_NOSLIP && b != LBM_BC_FREESLIP) return LBM_EINVAL;
        if ((c.bc_z_lo == LBM_BC_PERIODIC) != (c.bc_z_hi == LBM_BC_PERIODIC)) return LBM_EINVAL;
        if (c.check_every < 0) return LBM_EINVAL;
        if (c.rounding != LBM_ROUND_STOCHASTIC && c.rounding != LBM_ROUND_NEAREST) return LBM_EINVAL;

        lbm_ctx *x = new (std::nothrow) lbm_ctx();
        if (!x) return LBM_ENOMEM;
        x->cfg = c;
        x->n = n;
        x->esize = c.storage == LBM_F32 ? 4 : 2;
        const int bw = blk_width((int)x->esize);
        x->nbx = (c.nx + bw - 1) / bw;
        x->zplane = (size_t)c.ny * (size_t)x->nbx * 27 * bw;
        x->pop_bytes = round_up((size_t)c.nz * x->zplane * x->esize, 256);
        x->omega2 = c.omega_hi[0] == 0.0 ? 1.0f : (float)c.omega_hi[0];
        for (int k = 0; k < 8; ++k) {
            x->omega_hi[k] = c.omega_hi[k + 1] == 0.0 ? 1.0f : (float)c.omega_hi[k + 1];
            if (x->omega_hi[k] != 1.0f) x->general_rates = true;
        }
        const size_t plane = (size_t)c.ny * c.nz;
        x->off_ghost = 0;
        x->off_uin = round_up(9 * plane * x->esize, 256);
        x->off_part = x->off_uin + 2 * round_up(3 * plane * sizeof(float), 256);
        x->off_flag = x->off_part + round_up(((size_t)RED_NBLOCKS + 2) * RED_NMOM * sizeof(double), 256);
        x->aux_bytes = x->off_flag + 256;
        if (c.stream) {
            x->stream = (hipStream_t)c.stream;
        } else {
            if (hipStreamCreate(&x->stream) != hipSuccess) {
                delete x;
                return LBM_EHIP;
            }
            x->own_stream = true;
        }
        *out = x;
        return LBM_OK;
    });
}

int lbm_destroy(lbm_ctx *c) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        // work in flight may still use buffers freed below (a context that
        // was never attached has enqueued none)
        if (c->stream && (c->attached || c->own_stream)) (void)hipStreamSynchronize(c->stream);
        for (int r = 0; r < MAX_ROTORS; ++r) free_rotor(c->rot[r]);
        if (c->d_ffield) (void)hipFree(c->d_ffield);
        if (c->d_mlp) (void)hipFree(c->d_mlp);
        if (c->d_stage) (void)hipFree(c->d_stage);
        if (c->d_in_mean) (void)hipFree(c->d_in_mean);
        if (c->d_in_box) (void)hipFree(c->d_in_box);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return LBM_OK;
    });
}

int lbm_required_bytes(const lbm_ctx *c, size_t *pop_bytes, size_t *aux_bytes) {
    return guard(c, [&]() -> int {
        if (!c || !pop_bytes || !aux_bytes) return LBM_EINVAL;
        *pop_bytes = c->pop_bytes;
        *aux_bytes = c->aux_bytes;
        return LBM_OK;
    });
}

int lbm_attach(lbm_ctx *c, void *d_pops, void *d_aux) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        if (!d_pops || !d_aux) return fail(c, LBM_EINVAL, "null device buffer");
        if (((uintptr_t)d_pops & 255) || ((uintptr_t)d_aux & 255)) return fail(c, LBM_EINVAL, "buffers must be 256-byte aligned");
        c->pops = d_pops;
        c->aux = d_aux;
        c->attached = true;
        HIPCHK(c, hipMemsetAsync(d_aux, 0, c->aux_bytes, c->stream));
        // uniform inlet plane
        const size_t plane = (size_t)c->cfg.ny * c->cfg.nz;
        std::vector<float> uin(3 * plane);
        for (int d = 0; d < 3; ++d)
            for (size_t q = 0; q < plane; ++q) uin[d * plane + q] = (float)c->cfg.u_in[d];
        for (long b = 0; b < 2; ++b)
            HIPCHK(c, hipMemcpyAsync(uin_plane(c, b), uin.data(), uin.size() * sizeof(float), hipMemcpyHostToDevice,
                                     c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_init_tgv(lbm_ctx *c, double u0, double k, double rho0) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!(rho0 > 0.0) || !std::isfinite(u0) || !std::isfinite(k)) return fail(c, LBM_EINVAL, "bad TGV parameters");
        if (launch_init_tgv((int)c->cfg.storage, geo_of(c), u0, k, rho0, c->stream)) return fail(c, LBM_EHIP, "init launch");
        return after_init(c);
    });
}

int lbm_init_fields(lbm_ctx *c, const double *rho, const double *u) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!rho || !u) return fail(c, LBM_EINVAL, "null field");
        const size_t ch = chunk_cells(c);
        if ((rc = ensure_stage(c, 4 * ch * sizeof(double)))) return rc;
        Geo g = geo_of(c);
        for (size_t c0 = 0; c0 < c->n; c0 += ch) {
            const size_t m = c->n - c0 < ch ? c->n - c0 : ch;
            HIPCHK(c, hipMemcpyAsync(c->d_stage, rho + c0, m * sizeof(double), hipMemcpyHostToDevice, c->stream));
            for (int d = 0; d < 3; ++d)
                HIPCHK(c, hipMemcpyAsync(c->d_stage + m * (1 + d), u + d * c->n + c0, m * sizeof(double),
                                         hipMemcpyHostToDevice, c->stream));
            if (launch_init_eq((int)c->cfg.storage, g, c->d_stage, c->d_stage + m, c0, m, c->stream))
                return fail(c, LBM_EHIP, "init launch");
        }
        rc = after_init(c);
        if (rc) return rc;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_set_rotor(lbm_ctx *c, int id, const lbm_rotor *r) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        if (id < 0 || id >= MAX_ROTORS || !r) return fail(c, LBM_EINVAL, "bad rotor id or null rotor");
        if (r->axis[0] != 1.0 || r->axis[1] != 0.0 || r->axis[2] != 0.0)
            return fail(c, LBM_EINVAL, "rotor axis must be +x");
        if (r->n_blades < 1 || r->n_points < 1 || r->n_blades > ALM_MAX_POINTS || r->n_points > ALM_MAX_POINTS ||
            r->n_blades * r->n_points > ALM_MAX_POINTS)
            return fail(c, LBM_EINVAL, "n_blades*n_points must be in [1, %d]", ALM_MAX_POINTS);
        if (r->n_polar < 2 || !r->r || !r->chord || !r->twist_deg || !r->dl || !r->alpha_deg || !r->cl || !r->cd)
            return fail(c, LBM_EINVAL, "missing rotor arrays");
        {
            auto fin = [](const double *a, int n) {
                for (int k = 0; k < n; ++k)
                    if (!std::isfinite(a[k])) return false;
                return true;
            };
            const double sc[5] = {r->radius, r->omega_rot, r->azimuth0, r->eps, r->pitch_deg};
            if (!fin(r->hub, 3) || !fin(sc, 5) || !fin(r->r, r->n_points) || !fin(r->chord, r->n_points) ||
                !fin(r->twist_deg, r->n_points) || !fin(r->dl, r->n_points) || !fin(r->alpha_deg, r->n_polar) ||
                !fin(r->cl, r->n_polar) || !fin(r->cd, r->n_polar))
                return fail(c, LBM_EINVAL, "non-finite rotor value");
        }
        if (r->kernel != LBM_KERNEL_GAUSS && r->kernel != LBM_KERNEL_ROMA3)
            return fail(c, LBM_EINVAL, "unknown spreading kernel %d", r->kernel);
        if (r->tip_loss != 0 && r->tip_loss != 1) return fail(c, LBM_EINVAL, "tip_loss must be 0 or 1");
        if ((r->kernel == LBM_KERNEL_GAUSS && !(r->eps > 0.0)) || !(r->radius > 0.0))
            return fail(c, LBM_EINVAL, "eps (Gaussian kernel) and radius must be positive");
        // support half-width in nodes around the nearest node: the Roma delta
        // vanishes at 3/2 cells, so round(x_p) +- 1 holds all 27 of its nodes
        const int half = r->kernel == LBM_KERNEL_ROMA3 ? 1 : SUPPORT;
        const double a0 = r->alpha_deg[0], da = (r->alpha_deg[r->n_polar - 1] - a0) / (r->n_polar - 1);
        if (!(da > 0.0)) return fail(c, LBM_EINVAL, "polar angles must ascend");
        for (int k = 0; k < r->n_polar; ++k)
            if (std::fabs(r->alpha_deg[k] - (a0 + k * da)) > 1e-9 * (1.0 + std::fabs(a0)))
                return fail(c, LBM_EINVAL, "polar angle grid must be uniform");
        double rmax = 0.0;
        for (int k = 0; k < r->n_points; ++k) {
            rmax = std::fmax(rmax, std::fabs(r->r[k]));
            if (!(std::fabs(r->twist_deg[k] + r->pitch_deg) < 180.0))
                return fail(c, LBM_EINVAL, "|twist + pitch| must stay below 180 degrees");
        }
        // spreading box: every support node round(x_p) +- half of every point
        const int bx0 = (int)std::floor(r->hub[0] + 0.5) - half, bx1 = (int)std::floor(r->hub[0] + 0.5) + half;
        const int by0 = (int)std::floor(r->hub[1] - rmax + 0.5) - half, by1 = (int)std::floor(r->hub[1] + rmax + 0.5) + half;
        const int bz0 = (int)std::floor(r->hub[2] - rmax + 0.5) - half, bz1 = (int)std::floor(r->hub[2] + rmax + 0.5) + half;
        if (bx0 < 0 || by0 < 0 || bz0 < 0 || bx1 >= c->cfg.nx || by1 >= c->cfg.ny || bz1 >= c->cfg.nz)
            return fail(c, LBM_EINVAL, "rotor spreading box [%d,%d]x[%d,%d]x[%d,%d] leaves the domain", bx0, bx1, by0, by1,
                        bz0, bz1);
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        RotorHost &R = c->rot[id];
        free_rotor(R);
        // on any failure below the slot ends up empty, and the rotor table
        // must stop naming the freed buffers
        const int rc = [&]() -> int {
            const int np = r->n_points, npts = r->n_blades * np, nb = (bx1 - bx0 + 1) * (by1 - by0 + 1) * (bz1 - bz0 + 1);
            bool ok = hipMalloc((void **)&R.d_r, np * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_chord, np * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_twist, np * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_dl, np * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_cl, r->n_polar * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_cd, r->n_polar * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_pts, (size_t)npts * PT_STRIDE * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_ptf, (size_t)npts * 3 * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_loads, ALM_LOADS_LEN * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_Fbox, (size_t)nb * 3 * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_bcs, (size_t)r->n_blades * 2 * sizeof(double)) == hipSuccess;
            if (!ok) {
                free_rotor(R);
                return fail(c, LBM_ENOMEM, "rotor buffers");
            }
            std::vector<double> bcs(2 * (size_t)r->n_blades);
            for (int b = 0; b < r->n_blades; ++b) {
                const double phi = 2.0 * M_PI * b / r->n_blades;
                bcs[2 * b] = cos(phi);
                bcs[2 * b + 1] = sin(phi);
            }
            HIPCHK(c, hipMemcpy(R.d_bcs, bcs.data(), bcs.size() * sizeof(double), hipMemcpyHostToDevice));
            std::vector<float> cl(r->n_polar), cd(r->n_polar);
            for (int k = 0; k < r->n_polar; ++k) {
                cl[k] = (float)r->cl[k];
                cd[k] = (float)r->cd[k];
            }
            HIPCHK(c, hipMemcpy(R.d_r, r->r, np * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_chord, r->chord, np * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_twist, r->twist_deg, np * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_dl, r->dl, np * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_cl, cl.data(), r->n_polar * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_cd, cd.data(), r->n_polar * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemset(R.d_Fbox, 0, (size_t)nb * 3 * sizeof(float)));
            HIPCHK(c, hipMemset(R.d_loads, 0, ALM_LOADS_LEN * sizeof(double)));
            HIPCHK(c, hipMemset(R.d_ptf, 0, (size_t)npts * 3 * sizeof(double)));
            R.ptf_len = (size_t)npts * 3;
            RotorDev &D = R.dev;
            D = RotorDev{};
            for (int k = 0; k < 3; ++k) D.hub[k] = r->hub[k];
            D.omega_rot = r->omega_rot;
            D.azimuth0 = r->azimuth0;
            D.pitch_deg = r->pitch_deg;
            D.eps = r->eps;
            D.radius = r->radius;
            D.kernel = r->kernel;
            D.tip_loss = r->tip_loss;
            D.half = half;
            D.npts = npts;
            D.n_blades = r->n_blades;
            D.n_points = np;
            D.n_polar = r->n_polar;
            D.alpha0 = a0;
            D.dalpha = da;
            D.alpha0_f = (float)a0;
            D.inv_dalpha_f = (float)(1.0 / da);
            D.r = R.d_r;
            D.chord = R.d_chord;
            D.twist = R.d_twist;
            D.dl = R.d_dl;
            D.blade_cs = R.d_bcs;
            D.cl = R.d_cl;
            D.cd = R.d_cd;
            D.pts = R.d_pts;
            D.pt_force = R.d_ptf;
            D.loads = R.d_loads;
            D.box = ForceBox{bx0, by0, bz0, bx1 - bx0 + 1, by1 - by0 + 1, bz1 - bz0 + 1, R.d_Fbox};
            D.Fbox = R.d_Fbox;
            R.npts = npts;
            R.on = true;
            return LBM_OK;
        }();
        if (rc != LBM_OK) {
            free_rotor(R);
            (void)refresh_rotor_table(c);
            return rc;
        }
        return refresh_rotor_table(c);
    });
}

// ------------------------------------------------------------ turbine tree
namespace {

struct HostPose {
    double T[9], o[3];
};

void h_m3mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
void h_m3vec(const double *A, const double *x, double *y) {
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}
double h_norm(const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// Pose of every node in the reference configuration: each node's angle at
// angle0 and no oscillation (the centre of every oscillation).
void reference_poses(const lbm_turbine *tb, std::vector<HostPose> &P) {
    P.resize(tb->n_nodes);
    for (int k = 0; k < tb->n_nodes; ++k) {
        const lbm_node &N = tb->nodes[k];
        HostPose par{};
        par.T[0] = par.T[4] = par.T[8] = 1.0;
        if (N.parent >= 0) par = P[N.parent];
        const double ex[3] = {1.0, 0.0, 0.0};
        const bool turns = N.omega != 0.0 || N.amp != 0.0 || N.angle0 != 0.0;
        const double *a = turns ? N.axis : ex, th = N.angle0, ct = std::cos(th), st = std::sin(th), k1 = 1.0 - ct;
        const double R[9] = {ct + k1 * a[0] * a[0],        k1 * a[0] * a[1] - st * a[2], k1 * a[0] * a[2] + st * a[1],
                             k1 * a[1] * a[0] + st * a[2], ct + k1 * a[1] * a[1],        k1 * a[1] * a[2] - st * a[0],
                             k1 * a[2] * a[0] - st * a[1], k1 * a[2] * a[1] + st * a[0], ct + k1 * a[2] * a[2]};
        double TpTr[9], Tpr[3];
        h_m3mul(par.T, N.rot, TpTr);
        h_m3mul(TpTr, R, P[k].T);
        h_m3vec(par.T, N.pos, Tpr);
        for (int c = 0; c < 3; ++c) P[k].o[c] = par.o[c] + Tpr[c];
    }
}

// Interval [lo, hi] per axis that holds point q of node `node` at every time.
// A constant-rate rotation (the lowest one on the point's chain) sweeps a
// circle about its axis: exact bounding box of that circle, taken in the
// reference configuration. Every other motion on the chain moves the point
// by at most its angle excursion times the lever arm (2 lever arms for a full
// turn) plus the oscillation amplitude of the origin; lever arms bound
// |x - o_k| as |q| plus the lengths of the offsets below node k, which no
// rotation changes.
void point_reach(const lbm_turbine *tb, const std::vector<HostPose> &P, int node, const double q[3], double lo[3],
                 double hi[3]) {
    int chain[TREE_MAX_DEPTH], d = 0;
    for (int k = node; k >= 0 && d < TREE_MAX_DEPTH; k = tb->nodes[k].parent) chain[d++] = k;
    double xr[3], tq[3];
    h_m3vec(P[node].T, q, tq);
    for (int a = 0; a < 3; ++a) xr[a] = P[node].o[a] + tq[a];
    int circ = -1;
    for (int i = 0; i < d; ++i)
        if (tb->nodes[chain[i]].omega != 0.0) {
            circ = chain[i];
            break;
        }
    double cen[3] = {xr[0], xr[1], xr[2]}, ext[3] = {0, 0, 0};
    if (circ >= 0) {
        const lbm_node &N = tb->nodes[circ];
        HostPose par{};
        par.T[0] = par.T[4] = par.T[8] = 1.0;
        if (N.parent >= 0) par = P[N.parent];
        double TpTr[9], ah[3];
        h_m3mul(par.T, N.rot, TpTr);
        h_m3vec(TpTr, N.axis, ah);
        const double an = h_norm(ah);
        for (int a = 0; a < 3; ++a) ah[a] /= an;
        double rel[3];
        for (int a = 0; a < 3; ++a) rel[a] = xr[a] - P[circ].o[a];
        const double along = rel[0] * ah[0] + rel[1] * ah[1] + rel[2] * ah[2];
        double rad[3];
        for (int a = 0; a < 3; ++a) {
            cen[a] = P[circ].o[a] + along * ah[a];
            rad[a] = xr[a] - cen[a];
        }
        const double rho = h_norm(rad);
        for (int a = 0; a < 3; ++a) ext[a] = rho * std::sqrt(std::fmax(0.0, 1.0 - ah[a] * ah[a]));
    }
    double dev = 0.0, lever = h_norm(q);
    for (int i = 0; i < d; ++i) {
        const lbm_node &N = tb->nodes[chain[i]];
        if (chain[i] != circ) {
            if (N.omega != 0.0) dev += 2.0 * lever;
            else if (N.amp != 0.0) dev += std::fmin(std::fabs(N.amp), 2.0) * lever;
        }
        dev += h_norm(N.disp);
        lever += h_norm(N.pos) + h_norm(N.disp);
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = cen[a] - ext[a] - dev;
        hi[a] = cen[a] + ext[a] + dev;
    }
}

bool unit(const double *a) { return std::fabs(h_norm(a) - 1.0) < 1e-9; }

bool all_finite(const double *a, int n) {
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(a[k])) return false;
    return true;
}

}  // namespace

namespace {

// A validated turbine: its points in node order (disks: rings before
// azimuth), the node of each point, the polar grid and the spreading box
// (inclusive node range, not yet checked against a domain).
struct TurbineBuild {
    std::vector<TreePointDev> pts;
    std::vector<int> pt_node;
    bool any_blade = false;
    double a0 = 0.0, da = 1.0;
    int b0[3], b1[3];
};

// Argument checks, points and spreading box of a turbine; c may be null
// (then errors carry no message).
int build_turbine(lbm_ctx *c, const lbm_turbine *tb, TurbineBuild &out) {
    if (!tb || !tb->nodes) return fail(c, LBM_EINVAL, "null turbine");
    if (tb->n_nodes < 1 || tb->n_nodes > TREE_MAX_NODES)
        return fail(c, LBM_EINVAL, "n_nodes must be in [1, %d]", TREE_MAX_NODES);
    if (tb->kernel != LBM_KERNEL_GAUSS && tb->kernel != LBM_KERNEL_ROMA3)
        return fail(c, LBM_EINVAL, "unknown spreading kernel %d", tb->kernel);
    if (tb->kernel == LBM_KERNEL_GAUSS && !(tb->eps > 0.0 && std::isfinite(tb->eps)))
        return fail(c, LBM_EINVAL, "eps must be positive");
    if (!std::isfinite(tb->radius)) return fail(c, LBM_EINVAL, "non-finite radius");
    int npts = 0;
    for (int k = 0; k < tb->n_nodes; ++k) {
        const lbm_node &N = tb->nodes[k];
        if (N.parent < -1 || N.parent >= k) return fail(c, LBM_EINVAL, "node %d: parent must precede it", k);
        const double motion[9] = {N.omega, N.angle0, N.amp, N.freq, N.phase, N.coef, N.pitch_deg, 0.0, 0.0};
        if (!all_finite(N.pos, 3) || !all_finite(N.rot, 9) || !all_finite(N.axis, 3) || !all_finite(N.disp, 3) ||
            !all_finite(N.dir, 3) || !all_finite(N.normal, 3) || !all_finite(motion, 9))
            return fail(c, LBM_EINVAL, "node %d: non-finite value", k);
        int depth = 1;
        for (int q = N.parent; q >= 0; q = tb->nodes[q].parent) ++depth;
        if (depth > TREE_MAX_DEPTH) return fail(c, LBM_EINVAL, "node %d: tree deeper than %d", k, TREE_MAX_DEPTH);
        if (N.kind != LBM_NODE_FRAME && N.kind != LBM_NODE_LINE && N.kind != LBM_NODE_DISK)
            return fail(c, LBM_EINVAL, "node %d: unknown kind %d", k, N.kind);
        if (N.force != LBM_FORCE_NONE && N.force != LBM_FORCE_BLADE && N.force != LBM_FORCE_DRAG)
            return fail(c, LBM_EINVAL, "node %d: unknown force model %d", k, N.force);
        double RRt[9], Rt[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Rt[3 * i + j] = N.rot[3 * j + i];
        h_m3mul(N.rot, Rt, RRt);
        for (int i = 0; i < 9; ++i)
            if (std::fabs(RRt[i] - (i % 4 == 0 ? 1.0 : 0.0)) > 1e-9)
                return fail(c, LBM_EINVAL, "node %d: rot is not orthonormal", k);
        const double det = N.rot[0] * (N.rot[4] * N.rot[8] - N.rot[5] * N.rot[7]) -
                           N.rot[1] * (N.rot[3] * N.rot[8] - N.rot[5] * N.rot[6]) +
                           N.rot[2] * (N.rot[3] * N.rot[7] - N.rot[4] * N.rot[6]);
        if (!(det > 0.0)) return fail(c, LBM_EINVAL, "node %d: rot must have determinant +1", k);
        const bool turns = N.omega != 0.0 || N.amp != 0.0 || N.angle0 != 0.0;
        if (turns && !unit(N.axis)) return fail(c, LBM_EINVAL, "node %d: axis must be a unit vector", k);
        if (N.kind == LBM_NODE_FRAME) {
            if (N.force != LBM_FORCE_NONE) return fail(c, LBM_EINVAL, "node %d: a frame carries no force model", k);
            continue;
        }
        if (N.n_points < 1 || !N.s || !N.width) return fail(c, LBM_EINVAL, "node %d: needs n_points, s, width", k);
        if (!all_finite(N.s, N.n_points) || !all_finite(N.width, N.n_points) || (N.chord && !all_finite(N.chord, N.n_points)) ||
            (N.twist && !all_finite(N.twist, N.n_points)))
            return fail(c, LBM_EINVAL, "node %d: non-finite point data", k);
        if (N.kind == LBM_NODE_DISK && N.n_azimuth < 1) return fail(c, LBM_EINVAL, "node %d: n_azimuth < 1", k);
        if (N.kind == LBM_NODE_LINE && !unit(N.dir)) return fail(c, LBM_EINVAL, "node %d: dir must be a unit vector", k);
        if (N.force == LBM_FORCE_BLADE) {
            if (N.kind != LBM_NODE_LINE || !N.chord || !N.twist)
                return fail(c, LBM_EINVAL, "node %d: blade elements need a line with chord and twist", k);
            const double nd = N.normal[0] * N.dir[0] + N.normal[1] * N.dir[1] + N.normal[2] * N.dir[2];
            if (!unit(N.normal) || std::fabs(nd) > 1e-9)
                return fail(c, LBM_EINVAL, "node %d: normal must be a unit vector normal to dir", k);
            if (N.tip_loss != 0 && N.tip_loss != 1) return fail(c, LBM_EINVAL, "node %d: tip_loss must be 0 or 1", k);
            if (N.tip_loss && (tb->n_blades < 1 || !(tb->radius > 0.0)))
                return fail(c, LBM_EINVAL, "node %d: tip loss needs n_blades and radius", k);
            for (int m = 0; m < N.n_points; ++m)
                if (!(std::fabs(N.twist[m] + N.pitch_deg) < 180.0))
                    return fail(c, LBM_EINVAL, "node %d: |twist + pitch| must stay below 180 degrees", k);
            out.any_blade = true;
        }
        if (N.force == LBM_FORCE_DRAG && N.kind == LBM_NODE_LINE && !N.chord)
            return fail(c, LBM_EINVAL, "node %d: line drag needs the diameters (chord)", k);
        const long np = N.kind == LBM_NODE_LINE ? (long)N.n_points : (long)N.n_points * N.n_azimuth;
        if (npts + np > ALM_MAX_POINTS) return fail(c, LBM_EINVAL, "more than %d points", ALM_MAX_POINTS);
        npts += (int)np;
    }
    if (npts < 1) return fail(c, LBM_EINVAL, "a turbine needs at least one point");
    if (out.any_blade) {
        if (tb->n_polar < 2 || !tb->alpha_deg || !tb->cl || !tb->cd) return fail(c, LBM_EINVAL, "missing polars");
        if (!all_finite(tb->alpha_deg, tb->n_polar) || !all_finite(tb->cl, tb->n_polar) || !all_finite(tb->cd, tb->n_polar))
            return fail(c, LBM_EINVAL, "non-finite polar value");
        out.a0 = tb->alpha_deg[0];
        out.da = (tb->alpha_deg[tb->n_polar - 1] - out.a0) / (tb->n_polar - 1);
        if (!(out.da > 0.0)) return fail(c, LBM_EINVAL, "polar angles must ascend");
        for (int k = 0; k < tb->n_polar; ++k)
            if (std::fabs(tb->alpha_deg[k] - (out.a0 + k * out.da)) > 1e-9 * (1.0 + std::fabs(out.a0)))
                return fail(c, LBM_EINVAL, "polar angle grid must be uniform");
    }
    // points in node order (disks: rings before azimuth), element data
    std::vector<TreePointDev> &pts = out.pts;
    std::vector<int> &pt_node = out.pt_node;
    for (int k = 0; k < tb->n_nodes; ++k) {
        const lbm_node &N = tb->nodes[k];
        if (N.kind == LBM_NODE_LINE) {
            for (int m = 0; m < N.n_points; ++m) {
                TreePointDev p{};
                p.node = k;
                for (int a = 0; a < 3; ++a) p.q[a] = N.s[m] * N.dir[a];
                p.s = N.s[m];
                p.measure = N.width[m];
                p.chord = N.chord ? N.chord[m] : 0.0;
                p.twist = N.twist ? N.twist[m] : 0.0;
                pts.push_back(p);
                pt_node.push_back(k);
            }
        } else if (N.kind == LBM_NODE_DISK) {
            for (int j = 0; j < N.n_points; ++j)
                for (int m = 0; m < N.n_azimuth; ++m) {
                    const double phi = 2.0 * 3.14159265358979323846 * m / N.n_azimuth;
                    TreePointDev p{};
                    p.node = k;
                    p.q[1] = N.s[j] * std::cos(phi);
                    p.q[2] = N.s[j] * std::sin(phi);
                    p.s = N.s[j];
                    p.measure = 2.0 * 3.14159265358979323846 * N.s[j] * N.width[j] / N.n_azimuth;
                    pts.push_back(p);
                    pt_node.push_back(k);
                }
        }
    }
    // spreading box: the support of every point over all times
    const int half = tb->kernel == LBM_KERNEL_ROMA3 ? 1 : SUPPORT;
    std::vector<HostPose> ref;
    reference_poses(tb, ref);
    int *b0 = out.b0, *b1 = out.b1;
    for (int a = 0; a < 3; ++a) {
        b0[a] = 1 << 30;
        b1[a] = -(1 << 30);
    }
    for (const TreePointDev &p : pts) {
        double lo[3], hi[3];
        point_reach(tb, ref, p.node, p.q, lo, hi);
        for (int a = 0; a < 3; ++a) {
            // nearest node of any position in [lo, hi], with room for rounding
            b0[a] = std::min(b0[a], (int)std::floor(lo[a] + 0.5 - 1e-9) - half);
            b1[a] = std::max(b1[a], (int)std::floor(hi[a] + 0.5 + 1e-9) + half);
        }
    }
    return LBM_OK;
}

}  // namespace

int lbm_set_turbine(lbm_ctx *c, int id, const lbm_turbine *tb) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        if (id < 0 || id >= MAX_ROTORS || !tb || !tb->nodes) return fail(c, LBM_EINVAL, "bad turbine id or null turbine");
        TurbineBuild tbd;
        {
            const int rc = build_turbine(c, tb, tbd);
            if (rc != LBM_OK) return rc;
        }
        const std::vector<TreePointDev> &pts = tbd.pts;
        const bool any_blade = tbd.any_blade;
        const double a0 = tbd.a0, da = tbd.da;
        const int npts = (int)pts.size();
        const int half = tb->kernel == LBM_KERNEL_ROMA3 ? 1 : SUPPORT;
        const int *b0 = tbd.b0, *b1 = tbd.b1;
        const int dims[3] = {c->cfg.nx, c->cfg.ny, c->cfg.nz};
        for (int a = 0; a < 3; ++a)
            if (b0[a] < 0 || b1[a] >= dims[a])
                return fail(c, LBM_EINVAL, "turbine spreading box [%d,%d]x[%d,%d]x[%d,%d] leaves the domain", b0[0], b1[0],
                            b0[1], b1[1], b0[2], b1[2]);
        std::vector<NodeDev> nodes(tb->n_nodes);
        for (int k = 0; k < tb->n_nodes; ++k) {
            const lbm_node &N = tb->nodes[k];
            NodeDev &D = nodes[k];
            D = NodeDev{};
            D.parent = N.parent;
            D.kind = N.kind;
            D.force = N.force;
            D.tip_loss = N.tip_loss;
            // a node that never turns gets the rotation about +x by 0 (identity)
            const bool turns = N.omega != 0.0 || N.amp != 0.0 || N.angle0 != 0.0;
            for (int a = 0; a < 3; ++a) {
                D.pos[a] = N.pos[a];
                D.axis[a] = turns ? N.axis[a] : (a == 0 ? 1.0 : 0.0);
                D.disp[a] = N.disp[a];
                D.dir[a] = N.dir[a];
                D.normal[a] = N.normal[a];
            }
            for (int a = 0; a < 9; ++a) D.rot[a] = N.rot[a];
            D.omega = N.omega;
            D.angle0 = N.angle0;
            D.amp = N.amp;
            D.freq = N.freq;
            D.phase = N.phase;
            D.coef = N.coef;
            D.pitch_deg = N.pitch_deg;
        }
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        RotorHost &R = c->rot[id];
        free_rotor(R);
        // on any failure below the slot ends up empty, and the rotor table
        // must stop naming the freed buffers
        const int rc = [&]() -> int {
            const int np_pol = any_blade ? tb->n_polar : 2;
            const size_t nb = (size_t)(b1[0] - b0[0] + 1) * (b1[1] - b0[1] + 1) * (b1[2] - b0[2] + 1);
            R.ptf_len = (size_t)npts * TREE_PT_OUT;
            bool ok = hipMalloc((void **)&R.d_cl, np_pol * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_cd, np_pol * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_pts, (size_t)npts * PT_STRIDE * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_ptf, R.ptf_len * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_loads, ALM_LOADS_LEN * sizeof(double)) == hipSuccess &&
                      hipMalloc((void **)&R.d_Fbox, nb * 3 * sizeof(float)) == hipSuccess &&
                      hipMalloc((void **)&R.d_nodes, nodes.size() * sizeof(NodeDev)) == hipSuccess &&
                      hipMalloc((void **)&R.d_tpts, pts.size() * sizeof(TreePointDev)) == hipSuccess;
            if (!ok) {
                free_rotor(R);
                return fail(c, LBM_ENOMEM, "turbine buffers");
            }
            std::vector<float> cl(np_pol, 0.0f), cd(np_pol, 0.0f);
            if (any_blade)
                for (int k = 0; k < np_pol; ++k) {
                    cl[k] = (float)tb->cl[k];
                    cd[k] = (float)tb->cd[k];
                }
            HIPCHK(c, hipMemcpy(R.d_cl, cl.data(), np_pol * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_cd, cd.data(), np_pol * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_nodes, nodes.data(), nodes.size() * sizeof(NodeDev), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(R.d_tpts, pts.data(), pts.size() * sizeof(TreePointDev), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemset(R.d_Fbox, 0, nb * 3 * sizeof(float)));
            HIPCHK(c, hipMemset(R.d_loads, 0, ALM_LOADS_LEN * sizeof(double)));
            HIPCHK(c, hipMemset(R.d_ptf, 0, R.ptf_len * sizeof(double)));
            RotorDev &D = R.dev;
            D = RotorDev{};
            D.eps = tb->eps;
            D.radius = tb->radius;
            D.kernel = tb->kernel;
            D.half = half;
            D.npts = npts;
            D.n_blades = tb->n_blades;
            D.n_points = 1;
            D.n_polar = np_pol;
            D.alpha0 = a0;
            D.dalpha = da;
            D.alpha0_f = (float)a0;
            D.inv_dalpha_f = (float)(1.0 / da);
            D.cl = R.d_cl;
            D.cd = R.d_cd;
            D.nodes = R.d_nodes;
            D.n_nodes = tb->n_nodes;
            D.tpts = R.d_tpts;
            D.pts = R.d_pts;
            D.pt_force = R.d_ptf;
            D.loads = R.d_loads;
            D.box = ForceBox{b0[0], b0[1], b0[2], b1[0] - b0[0] + 1, b1[1] - b0[1] + 1, b1[2] - b0[2] + 1, R.d_Fbox};
            D.Fbox = R.d_Fbox;
            R.npts = npts;
            R.n_nodes = tb->n_nodes;
            R.pt_node = tbd.pt_node;
            R.on = true;
            return LBM_OK;
        }();
        if (rc != LBM_OK) {
            free_rotor(R);
            (void)refresh_rotor_table(c);
            return rc;
        }
        return refresh_rotor_table(c);
    });
}

int lbm_turbine_box(const lbm_turbine *tb, int lo[3], int hi[3]) {
    return guard(nullptr, [&]() -> int {
        if (!lo || !hi) return LBM_EINVAL;
        TurbineBuild tbd;
        const int rc = build_turbine(nullptr, tb, tbd);
        if (rc != LBM_OK) return rc;
        for (int a = 0; a < 3; ++a) {
            lo[a] = tbd.b0[a];
            hi[a] = tbd.b1[a];
        }
        return LBM_OK;
    });
}

int lbm_turbine_points(const lbm_ctx *c, int id, int *n_points_total) {
    return guard(c, [&]() -> int {
        if (!c || id < 0 || id >= MAX_ROTORS || !n_points_total) return LBM_EINVAL;
        const RotorHost &R = c->rot[id];
        if (!R.on || !R.d_nodes) return LBM_EINVAL;
        *n_points_total = R.npts;
        return LBM_OK;
    });
}

int lbm_turbine_loads(lbm_ctx *c, int id, double *node_loads, double *pts) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (id < 0 || id >= MAX_ROTORS || !node_loads) return fail(c, LBM_EINVAL, "bad turbine id or null output");
        RotorHost &R = c->rot[id];
        if (!R.on || !R.d_nodes) return fail(c, LBM_EINVAL, "slot %d holds no turbine tree", id);
        std::vector<double> o(R.ptf_len);
        HIPCHK(c, hipMemcpyAsync(o.data(), R.d_ptf, R.ptf_len * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        // per node, in point order: force, moment about the node origin, power
        for (int k = 0; k < 7 * R.n_nodes; ++k) node_loads[k] = 0.0;
        for (int p = 0; p < R.npts; ++p) {
            const double *q = o.data() + (size_t)TREE_PT_OUT * p;
            double *L = node_loads + 7 * R.pt_node[p];
            for (int a = 0; a < 3; ++a) {
                L[a] += q[6 + a];
                L[3 + a] += q[9 + a];
            }
            L[6] += q[6] * q[3] + q[7] * q[4] + q[8] * q[5];
            if (pts)
                for (int a = 0; a < 9; ++a) pts[9 * (size_t)p + a] = q[a];
        }
        return LBM_OK;
    });
}

// inlet planes of the current and the previous step
static int refresh_inflow_planes(lbm_ctx *c) {
    if (!c->d_in_mean) return LBM_OK;
    const int plane = c->cfg.ny * c->cfg.nz, lt = c->in_lt > 0 ? c->in_lt : 1;
    const long ts[2] = {c->t, c->t > 0 ? c->t - 1 : c->t};
    for (long t : ts)
        if (launch_inflow(uin_plane(c, t), c->d_in_mean, c->d_in_box, lt, plane, c->in_advect * (double)t, c->stream))
            return fail(c, LBM_EHIP, "inflow launch");
    if (c->t == 0 &&
        launch_inflow(uin_plane(c, 1), c->d_in_mean, c->d_in_box, lt, plane, 0.0, c->stream))
        return fail(c, LBM_EHIP, "inflow launch");
    return LBM_OK;
}

int lbm_set_inflow(lbm_ctx *c, const double *mean, const double *box, int lt, double advect) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (c->cfg.bc_x != LBM_BC_INFLOW_OUTFLOW) return fail(c, LBM_EINVAL, "the x boundary is not inflow/outflow");
        if (!mean || (box && lt < 1) || !std::isfinite(advect)) return fail(c, LBM_EINVAL, "bad inflow arguments");
        (void)hipStreamSynchronize(c->stream);
        const size_t plane = (size_t)c->cfg.ny * c->cfg.nz;
        if (c->d_in_mean) (void)hipFree(c->d_in_mean);
        if (c->d_in_box) (void)hipFree(c->d_in_box);
        c->d_in_mean = c->d_in_box = nullptr;
        c->in_lt = 0;
        std::vector<float> tmp(3 * plane);
        for (size_t k = 0; k < 3 * plane; ++k) tmp[k] = (float)mean[k];
        if (hipMalloc((void **)&c->d_in_mean, 3 * plane * sizeof(float)) != hipSuccess) {
            c->d_in_mean = nullptr;
            return fail(c, LBM_ENOMEM, "inflow mean plane");
        }
        HIPCHK(c, hipMemcpy(c->d_in_mean, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice));
        if (box) {
            const size_t nb = 3 * (size_t)lt * plane;
            std::vector<float> tb(nb);
            for (size_t k = 0; k < nb; ++k) tb[k] = (float)box[k];
            if (hipMalloc((void **)&c->d_in_box, nb * sizeof(float)) != hipSuccess) {
                c->d_in_box = nullptr;
                return fail(c, LBM_ENOMEM, "inflow turbulence box");
            }
            HIPCHK(c, hipMemcpy(c->d_in_box, tb.data(), nb * sizeof(float), hipMemcpyHostToDevice));
            c->in_lt = lt;
        }
        c->in_advect = advect;
        if ((rc = refresh_inflow_planes(c))) return rc;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_step(lbm_ctx *c, int nsteps) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (nsteps < 0) return fail(c, LBM_EINVAL, "negative step count");
        if (c->cfg.closure == LBM_CLOSURE_MLP && !c->mlp_set) return fail(c, LBM_ESTATE, "closure weights not set");
        const int st = (int)c->cfg.storage;
        const int mode = sc_mode(c);
        int *flag = (int *)((char *)c->aux + c->off_flag);
        double *part = (double *)((char *)c->aux + c->off_part);
        // relative mass drift that counts as a failure: well above the drift that
        // rounding of the stored populations produces over long runs
        const double tol = c->cfg.storage == LBM_F32 ? 1e-6 : (c->cfg.storage == LBM_F16 ? 1e-5 : 1e-4);
        if (c->cfg.check_every > 0 && !c->mass0_set) {
            double m[RED_NMOM];
            if ((rc = moments_now(c, m))) return rc;
            c->mass0 = m[0];
            c->mass0_set = true;
            HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
        }
        Geo g = geo_of(c);
        const int nrot = (int)c->h_rots.size();
        for (int s = 0; s < nsteps; ++s) {
            Physics ph = physics_of(c);
            ph.sr_seed = mix32((uint32_t)c->t * SR_WEYL + 0x632be5abu);
            const bool frc = has_force(c);
            if (c->d_in_mean &&
                launch_inflow(uin_plane(c, c->t), c->d_in_mean, c->d_in_box, c->in_lt > 0 ? c->in_lt : 1,
                              c->cfg.ny * c->cfg.nz, c->in_advect * (double)c->t, c->stream))
                return fail(c, LBM_EHIP, "inflow launch failed");
            g = geo_of(c);
            const int sr = c->cfg.rounding == LBM_ROUND_STOCHASTIC;
            if (nrot > 0 && launch_alm(st, c->parity, g, ph, c->h_rots.data(), nrot, c->t, c->stream))
                return fail(c, LBM_EHIP, "actuator-line launch failed");
            if (launch_stream_collide(st, sr, c->parity, (int)c->cfg.closure, mode, frc, c->general_rates, g, ph,
                                      c->stream))
                return fail(c, LBM_EHIP, "stream-collide launch failed");
            c->parity ^= 1;
            c->t += 1;
            if (c->cfg.check_every > 0 && (c->t % c->cfg.check_every == 0 || s == nsteps - 1)) {
                // an open (inflow/outflow) domain does not conserve mass: validity only
                const double mtol = c->cfg.bc_x == LBM_BC_PERIODIC ? tol : 1e300;
                if (launch_check(st, c->parity, geo_of(c), ph, part, RED_NBLOCKS, c->mass0, mtol, flag, c->stream))
                    return fail(c, LBM_EHIP, "check launch failed");
            }
        }
        if (c->cfg.check_every > 0) {
            int h = 0;
            HIPCHK(c, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (h) return fail(c, LBM_EUNSTABLE, "mass drift above %g, or a cell with NaN, rho <= 0 or |u| > 1", tol);
        }
        return LBM_OK;
    });
}

int lbm_get_fields(lbm_ctx *c, double *rho, double *u) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!rho || !u) return fail(c, LBM_EINVAL, "null output");
        const size_t ch = chunk_cells(c);
        if ((rc = ensure_stage(c, 4 * ch * sizeof(double)))) return rc;
        Geo g = geo_of(c);
        Physics ph = physics_of(c);
        for (size_t c0 = 0; c0 < c->n; c0 += ch) {
            const size_t m = c->n - c0 < ch ? c->n - c0 : ch;
            if (launch_fields((int)c->cfg.storage, c->parity, g, ph, c->d_stage, c->d_stage + m, c0, m, c->stream))
                return fail(c, LBM_EHIP, "field launch");
            HIPCHK(c, hipMemcpyAsync(rho + c0, c->d_stage, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            for (int d = 0; d < 3; ++d)
                HIPCHK(c, hipMemcpyAsync(u + d * c->n + c0, c->d_stage + m * (1 + d), m * sizeof(double),
                                         hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        return LBM_OK;
    });
}

int lbm_get_filtered(lbm_ctx *c, int w, double *out) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!out || w < 1 || c->cfg.nx % w || c->cfg.ny % w || c->cfg.nz % w)
            return fail(c, LBM_EINVAL, "filter width must divide nx, ny and nz");
        const size_t nc = c->n / ((size_t)w * w * w);
        const size_t ch = nc < ((size_t)1 << 20) ? nc : ((size_t)1 << 20);
        if ((rc = ensure_stage(c, 10 * ch * sizeof(double)))) return rc;
        Geo g = geo_of(c);
        Physics ph = physics_of(c);
        for (size_t c0 = 0; c0 < nc; c0 += ch) {
            const size_t m = nc - c0 < ch ? nc - c0 : ch;
            if (launch_filtered((int)c->cfg.storage, c->parity, g, ph, w, c->d_stage, c0, m, c->stream))
                return fail(c, LBM_EHIP, "filter launch");
            for (int k = 0; k < 10; ++k)
                HIPCHK(c, hipMemcpyAsync(out + (size_t)k * nc + c0, c->d_stage + (size_t)k * m, m * sizeof(double),
                                         hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        return LBM_OK;
    });
}

int lbm_get_pops(lbm_ctx *c, double *f) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!f) return fail(c, LBM_EINVAL, "null output");
        const size_t ch = chunk_cells(c) / 8 > 0 ? chunk_cells(c) / 8 : 1;
        if ((rc = ensure_stage(c, 27 * ch * sizeof(double)))) return rc;
        Geo g = geo_of(c);
        for (size_t c0 = 0; c0 < c->n; c0 += ch) {
            const size_t m = c->n - c0 < ch ? c->n - c0 : ch;
            if (launch_pops((int)c->cfg.storage, c->parity, g, c->d_stage, c0, m, c->stream))
                return fail(c, LBM_EHIP, "population launch");
            for (int i = 0; i < 27; ++i)
                HIPCHK(c, hipMemcpyAsync(f + (size_t)i * c->n + c0, c->d_stage + (size_t)i * m, m * sizeof(double),
                                         hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        return LBM_OK;
    });
}

int lbm_sample_pops(lbm_ctx *c, const size_t *cells, size_t m, double *f) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!cells || !f) return fail(c, LBM_EINVAL, "null argument");
        if (m == 0) return LBM_OK;
        for (size_t k = 0; k < m; ++k)
            if (cells[k] >= c->n) return fail(c, LBM_EINVAL, "cell index %zu out of range", cells[k]);
        const size_t bytes = m * sizeof(size_t) + 27 * m * sizeof(double);
        if ((rc = ensure_stage(c, round_up(bytes, 256)))) return rc;
        double *d_f = c->d_stage;
        size_t *d_cells = (size_t *)(c->d_stage + 27 * m);
        HIPCHK(c, hipMemcpyAsync(d_cells, cells, m * sizeof(size_t), hipMemcpyHostToDevice, c->stream));
        if (launch_sample_pops((int)c->cfg.storage, c->parity, geo_of(c), d_cells, m, d_f, c->stream))
            return fail(c, LBM_EHIP, "sample launch");
        HIPCHK(c, hipMemcpyAsync(f, d_f, 27 * m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_rotor_loads(lbm_ctx *c, int id, double out[3], double *pt_force) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (id < 0 || id >= MAX_ROTORS || !out) return fail(c, LBM_EINVAL, "bad rotor id or null output");
        RotorHost &R = c->rot[id];
        if (!R.on) return fail(c, LBM_EINVAL, "rotor %d not set", id);
        if (R.d_nodes) return fail(c, LBM_EINVAL, "slot %d holds a turbine tree: use lbm_turbine_loads", id);
        // the step leaves FP64 partial thrust and torque per batch of 32 points;
        // they are added here in batch order (deterministic, no extra kernel on
        // the step's critical path)
        double part[ALM_LOADS_LEN];
        HIPCHK(c, hipMemcpyAsync(part, R.d_loads, sizeof(part), hipMemcpyDeviceToHost, c->stream));
        if (pt_force)
            HIPCHK(c, hipMemcpyAsync(pt_force, R.d_ptf, 3 * (size_t)R.npts * sizeof(double), hipMemcpyDeviceToHost,
                                     c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int nb = (R.npts + ALM_BATCH_PTS - 1) / ALM_BATCH_PTS;
        double T = 0.0, Q = 0.0;
        for (int b = 0; b < nb; ++b) {
            T += part[3 + 2 * b];
            Q += part[4 + 2 * b];
        }
        out[0] = T;
        out[1] = Q;
        out[2] = Q * R.dev.omega_rot;
        return LBM_OK;
    });
}

int lbm_pattern_probe(lbm_ctx *c, int parity) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (parity != 0 && parity != 1) return fail(c, LBM_EINVAL, "parity must be 0 or 1");
        if (!fast_offsets_fit(c)) return fail(c, LBM_EINVAL, "probe needs 32-bit offsets within a z plane");
        if (launch_pattern_probe((int)c->cfg.storage, parity, geo_of(c), c->stream))
            return fail(c, LBM_EHIP, "probe launch failed");
        return LBM_OK;
    });
}

int lbm_global_moments(lbm_ctx *c, double *mass, double mom[3], double *ke) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        if (!mass || !mom || !ke) return fail(c, LBM_EINVAL, "null output");
        double m[RED_NMOM];
        if ((rc = moments_now(c, m))) return rc;
        *mass = m[0];
        mom[0] = m[1];
        mom[1] = m[2];
        mom[2] = m[3];
        *ke = m[4];
        return LBM_OK;
    });
}

int lbm_time(const lbm_ctx *c, long *t) {
    return guard(c, [&]() -> int {
        if (!c || !t) return LBM_EINVAL;
        *t = c->t;
        return LBM_OK;
    });
}

int lbm_set_force_field(lbm_ctx *c, const double *F) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        if (!F) {
            if (c->d_ffield) (void)hipFree(c->d_ffield);
            c->d_ffield = nullptr;
            return LBM_OK;
        }
        if (!c->d_ffield && hipMalloc((void **)&c->d_ffield, 3 * c->n * sizeof(float)) != hipSuccess) {
            c->d_ffield = nullptr;
            return fail(c, LBM_ENOMEM, "force field");
        }
        std::vector<float> tmp(3 * c->n);
        for (size_t k = 0; k < 3 * c->n; ++k) tmp[k] = (float)F[k];
        HIPCHK(c, hipMemcpy(c->d_ffield, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice));
        return LBM_OK;
    });
}

int lbm_set_closure_weights(lbm_ctx *c, const float *w, size_t n) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        if (!w || n != (size_t)MLP_NBLOB) return fail(c, LBM_EINVAL, "expected %d closure parameters", MLP_NBLOB);
        for (int j = 0; j < 6; ++j)
            if (!(w[MLP_NPARAM + 6 + j] > 0.0f)) return fail(c, LBM_EINVAL, "sigma must be positive");
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        if (!c->d_mlp && hipMalloc((void **)&c->d_mlp, sizeof(MlpDev)) != hipSuccess) {
            c->d_mlp = nullptr;
            return fail(c, LBM_ENOMEM, "closure weights");
        }
        MlpDev h;
        mlp_pack(w, &h);
        HIPCHK(c, hipMemcpy(c->d_mlp, &h, sizeof h, hipMemcpyHostToDevice));
        c->mlp_set = true;
        return LBM_OK;
    });
}

// checkpoint header: magic, time, parity, storage, force-box bytes, nx, ny, nz
constexpr long STATE_MAGIC = 0x4c424d34L;  // blocked population layout, 32-cell FP32 blocks

// bytes of the force boxes of the active rotor / turbine slots (slot order)
static size_t box_state_bytes(const lbm_ctx *c) {
    size_t n = 0;
    for (int r = 0; r < MAX_ROTORS; ++r)
        if (c->rot[r].on) {
            const ForceBox &B = c->rot[r].dev.box;
            n += (size_t)3 * B.bnx * B.bny * B.bnz * sizeof(float);
        }
    return n;
}

int lbm_state_bytes(const lbm_ctx *c, size_t *bytes) {
    return guard(c, [&]() -> int {
        if (!c || !bytes) return LBM_EINVAL;
        *bytes = 64 + c->pop_bytes + c->off_uin + box_state_bytes(c);
        return LBM_OK;
    });
}

int lbm_get_state(lbm_ctx *c, void *buf, size_t bytes) {
    return guard(c, [&]() -> int {
        int rc = ready(c);
        if (rc) return rc;
        size_t need;
        lbm_state_bytes(c, &need);
        if (!buf || bytes < need) return fail(c, LBM_EINVAL, "state buffer needs %zu bytes", need);
        char *b = (char *)buf;
        memset(b, 0, 64);
        const long hdr[8] = {STATE_MAGIC,      c->t,         c->parity,    (long)c->cfg.storage,
                             (long)box_state_bytes(c), (long)c->cfg.nx, (long)c->cfg.ny, (long)c->cfg.nz};
        memcpy(b, hdr, sizeof hdr);
        HIPCHK(c, hipMemcpyAsync(b + 64, c->pops, c->pop_bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(b + 64 + c->pop_bytes, (char *)c->aux + c->off_ghost, c->off_uin, hipMemcpyDeviceToHost,
                                 c->stream));
        // the spread force of the last step: the next step samples u with half of it
        size_t off = 64 + c->pop_bytes + c->off_uin;
        for (int r = 0; r < MAX_ROTORS; ++r)
            if (c->rot[r].on) {
                const ForceBox &B = c->rot[r].dev.box;
                const size_t nbytes = (size_t)3 * B.bnx * B.bny * B.bnz * sizeof(float);
                HIPCHK(c, hipMemcpyAsync(b + off, c->rot[r].d_Fbox, nbytes, hipMemcpyDeviceToHost, c->stream));
                off += nbytes;
            }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_set_state(lbm_ctx *c, const void *buf, size_t bytes) {
    return guard(c, [&]() -> int {
        if (!c) return LBM_EINVAL;
        // the buffer and its header are checked before any device work
        size_t need;
        lbm_state_bytes(c, &need);
        if (!buf || bytes < need) return fail(c, LBM_EINVAL, "state buffer needs %zu bytes", need);
        const char *b = (const char *)buf;
        long hdr[8];
        memcpy(hdr, b, sizeof hdr);
        if (hdr[0] != STATE_MAGIC || (hdr[2] != 0 && hdr[2] != 1))
            return fail(c, LBM_EINVAL, "not a state written by lbm_get_state");
        if (hdr[3] != (long)c->cfg.storage)
            return fail(c, LBM_EINVAL, "state has storage type %ld, this context %d", hdr[3], c->cfg.storage);
        if (hdr[5] != c->cfg.nx || hdr[6] != c->cfg.ny || hdr[7] != c->cfg.nz)
            return fail(c, LBM_EINVAL, "state of a %ldx%ldx%ld grid, this context is %dx%dx%d", hdr[5], hdr[6], hdr[7],
                        c->cfg.nx, c->cfg.ny, c->cfg.nz);
        if (hdr[4] != (long)box_state_bytes(c))
            return fail(c, LBM_EINVAL, "state holds %ld bytes of rotor force boxes, this context's slots %zu: set the "
                                       "same rotors and turbines before restoring", hdr[4], box_state_bytes(c));
        int rc = ready(c);
        if (rc) return rc;
        HIPCHK(c, hipMemcpyAsync(c->pops, b + 64, c->pop_bytes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync((char *)c->aux + c->off_ghost, b + 64 + c->pop_bytes, c->off_uin, hipMemcpyHostToDevice,
                                 c->stream));
        size_t off = 64 + c->pop_bytes + c->off_uin;
        for (int r = 0; r < MAX_ROTORS; ++r)
            if (c->rot[r].on) {
                const ForceBox &B = c->rot[r].dev.box;
                const size_t nbytes = (size_t)3 * B.bnx * B.bny * B.bnz * sizeof(float);
                HIPCHK(c, hipMemcpyAsync(c->rot[r].d_Fbox, b + off, nbytes, hipMemcpyHostToDevice, c->stream));
                off += nbytes;
            }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->t = hdr[1];
        c->parity = (int)hdr[2];
        c->mass0_set = false;
        int rc2 = refresh_inflow_planes(c);
        if (rc2) return rc2;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

}  // extern "C"
