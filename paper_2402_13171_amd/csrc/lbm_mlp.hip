// Learned eddy-viscosity closure: batched inference, loss and gradient, and
// the Adam update, all on the device (the lattice kernel evaluates the same
// network in place through lbm_mlp_dev.h).
//
// Training step on a batch of B cells (features x, scaled targets y):
//   forward   : matrix-core layers as in inference, keeping pre-activations;
//   loss      : L = (1/B) sum_b (softplus(z_b) - y_b)^2;
//   backward  : dz = 2 (softplus(z) - y) sigmoid(z) / B;
//               da2 = dz w3 [a2 > 0];
//               dh1 = W2^T da2 on the matrix cores (da2 rounded to bf16);
//               da1 = dh1 [a1 > 0];
//               weight and bias gradients as FP32 sums over the wave's 64
//               cells (vector ALU, from LDS), then a fixed-order sum over
//               waves (deterministic);
//   Adam      : FP32 master weights (Kingma and Ba 2015), refreshed bf16
//               copies for the matrix cores.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_mlp_dev.h"

namespace lbm {

// blob offsets (W1[32][6] b1 W2[32][32] b2 w3 b3 mu[6] sigma[6] nu_scale)
constexpr int O_W1 = 0, O_B1 = 192, O_W2 = 224, O_B2 = 1248, O_W3 = 1280, O_B3 = 1312;
constexpr int O_MU = 1313, O_SG = 1319, O_NS = 1325;

static uint16_t host_bf16(float v) {
    uint32_t b;
    std::memcpy(&b, &v, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)(b >> 16) | ((b & 0xffffu) ? 0x40u : 0u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

void mlp_pack(const float *blob, MlpDev *M) {
    std::memset(M, 0, sizeof(*M));
    for (int o = 0; o < 32; ++o) {
        for (int j = 0; j < 6; ++j) M->W1[o * 8 + j] = host_bf16(blob[O_W1 + 6 * o + j]);
        for (int k = 0; k < 32; ++k) {
            const uint16_t w = host_bf16(blob[O_W2 + 32 * o + k]);
            M->W2[o * 32 + k] = w;
            M->W2T[k * 32 + o] = w;
        }
        M->b1[o] = blob[O_B1 + o];
        M->b2[o] = blob[O_B2 + o];
        M->w3[o] = blob[O_W3 + o];
    }
    M->b3 = blob[O_B3];
    for (int j = 0; j < 6; ++j) {
        M->mu[j] = blob[O_MU + j];
        M->inv_sigma[j] = (float)(1.0 / (double)blob[O_SG + j]);
    }
    M->nu_scale = blob[O_NS];
}

constexpr int TB = 256;

__global__ __launch_bounds__(TB) void k_mlp_forward(const MlpDev *M, const float *feat, size_t m, float *nu) {
    __shared__ MlpLds S;
    mlp_stage_lds(M, &S);
    const size_t q = blockIdx.x * (size_t)TB + threadIdx.x;
    const bool valid = q < m;
    float f[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) f[j] = valid ? feat[q * 6 + j] : M->mu[j];
    mlp_stage_wait();
    const float v = mlp_nu_t_wave(*M, S, f);
    if (valid) nu[q] = v;
}

// One wave (64 cells) per block.
constexpr int GW = 64;
__global__ __launch_bounds__(GW) void k_mlp_grad(const MlpDev *M, const float *feat, const float *target, size_t m,
                                                 float inv_batch, float *partials, double *loss_partials) {
    __shared__ float s_da2[32][GW], s_h1[32][GW], s_da1[32][GW], s_h2[32][GW], s_x[8][GW], s_dz[GW];
    const int lane = (int)__lane_id();
    const int row = lane & 31, hi = lane >> 5;
    const size_t q = blockIdx.x * (size_t)GW + lane;
    const bool valid = q < m;
    float f[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) f[j] = valid ? feat[q * 6 + j] : M->mu[j];
    const float y = valid ? target[q] : 0.0f;
    uint32_t p[4];
    pack_features(*M, f, p);
    // x^ (bf16 values) of the own cell into LDS
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        s_x[2 * qq][lane] = bf16_bits_to_f32((uint16_t)(p[qq] & 0xffff));
        s_x[2 * qq + 1][lane] = bf16_bits_to_f32((uint16_t)(p[qq] >> 16));
    }
    const uint32_t s0 = lane < 32 ? p[2] : p[0];
    const uint32_t s1 = lane < 32 ? p[3] : p[1];
    const uint32_t r0 = (uint32_t)__shfl_xor((int)s0, 32);
    const uint32_t r1 = (uint32_t)__shfl_xor((int)s1, 32);
    const bf16x4_t xin[2] = {lane < 32 ? as_bf16x4(p[0], p[1]) : as_bf16x4(r0, r1),
                             lane < 32 ? as_bf16x4(r0, r1) : as_bf16x4(p[2], p[3])};
    f32x16_t a1[2], a2[2];
    float zc[2];
    for (int h = 0; h < 2; ++h) {
        f32x16_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = M->b1[8 * (r >> 2) + 4 * hi + (r & 3)];
        const uint2 w1 = *(const uint2 *)(M->W1 + row * 8 + 4 * hi);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(as_bf16x4(w1.x, w1.y), xin[h], acc, 0, 0, 0);
        a1[h] = acc;
        bf16x4_t hb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hb[s][j] = bf16s(fmaxf(acc[4 * s + j], 0.0f));
                s_h1[8 * s + 4 * hi + j][32 * h + row] = bf16_bits_to_f32((uint16_t)hb[s][j]);
            }
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = M->b2[8 * (r >> 2) + 4 * hi + (r & 3)];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint2 w = *(const uint2 *)(M->W2 + row * 32 + 8 * s + 4 * hi);
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(as_bf16x4(w.x, w.y), hb[s], acc, 0, 0, 0);
        }
        a2[h] = acc;
        float z = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float h2 = fmaxf(acc[r], 0.0f);
            s_h2[8 * (r >> 2) + 4 * hi + (r & 3)][32 * h + row] = h2;
            z = fmaf(M->w3[8 * (r >> 2) + 4 * hi + (r & 3)], h2, z);
        }
        z += __shfl_xor(z, 32);
        zc[h] = z + M->b3;  // z of cell 32 h + row
    }
    // loss and dz for the own cell
    const float z = lane < 32 ? zc[0] : zc[1];
    const float sp = softplusf(z);
    const float diff = valid ? sp - y : 0.0f;
    const float sig = 1.0f / (1.0f + expf(-z));
    const float dz = 2.0f * diff * sig * inv_batch;
    s_dz[lane] = dz;
    // dz of the column cell of each half
    const float dzc[2] = {__shfl(dz, row), __shfl(dz, 32 + row)};
    for (int h = 0; h < 2; ++h) {
        bf16x4_t db[4];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 8 * (r >> 2) + 4 * hi + (r & 3);
            const float da2 = a2[h][r] > 0.0f ? dzc[h] * M->w3[o] : 0.0f;
            s_da2[o][32 * h + row] = da2;
            db[r >> 2][r & 3] = bf16s(da2);
        }
        // dh1 = W2^T da2
        f32x16_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint2 w = *(const uint2 *)(M->W2T + row * 32 + 8 * s + 4 * hi);
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(as_bf16x4(w.x, w.y), db[s], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k = 8 * (r >> 2) + 4 * hi + (r & 3);
            s_da1[k][32 * h + row] = a1[h][r] > 0.0f ? acc[r] : 0.0f;
        }
    }
    __syncthreads();
    // weight / bias gradients: FP32 sums over the 64 cells, lane-strided over parameters
    float *out = partials + (size_t)blockIdx.x * MLP_NPARAM;
    for (int prm = lane; prm < MLP_NPARAM; prm += GW) {
        float acc = 0.0f;
        if (prm < O_B1) {  // W1[o][j]
            const int o = prm / 6, j = prm % 6;
            for (int c = 0; c < GW; ++c) acc = fmaf(s_da1[o][c], s_x[j][c], acc);
        } else if (prm < O_W2) {  // b1
            const int o = prm - O_B1;
            for (int c = 0; c < GW; ++c) acc += s_da1[o][c];
        } else if (prm < O_B2) {  // W2[o][k]
            const int o = (prm - O_W2) / 32, k = (prm - O_W2) % 32;
            for (int c = 0; c < GW; ++c) acc = fmaf(s_da2[o][c], s_h1[k][c], acc);
        } else if (prm < O_W3) {  // b2
            const int o = prm - O_B2;
            for (int c = 0; c < GW; ++c) acc += s_da2[o][c];
        } else if (prm < O_B3) {  // w3
            const int o = prm - O_W3;
            for (int c = 0; c < GW; ++c) acc = fmaf(s_dz[c], s_h2[o][c], acc);
        } else {  // b3
            for (int c = 0; c < GW; ++c) acc += s_dz[c];
        }
        out[prm] = acc;
    }
    // loss partial
    double l = (double)diff * (double)diff;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) loss_partials[blockIdx.x] = l;
}

// Fixed-order sum of the per-wave partials in two stages: group g (blockIdx.y)
// adds waves [g per, (g+1) per) in FP64 for every parameter and the loss
// (index MLP_NPARAM), then one pass adds the groups in order. The grouping
// depends only on the batch size, so the result is deterministic.
constexpr int RED_GROUPS = 64;
__global__ __launch_bounds__(TB) void k_mlp_reduce_groups(const float *partials, const double *loss_partials,
                                                          int nwaves, int per, double *groups) {
    const int prm = blockIdx.x * TB + threadIdx.x, g = blockIdx.y;
    if (prm > MLP_NPARAM) return;
    const int w0 = g * per, w1 = min(nwaves, w0 + per);
    double a = 0.0;
    if (prm < MLP_NPARAM)
#pragma unroll 8
        for (int w = w0; w < w1; ++w) a += partials[(size_t)w * MLP_NPARAM + prm];
    else
        for (int w = w0; w < w1; ++w) a += loss_partials[w];
    groups[(size_t)g * (MLP_NPARAM + 1) + prm] = a;
}

__global__ __launch_bounds__(TB) void k_mlp_reduce(const double *groups, int ngroups, float *grad, double count,
                                                   double *loss_acc) {
    const int prm = blockIdx.x * TB + threadIdx.x;
    if (prm > MLP_NPARAM) return;
    double a = 0.0;
    // unrolled so that the loads are issued ahead; the additions keep their order
#pragma unroll 8
    for (int g = 0; g < ngroups; ++g) a += groups[(size_t)g * (MLP_NPARAM + 1) + prm];
    if (prm < MLP_NPARAM) {
        grad[prm] = (float)a;
    } else {
        loss_acc[0] += a;
        loss_acc[1] += count;
    }
}

__global__ __launch_bounds__(TB) void k_mlp_adam(float *params, const float *grad, float *mom1, float *mom2,
                                                 int step, float lr, float beta1, float beta2, float eps) {
    const int prm = blockIdx.x * TB + threadIdx.x;
    if (prm >= MLP_NPARAM) return;
    const float g = grad[prm];
    const float m1 = beta1 * mom1[prm] + (1.0f - beta1) * g;
    const float m2 = beta2 * mom2[prm] + (1.0f - beta2) * g * g;
    mom1[prm] = m1;
    mom2[prm] = m2;
    const float mh = m1 / (1.0f - powf(beta1, (float)step));
    const float vh = m2 / (1.0f - powf(beta2, (float)step));
    params[prm] -= lr * mh / (sqrtf(vh) + eps);
}

// refresh the device network from the master parameters
__global__ __launch_bounds__(TB) void k_mlp_refresh(const float *params, MlpDev *M) {
    for (int prm = threadIdx.x; prm < MLP_NPARAM; prm += TB) {
        const float v = params[prm];
        if (prm < O_B1) {
            M->W1[(prm / 6) * 8 + prm % 6] = f32_to_bf16_bits(v);
        } else if (prm < O_W2) {
            M->b1[prm - O_B1] = v;
        } else if (prm < O_B2) {
            const int o = (prm - O_W2) / 32, k = (prm - O_W2) % 32;
            const uint16_t w = f32_to_bf16_bits(v);
            M->W2[o * 32 + k] = w;
            M->W2T[k * 32 + o] = w;
        } else if (prm < O_W3) {
            M->b2[prm - O_B2] = v;
        } else if (prm < O_B3) {
            M->w3[prm - O_W3] = v;
        } else {
            M->b3 = v;
        }
    }
}

// Scratch of lbm_mlp_loss_grad_noalloc: the per-wave gradient partials
// (float, MLP_NPARAM per wave) followed by the per-wave loss partials
// (double) for batches of up to NOALLOC_MAX_COUNT samples (5.4 MB). One copy
// per device, held until the process ends. Host code never passes the
// array's name to a kernel: it takes the device address of this device's
// copy from hipGetSymbolAddress (noalloc_scratch below).
constexpr size_t NOALLOC_MAX_COUNT = 65536;
constexpr size_t NOALLOC_MAX_WAVES = NOALLOC_MAX_COUNT / GW;
constexpr size_t NOALLOC_PART_FLOATS = NOALLOC_MAX_WAVES * MLP_NPARAM;  // even: the doubles stay 8-byte aligned
static __device__ __align__(256) float scratch[NOALLOC_PART_FLOATS + 2 * NOALLOC_MAX_WAVES];

}  // namespace lbm

using namespace lbm;

namespace {
// Device address of the scratch array, looked up once per device with that
// device current.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_scratch(float **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LBM_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EHIP;
        g_scratch_ptr[dev] = (float *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

struct lbm_mlp {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    MlpDev *d_M = nullptr;
    float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr, *d_part = nullptr;
    double *d_lpart = nullptr, *d_loss = nullptr, *d_groups = nullptr;
    size_t cap_waves = 0;
    float *d_scratch = nullptr;  // this device's copy of lbm::scratch
    int dev = -1;                // device current at creation
    float blob_tail[13] = {0};
    int step = 0;
    bool has_params = false;
    bool has_grad = false;
    std::string err;
};

namespace {
int mfail(lbm_mlp *m, int code, const char *msg) {
    if (m) m->err = msg;
    return code;
}
#define MCHK(m, expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) return mfail(m, LBM_EHIP, hipGetErrorString(e_)); \
    } while (0)

// No exception crosses the C ABI (the error string is the only host
// allocation here): a failure returns LBM_ENOMEM or LBM_EINVAL.
template <typename F>
int guard(const lbm_mlp *cm, F &&body) noexcept {
    lbm_mlp *m = const_cast<lbm_mlp *>(cm);
    int code;
    const char *msg;
    try {
        return body();
    } catch (const std::bad_alloc &) {
        code = LBM_ENOMEM;
        msg = "host allocation failed";
    } catch (...) {
        code = LBM_EINVAL;
        msg = "unexpected host error";
    }
    if (m) {
        try {
            m->err = msg;
        } catch (...) {
        }
    }
    return code;
}

int ensure_waves(lbm_mlp *m, size_t nw) {
    if (nw <= m->cap_waves) return LBM_OK;
    if (m->d_part) (void)hipFree(m->d_part);
    if (m->d_lpart) (void)hipFree(m->d_lpart);
    m->d_part = nullptr;
    m->d_lpart = nullptr;
    m->cap_waves = 0;
    if (hipMalloc((void **)&m->d_part, nw * MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_lpart, nw * sizeof(double)) != hipSuccess)
        return mfail(m, LBM_ENOMEM, "gradient partials");
    m->cap_waves = nw;
    return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_mlp_create(void *stream, lbm_mlp **out) {
    return guard(nullptr, [&]() -> int {
        if (!out) return LBM_EINVAL;
        *out = nullptr;
        lbm_mlp *m = new (std::nothrow) lbm_mlp();
        if (!m) return LBM_ENOMEM;
        if (stream) {
            m->stream = (hipStream_t)stream;
        } else if (hipStreamCreate(&m->stream) != hipSuccess) {
            delete m;
            return LBM_EHIP;
        } else {
            m->own_stream = true;
        }
        bool ok = hipMalloc((void **)&m->d_M, sizeof(MlpDev)) == hipSuccess &&
                  hipMalloc((void **)&m->d_params, MLP_NPARAM * sizeof(float)) == hipSuccess &&
                  hipMalloc((void **)&m->d_m, MLP_NPARAM * sizeof(float)) == hipSuccess &&
                  hipMalloc((void **)&m->d_v, MLP_NPARAM * sizeof(float)) == hipSuccess &&
                  hipMalloc((void **)&m->d_grad, MLP_NPARAM * sizeof(float)) == hipSuccess &&
                  hipMalloc((void **)&m->d_loss, 2 * sizeof(double)) == hipSuccess &&
                  hipMalloc((void **)&m->d_groups, (size_t)RED_GROUPS * (MLP_NPARAM + 1) * sizeof(double)) == hipSuccess;
        if (!ok || hipMemsetAsync(m->d_loss, 0, 2 * sizeof(double), m->stream) != hipSuccess) {
            lbm_mlp_destroy(m);
            return LBM_ENOMEM;
        }
        if (hipGetDevice(&m->dev) != hipSuccess || noalloc_scratch(&m->d_scratch) != LBM_OK) {
            lbm_mlp_destroy(m);
            return LBM_EHIP;
        }
        *out = m;
        return LBM_OK;
    });
}

int lbm_mlp_destroy(lbm_mlp *m) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (m->stream) (void)hipStreamSynchronize(m->stream);
        void *ptrs[] = {m->d_M, m->d_params, m->d_m, m->d_v, m->d_grad, m->d_part, m->d_lpart, m->d_loss, m->d_groups};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        if (m->own_stream) (void)hipStreamDestroy(m->stream);
        delete m;
        return LBM_OK;
    });
}

int lbm_mlp_set_params(lbm_mlp *m, const float *blob, size_t n) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!blob || n != (size_t)MLP_NBLOB) return mfail(m, LBM_EINVAL, "expected 1326 parameters");
        for (int j = 0; j < 6; ++j)
            if (!(blob[O_SG + j] > 0.0f)) return mfail(m, LBM_EINVAL, "sigma must be positive");
        MlpDev h;
        mlp_pack(blob, &h);
        MCHK(m, hipMemcpyAsync(m->d_M, &h, sizeof h, hipMemcpyHostToDevice, m->stream));
        MCHK(m, hipMemcpyAsync(m->d_params, blob, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, m->stream));
        MCHK(m, hipMemsetAsync(m->d_m, 0, MLP_NPARAM * sizeof(float), m->stream));
        MCHK(m, hipMemsetAsync(m->d_v, 0, MLP_NPARAM * sizeof(float), m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
        std::memcpy(m->blob_tail, blob + MLP_NPARAM, sizeof m->blob_tail);
        m->step = 0;
        m->has_params = true;
        m->has_grad = false;
        return LBM_OK;
    });
}

int lbm_mlp_get_params(lbm_mlp *m, float *blob, size_t n) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!blob || n != (size_t)MLP_NBLOB) return mfail(m, LBM_EINVAL, "expected 1326 parameters");
        if (!m->has_params) return mfail(m, LBM_ESTATE, "parameters not set");
        MCHK(m, hipMemcpyAsync(blob, m->d_params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
        std::memcpy(blob + MLP_NPARAM, m->blob_tail, sizeof m->blob_tail);
        return LBM_OK;
    });
}

int lbm_mlp_forward(lbm_mlp *m, const float *d_feat, size_t count, float *d_nu) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!m->has_params) return mfail(m, LBM_ESTATE, "parameters not set");
        if (count == 0) return LBM_OK;
        if (!d_feat || !d_nu) return mfail(m, LBM_EINVAL, "null device array");
        k_mlp_forward<<<(unsigned)((count + TB - 1) / TB), TB, 0, m->stream>>>(m->d_M, d_feat, count, d_nu);
        MCHK(m, hipGetLastError());
        return LBM_OK;
    });
}

}  // extern "C"

namespace {
// Gradient kernels of one batch with the per-wave partials in part / lpart
// (room for nw waves each).
int loss_grad_launch(lbm_mlp *m, const float *d_feat, const float *d_target, size_t count, size_t nw, float *part,
                     double *lpart, float *grad) {
    k_mlp_grad<<<(unsigned)nw, GW, 0, m->stream>>>(m->d_M, d_feat, d_target, count, 1.0f / (float)count, part, lpart);
    const int per = (int)((nw + RED_GROUPS - 1) / RED_GROUPS), ngroups = (int)((nw + per - 1) / per);
    const unsigned pblocks = (MLP_NPARAM + 1 + TB - 1) / TB;
    k_mlp_reduce_groups<<<dim3(pblocks, ngroups), TB, 0, m->stream>>>(part, lpart, (int)nw, per, m->d_groups);
    k_mlp_reduce<<<pblocks, TB, 0, m->stream>>>(m->d_groups, ngroups, m->d_grad, (double)count, m->d_loss);
    MCHK(m, hipGetLastError());
    m->has_grad = true;
    if (grad) {
        MCHK(m, hipMemcpyAsync(grad, m->d_grad, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_mlp_loss_grad(lbm_mlp *m, const float *d_feat, const float *d_target, size_t count, float *grad) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!m->has_params) return mfail(m, LBM_ESTATE, "parameters not set");
        if (count == 0 || !d_feat || !d_target) return mfail(m, LBM_EINVAL, "empty batch or null device array");
        const size_t nw = (count + GW - 1) / GW;
        int rc = ensure_waves(m, nw);
        if (rc) return rc;
        return loss_grad_launch(m, d_feat, d_target, count, nw, m->d_part, m->d_lpart, grad);
    });
}

int lbm_mlp_loss_grad_noalloc(lbm_mlp *m, const float *d_feat, const float *d_target, size_t count, float *grad) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!m->has_params) return mfail(m, LBM_ESTATE, "parameters not set");
        if (count == 0 || !d_feat || !d_target) return mfail(m, LBM_EINVAL, "empty batch or null device array");
        if (count > NOALLOC_MAX_COUNT)
            return mfail(m, LBM_EINVAL, "batch exceeds the 65536 samples of the no-allocation scratch");
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess) return mfail(m, LBM_EHIP, "hipGetDevice failed");
        if (dev != m->dev)
            return mfail(m, LBM_EINVAL, "current device is not the trainer's device");
        const size_t nw = (count + GW - 1) / GW;
        return loss_grad_launch(m, d_feat, d_target, count, nw, m->d_scratch,
                                (double *)(m->d_scratch + NOALLOC_PART_FLOATS), grad);
    });
}

int lbm_mlp_adam_step(lbm_mlp *m, float lr, float beta1, float beta2, float eps) {
    return guard(m, [&]() -> int {
        if (!m) return LBM_EINVAL;
        if (!m->has_grad) return mfail(m, LBM_ESTATE, "no gradient computed");
        if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
            return mfail(m, LBM_EINVAL, "bad Adam hyper-parameters");
        m->step += 1;
        k_mlp_adam<<<(MLP_NPARAM + TB - 1) / TB, TB, 0, m->stream>>>(m->d_params, m->d_grad, m->d_m, m->d_v, m->step, lr,
                                                                     beta1, beta2, eps);
        k_mlp_refresh<<<1, TB, 0, m->stream>>>(m->d_params, m->d_M);
        MCHK(m, hipGetLastError());
        return LBM_OK;
    });
}

int lbm_mlp_take_loss(lbm_mlp *m, double *mean_loss) {
    return guard(m, [&]() -> int {
        if (!m || !mean_loss) return LBM_EINVAL;
        double h[2];
        MCHK(m, hipMemcpyAsync(h, m->d_loss, 2 * sizeof(double), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
        MCHK(m, hipMemsetAsync(m->d_loss, 0, 2 * sizeof(double), m->stream));
        *mean_loss = h[1] > 0 ? h[0] / h[1] : 0.0;
        return LBM_OK;
    });
}

const char *lbm_mlp_last_error(const lbm_mlp *m) { return m ? m->err.c_str() : "null handle"; }

}  // extern "C"
