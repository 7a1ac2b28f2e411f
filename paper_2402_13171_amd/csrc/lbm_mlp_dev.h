// Learned eddy-viscosity closure on the matrix cores (gfx950).
//
// A wave of 64 cells evaluates the per-cell network 6 -> 32 -> 32 -> 1 with
// v_mfma_f32_32x32x8_bf16 (32x32 output tile, K = 8, bfloat16 inputs, FP32
// accumulation), one half-wave of 32 cells per tile:
//   layer 1: H1 = W1 (32 x 8) * X (8 x 32 cells), features padded 6 -> 8;
//   layer 2: H2 = W2 (32 x 32) * relu(H1) (32 x 32 cells), 4 K-blocks;
//   layer 3: z = w3 . relu(H2) + b3 on the vector ALU, softplus output.
// Operand layout of the 32x32x8 instruction (lane l of 64):
//   A (M x K): row l % 32, k = 4 (l / 32) + j, j = 0..3
//   B (K x N): col l % 32, k = 4 (l / 32) + j
//   D (M x N): register r holds row 8 (r / 4) + 4 (l / 32) + r % 4, col l % 32
// so the D registers 4s..4s+3 of layer 1 are exactly the B operand of K-block
// s of layer 2: the hidden layer never leaves registers. Feature vectors of
// one cell per lane reach the B layout of layer 1 with one cross-half swap.
#pragma once
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16s(float v) { return (short)f32_to_bf16_bits(v); }

// The six closure inputs of one cell: invariants of A = Pi_neq/rho, the norm
// of its deviator, rho - 1 and the Smagorinsky viscosity for Cs = 0.1.
__device__ __forceinline__ void closure_features(const CellMoments &m, float tau0, float f[6]) {
    const float ex = m.ex, ey = m.ey, ez = m.ez, a = m.kxy, b = m.kxz, c = m.kyz;
    const float i1 = ex + ey + ez;
    const float tr2 = ex * ex + ey * ey + ez * ez + 2.0f * (a * a + b * b + c * c);
    f[0] = i1;
    f[1] = 0.5f * (i1 * i1 - tr2);
    f[2] = ex * (ey * ez - c * c) - a * (a * ez - c * b) + b * (a * c - ey * b);
    const float q = q_norm(m);
    f[3] = q;
    f[4] = m.drho;
    const float tau = 0.5f * (tau0 + sqrtf(tau0 * tau0 + 18.0f * 1.41421356237f * 0.01f * q));
    f[5] = (tau - tau0) * (1.0f / 3.0f);
}

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

// Normalised, bf16-rounded features of the lane's cell packed as 4 x 2 bf16.
__device__ __forceinline__ void pack_features(const MlpDev &M, const float f[6], uint32_t p[4]) {
    short s[8];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float d = f[j] - M.mu[j];
        s[j] = bf16s(d * M.inv_sigma[j]);
    }
    s[6] = 0;
    s[7] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = (uint32_t)(uint16_t)s[2 * q] | ((uint32_t)(uint16_t)s[2 * q + 1] << 16);
}

__device__ __forceinline__ bf16x4_t as_bf16x4(uint32_t lo, uint32_t hi) {
    bf16x4_t v;
    v[0] = (short)(lo & 0xffff);
    v[1] = (short)(lo >> 16);
    v[2] = (short)(hi & 0xffff);
    v[3] = (short)(hi >> 16);
    return v;
}

// Per-half-wave network evaluation. xin: B operand of layer 1 for this half.
// Returns z for the cell in column lane % 32 (valid in both lane halves).
__device__ __forceinline__ float mlp_half(const MlpDev &M, bf16x4_t xin, int lane) {
    const int row = lane & 31, hi = lane >> 5;
    // layer 1
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = M.b1[8 * (r >> 2) + 4 * hi + (r & 3)];
    {
        const uint2 w = *(const uint2 *)(M.W1 + row * 8 + 4 * hi);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(as_bf16x4(w.x, w.y), xin, acc, 0, 0, 0);
    }
    // relu + bf16: registers 4s..4s+3 form the B operand of K-block s
    bf16x4_t h[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) h[s][j] = bf16s(fmaxf(acc[4 * s + j], 0.0f));
    // layer 2
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = M.b2[8 * (r >> 2) + 4 * hi + (r & 3)];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint2 w = *(const uint2 *)(M.W2 + row * 32 + 8 * s + 4 * hi);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(as_bf16x4(w.x, w.y), h[s], acc, 0, 0, 0);
    }
    // layer 3: this lane holds 16 of the 32 hidden units of its column
    float z = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) z = fmaf(M.w3[8 * (r >> 2) + 4 * hi + (r & 3)], fmaxf(acc[r], 0.0f), z);
    z += __shfl_xor(z, 32);
    return z + M.b3;
}

// Eddy viscosity of the lane's own cell; all 64 lanes of the wave must call
// this together (matrix-core instructions act on the whole wave).
__device__ __forceinline__ float mlp_nu_t_wave(const MlpDev &M, const float f[6]) {
    const int lane = (int)__lane_id();
    uint32_t p[4];
    pack_features(M, f, p);
    // lanes < 32 need their own features 0..3 for half 0 and the partner's
    // 0..3 for half 1; lanes >= 32 the partner's 4..7 for half 0 and their
    // own 4..7 for half 1: send what the partner lacks
    const uint32_t s0 = lane < 32 ? p[2] : p[0];
    const uint32_t s1 = lane < 32 ? p[3] : p[1];
    const uint32_t r0 = (uint32_t)__shfl_xor((int)s0, 32);
    const uint32_t r1 = (uint32_t)__shfl_xor((int)s1, 32);
    const bf16x4_t x0 = lane < 32 ? as_bf16x4(p[0], p[1]) : as_bf16x4(r0, r1);
    const bf16x4_t x1 = lane < 32 ? as_bf16x4(r0, r1) : as_bf16x4(p[2], p[3]);
    const float z0 = mlp_half(M, x0, lane);
    const float z1 = mlp_half(M, x1, lane);
    const float z = lane < 32 ? z0 : z1;
    return M.nu_scale * softplusf(z);
}

}  // namespace lbm
