// Learned eddy-viscosity closure on the matrix cores (gfx950).
//
// A wave of 64 cells evaluates the per-cell network 6 -> 32 -> 32 -> 1 with
// gfx950's v_mfma_f32_32x32x16_bf16 (32x32 output tile, K = 16, bfloat16
// inputs, FP32 accumulation), one half-wave of 32 cells per output tile:
//   layer 1: H1 = [W1 | 0] or [0 | W1] (32 x 16) * X (16 x 32), where column
//            c of X holds the features of cells c and c + 32 (6 each, padded
//            to 8): the zero block picks the half-wave, and every lane passes
//            its own features, unshuffled;
//   layer 2: H2 = W2 (32 x 32) * relu(H1) (32 x 32 cells), 2 K-blocks;
//   layer 3: z = w3 . relu(H2) + b3 on the vector ALU, softplus output.
// Operand layout of the 32x32x16 instruction (lane l of 64):
//   A (M x K): row l % 32, k = 8 (l / 32) + j, j = 0..7
//   B (K x N): col l % 32, k = 8 (l / 32) + j
//   D (M x N): register r holds row 8 (r / 4) + 4 (l / 32) + r % 4, col l % 32
// The D registers 8s..8s+7 of layer 1 serve as the B operand of K-block s of
// layer 2 as they are: the hidden layer never leaves registers, and the A
// operand of that block takes the matching columns of W2 (hidden units
// 16s + 4 (l / 32) + 0..3 and 16s + 8 + 4 (l / 32) + 0..3); a sum over k does
// not depend on the order of its terms.
// The training kernels evaluate the same network with the K = 8 instruction
// (v_mfma_f32_32x32x8_bf16, A/B lane l: k = 4 (l / 32) + j, j = 0..3) and
// the same D layout.
#pragma once
#include <cstddef>
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
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
    const float tau = 0.5f * (tau0 + fsqrt(tau0 * tau0 + 18.0f * 1.41421356237f * 0.01f * q));
    f[5] = (tau - tau0) * (1.0f / 3.0f);
}

// max(x, 0) as one integer max on the bit pattern: a negative float has a
// negative two's-complement pattern, a positive one keeps its order
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// softplus(z) = max(z, 0) + log(1 + e), e = exp(-|z|) in (0, 1]. The
// logarithm uses log(1 + e) = 2 atanh(s), s = e / (2 + e) in (0, 1/3], and
// the odd series 2 (s + s^3/3 + ... + s^15/15): the first dropped term is
// below s^16/17 < 2e-9 of the sum, and the result keeps its relative
// accuracy for tiny e, where log(1 + e) would round to zero. e comes from the
// hardware base-2 exponential of -|z| log2(e) (two instructions instead of
// the thirteen of the range-reduced expf): its relative error, about
// |z| 2^-24 from the rounded product, stays below 1e-6 for |z| < 16; beyond
// |z| = 87, e < 2^-126, whether kept or flushed, leaves max(z, 0) (or a
// viscosity below 1e-37) to FP32 precision.
__device__ __forceinline__ float softplusf(float z) {
    const float e = __expf(-fabsf(z));
    const float s = e * frcp(2.0f + e), t = s * s;
    float p = 1.0f / 15.0f;
    p = fmaf(p, t, 1.0f / 13.0f);
    p = fmaf(p, t, 1.0f / 11.0f);
    p = fmaf(p, t, 1.0f / 9.0f);
    p = fmaf(p, t, 1.0f / 7.0f);
    p = fmaf(p, t, 1.0f / 5.0f);
    p = fmaf(p, t, 1.0f / 3.0f);
    p = fmaf(p, t, 1.0f);
    return fmaxf(z, 0.0f) + 2.0f * s * p;
}

// Normalised, bf16-rounded features of the lane's cell packed as 4 x 2 bf16.
__device__ __forceinline__ void pack_features(const MlpDev &M, const float f[6], uint32_t p[4]) {
    float s[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) s[j] = (f[j] - M.mu[j]) * M.inv_sigma[j];
    p[0] = f32x2_to_bf16x2_bits(s[0], s[1]);
    p[1] = f32x2_to_bf16x2_bits(s[2], s[3]);
    p[2] = f32x2_to_bf16x2_bits(s[4], s[5]);
    p[3] = 0u;
}

typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4_t as_bf16x4(uint32_t lo, uint32_t hi) {
    const u32x2_t v = {lo, hi};
    return __builtin_bit_cast(bf16x4_t, v);
}

// Copy of the network operands in LDS, one per workgroup: W1 and W2 (the A
// operands) and b1, b2, w3. Every lane of a half-wave reads the same bias and
// output-weight entries, so LDS broadcasts them; read from global memory they
// would cost each wave 17 vector loads of up to 1 KB behind its population
// loads.
struct MlpLds {
    uint16_t W1[32 * 8];
    uint16_t W2[32 * 32];
    float b1[32], b2[32], w3[32];
};
static_assert(sizeof(MlpLds) == 2944, "LDS image of the network");
static_assert(offsetof(MlpDev, W2) == offsetof(MlpDev, W1) + sizeof(MlpLds::W1), "W1, W2 adjacent");
static_assert(offsetof(MlpDev, b2) == offsetof(MlpDev, b1) + 128 && offsetof(MlpDev, w3) == offsetof(MlpDev, b1) + 256,
              "b1, b2, w3 adjacent");
static_assert(offsetof(MlpDev, b1) % 16 == 0, "16-byte chunks");

// Start the copy of the network into LDS: 184 chunks of 16 bytes, one per
// thread of the first 184 threads of the block (blockDim.x >= 192), moved by
// the global-to-LDS DMA of gfx950 (global_load_lds_dwordx4) without passing
// through registers. Lane l of a wave writes chunk (wave base + l).
__device__ __forceinline__ void mlp_stage_lds(const MlpDev *M, MlpLds *S) {
    constexpr unsigned NW12 = (sizeof(MlpLds::W1) + sizeof(MlpLds::W2)) / 16;  // 160
    constexpr unsigned NCH = sizeof(MlpLds) / 16;                                  // 184
    const unsigned c = threadIdx.x, wave_base = threadIdx.x & ~63u;
    if (wave_base < NCH && c < NCH) {
        const char *src = c < NW12 ? (const char *)M->W1 + 16 * c : (const char *)M->b1 + 16 * (c - NW12);
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)((char *)S + 16 * wave_base), 16, 0,
                                         0);
    }
}

// Wait for the copy: the DMA counts as an outstanding vector-memory load of
// the issuing wave, then the block barrier makes every wave's part visible.
// Every thread of the block must call this.
__device__ __forceinline__ void mlp_stage_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// The network operands one lane needs, read once per wave from LDS and shared
// by both half-wave evaluations: its row of W1 in the half of K that selects
// each half-wave (zero in the other), its columns of W2 for the two K-blocks
// of layer 2, and the 16 bias / output-weight entries of the D-register rows
// it holds.
struct MlpLane {
    bf16x8_t w1a, w1b, w2[2];
    f32x16_t b1, b2, w3;
};

__device__ __forceinline__ f32x16_t load_drows(const float *v, int hi) {
    f32x16_t r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 t = *(const float4 *)(v + 8 * q + 4 * hi);
        r[4 * q] = t.x;
        r[4 * q + 1] = t.y;
        r[4 * q + 2] = t.z;
        r[4 * q + 3] = t.w;
    }
    return r;
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x8_t as_bf16x8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const u32x4_t v = {a, b, c, d};
    return __builtin_bit_cast(bf16x8_t, v);
}

__device__ __forceinline__ MlpLane mlp_lane(const MlpLds &S, int lane) {
    const int row = lane & 31, hi = lane >> 5;
    MlpLane L;
    const uint4 w = *(const uint4 *)(S.W1 + row * 8);
    const bf16x8_t w1 = as_bf16x8(w.x, w.y, w.z, w.w), zero = as_bf16x8(0u, 0u, 0u, 0u);
    L.w1a = hi ? zero : w1;  // half-wave 0: cells 0..31 are k = 0..7
    L.w1b = hi ? w1 : zero;  // half-wave 1: cells 32..63 are k = 8..15
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const uint2 u = *(const uint2 *)(S.W2 + row * 32 + 16 * s + 4 * hi);
        const uint2 v = *(const uint2 *)(S.W2 + row * 32 + 16 * s + 8 + 4 * hi);
        L.w2[s] = as_bf16x8(u.x, u.y, v.x, v.y);
    }
    L.b1 = load_drows(S.b1, hi);
    L.b2 = load_drows(S.b2, hi);
    L.w3 = load_drows(S.w3, hi);
    return L;
}

typedef short s16x2_t __attribute__((ext_vector_type(2)));
// ReLU of two packed bfloat16 values as one packed 16-bit integer max: the
// sign bit of a bfloat16 is the sign bit of its 16-bit pattern, and rounding
// to bfloat16 keeps the sign, so relu(bf16(x)) = bf16(relu(x)).
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
    const s16x2_t z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2_t, v), z));
}

// relu(H1) in bfloat16 from the layer-1 accumulator: registers 8s..8s+7
// form the B operand of K-block s of layer 2
__device__ __forceinline__ void hidden_bf16(const f32x16_t &acc, bf16x8_t h[2]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
        h[s] = as_bf16x8(relu_bf16x2(f32x2_to_bf16x2_bits(acc[8 * s], acc[8 * s + 1])),
                         relu_bf16x2(f32x2_to_bf16x2_bits(acc[8 * s + 2], acc[8 * s + 3])),
                         relu_bf16x2(f32x2_to_bf16x2_bits(acc[8 * s + 4], acc[8 * s + 5])),
                         relu_bf16x2(f32x2_to_bf16x2_bits(acc[8 * s + 6], acc[8 * s + 7])));
}

// Both half-wave evaluations, interleaved so that the dependent matrix-core
// chains of one half overlap the other's. x: the B operand of layer 1 (each
// lane's own features). Returns z - b3 for the cell in column lane % 32 of
// each half (valid in both lane halves).
__device__ __forceinline__ void mlp_halves(const MlpLane &L, bf16x8_t x, float &z0, float &z1) {
    // layer 1 (bias as the accumulator input)
    f32x16_t a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w1a, x, L.b1, 0, 0, 0);
    f32x16_t a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w1b, x, L.b1, 0, 0, 0);
    bf16x8_t h0[2], h1[2];
    hidden_bf16(a0, h0);
    hidden_bf16(a1, h1);
    // layer 2
    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w2[0], h0[0], L.b2, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w2[0], h1[0], L.b2, 0, 0, 0);
    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w2[1], h0[1], a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w2[1], h1[1], a1, 0, 0, 0);
    // layer 3: this lane holds 16 of the 32 hidden units of its column
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        s0 = fmaf(L.w3[r], relu(a0[r]), s0);
        s1 = fmaf(L.w3[r], relu(a1[r]), s1);
    }
    z0 = s0 + __shfl_xor(s0, 32);
    z1 = s1 + __shfl_xor(s1, 32);
}

// Eddy viscosity of the lane's own cell; all 64 lanes of the wave must call
// this together (matrix-core instructions act on the whole wave).
// S: the LDS copy of the network (mlp_stage_lds, mlp_stage_wait).
__device__ __forceinline__ float mlp_nu_t_wave(const MlpDev &M, const MlpLds &S, const float f[6]) {
    const int lane = (int)__lane_id();
    uint32_t p[4];
    pack_features(M, f, p);
    const MlpLane L = mlp_lane(S, lane);
    float z0, z1;
    mlp_halves(L, as_bf16x8(p[0], p[1], p[2], p[3]), z0, z1);
    const float z = (lane < 32 ? z0 : z1) + M.b3;
    return M.nu_scale * softplusf(z);
}

}  // namespace lbm
