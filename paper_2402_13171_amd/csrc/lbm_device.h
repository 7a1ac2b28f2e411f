// Device-side building blocks of the D3Q27 cumulant update (gfx950).
//
// Populations are stored as deviations d_i = f_i - w_i from the lattice
// weights, so every quantity the collision forms (density deviation,
// momentum, second moments, cumulant deviations) is a small number and FP32
// keeps its relative precision. The collision works on these deviations end
// to end: it never rebuilds f_i = w_i + d_i.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------ lattice
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int opp(int i) { return 26 - i; }
__host__ __device__ constexpr int refl_z(int i) { return i - 18 * cz_of(i); }
__host__ __device__ constexpr float w1d(int c) { return c == 0 ? 2.0f / 3.0f : 1.0f / 6.0f; }
__host__ __device__ constexpr float wgt(int i) { return w1d(cx_of(i)) * w1d(cy_of(i)) * w1d(cz_of(i)); }

// ------------------------------------------------------------ storage types
struct bf16_t { uint16_t v; };

template <typename T> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float ld(const __half *p) { return __half2float(*p); }
    static __device__ __forceinline__ void st(__half *p, float v) { *p = __float2half_rn(v); }
};
// bfloat16: upper half of the float32 pattern, rounded to nearest even by
// the gfx950 conversion instruction (v_cvt_pk_bf16_f32, default round mode)
typedef __bf16 bf16x2_native __attribute__((ext_vector_type(2)));
typedef float f32x2_native __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
// two values in one instruction: lo in bits 0..15, hi in bits 16..31
__device__ __forceinline__ uint32_t f32x2_to_bf16x2_bits(float lo, float hi) {
    const f32x2_native v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_native));
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
template <> struct Store<bf16_t> {
    static __device__ __forceinline__ float ld(const bf16_t *p) { return bf16_bits_to_f32(p->v); }
    static __device__ __forceinline__ void st(bf16_t *p, float v) { p->v = f32_to_bf16_bits(v); }
};
// The same two storage formats as written by the stepping kernels with
// stochastic rounding (the values reach the store already on the grid, see
// sr_round_cell; the conversion there is exact).
struct f16_sr { uint16_t v; };
struct bf16_sr { uint16_t v; };
template <> struct Store<f16_sr> {
    static __device__ __forceinline__ float ld(const f16_sr *p) { return Store<__half>::ld((const __half *)p); }
    static __device__ __forceinline__ void st(f16_sr *p, float v) { Store<__half>::st((__half *)p, v); }
};
template <> struct Store<bf16_sr> {
    static __device__ __forceinline__ float ld(const bf16_sr *p) { return Store<bf16_t>::ld((const bf16_t *)p); }
    static __device__ __forceinline__ void st(bf16_sr *p, float v) { Store<bf16_t>::st((bf16_t *)p, v); }
};

// ------------------------------------------------------------ stochastic rounding
// With LBM_ROUND_STOCHASTIC (storage types f16_sr / bf16_sr below), the
// 16-bit stores of the stepping kernels round stochastically: a value between
// two representable neighbours goes to the upper one with probability equal
// to its distance from the lower one over their spacing, using gfx950's
// conversion instructions with a random operand (v_cvt_sr_f16_f32,
// v_cvt_sr_bf16_f32). The expected stored value is then the value itself, so
// the rounding of a steady flow does not add up to a drift step after step
// (round-to-nearest rounds a steady value the same way every step); the
// error becomes a zero-mean perturbation that the viscosity damps. Values
// already representable (the rest state, for one) are stored exactly.
// Random words: mix32 (lbm_internal.h) of the cell index and a per-step
// seed, plus a Weyl increment per direction; deterministic for a given cell,
// step and direction.

typedef _Float16 f16x2_native __attribute__((ext_vector_type(2)));
// Two values rounded stochastically to the storage type's grid, returned as
// floats (exact in the storage type, so the store's own conversion keeps
// them unchanged); the two conversions fill the halves of one register.
template <typename T> struct SrRound {
    static __device__ __forceinline__ void q2(float &a, float &b, uint32_t, uint32_t) {}
};
template <> struct SrRound<f16_sr> {
    static __device__ __forceinline__ void q2(float &a, float &b, uint32_t ra, uint32_t rb) {
        f16x2_native z = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(f16x2_native, a), a, ra, false);
        z = __builtin_amdgcn_cvt_sr_f16_f32(z, b, rb, true);
        a = (float)z[0];
        b = (float)z[1];
    }
};
template <> struct SrRound<bf16_sr> {
    static __device__ __forceinline__ void q2(float &a, float &b, uint32_t ra, uint32_t rb) {
        bf16x2_native z = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(bf16x2_native, a), a, ra, false);
        z = __builtin_amdgcn_cvt_sr_bf16_f32(z, b, rb, true);
        a = (float)z[0];
        b = (float)z[1];
    }
};
// the 27 post-collision values of one cell
template <typename T> inline constexpr bool rounds_stochastically = false;
template <> inline constexpr bool rounds_stochastically<f16_sr> = true;
template <> inline constexpr bool rounds_stochastically<bf16_sr> = true;
template <typename T>
__device__ __forceinline__ void sr_round_cell(float *o, uint32_t cell, uint32_t seed) {
    if constexpr (rounds_stochastically<T>) {
        const uint32_t h = mix32(cell ^ seed);
        float spare = 0.0f;
#pragma unroll
        for (int i = 0; i < 27; i += 2) {
            float &b = i + 1 < 27 ? o[i + 1] : spare;
            SrRound<T>::q2(o[i], b, h + (uint32_t)i * SR_WEYL, h + (uint32_t)(i + 1) * SR_WEYL);
        }
    }
}

// ------------------------------------------------------------ collision
// Closure kinds (values match lbm_closure).
enum { CL_NONE = 0, CL_SMAG = 1, CL_MLP = 2 };

struct CellMoments {
    float drho, rho, ux, uy, uz;
    float ex, ey, ez;      // k_aa - 1/3, normalised diagonal second central moments
    float kxy, kxz, kyz;   // normalised off-diagonal second central moments
};

// Density deviation, momentum and second raw moments of the deviations,
// taken one axis at a time (z lines, then y, then x), then the velocity
// u = (j + F/2)/rho and the normalised second central moments about u.
// Hardware reciprocal and square root (v_rcp_f32, v_sqrt_f32: about 1 ulp),
// used where a correctly rounded result buys nothing.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// FRC = false drops the force terms at compile time (F = 0).
template <bool FRC = true>
__device__ __forceinline__ CellMoments moments_of(const float d[27], float Fx, float Fy, float Fz) {
    float Z0[9], Z1[9], Z2[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        float a = d[p], b = d[p + 9], c = d[p + 18];
        Z2[p] = c + a;
        Z1[p] = c - a;
        Z0[p] = Z2[p] + b;  // the zeroth moment reuses the outer pair's sum
    }
    // y pass: index p = ix + 3*iy
    float Y00[3], Y01[3], Y02[3], Y10[3], Y11[3], Y20[3];
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
        Y02[ix] = Z0[ix + 6] + Z0[ix];
        Y01[ix] = Z0[ix + 6] - Z0[ix];
        Y00[ix] = Y02[ix] + Z0[ix + 3];
        Y10[ix] = Z1[ix] + Z1[ix + 3] + Z1[ix + 6];
        Y11[ix] = Z1[ix + 6] - Z1[ix];
        Y20[ix] = Z2[ix] + Z2[ix + 3] + Z2[ix + 6];
    }
    const float m200 = Y00[2] + Y00[0];
    const float m100 = Y00[2] - Y00[0];
    const float m000 = m200 + Y00[1];
    const float m010 = Y01[0] + Y01[1] + Y01[2];
    const float m110 = Y01[2] - Y01[0];
    const float m020 = Y02[0] + Y02[1] + Y02[2];
    const float m001 = Y10[0] + Y10[1] + Y10[2];
    const float m101 = Y10[2] - Y10[0];
    const float m011 = Y11[0] + Y11[1] + Y11[2];
    const float m002 = Y20[0] + Y20[1] + Y20[2];

    CellMoments m;
    m.drho = m000;
    m.rho = 1.0f + m000;
    const float irho = frcp(m.rho);
    // kappa_ab = Pi_ab - rho u_a u_b + (u_a F_b + u_b F_a)/2, Pi_aa = m_aa + 1/3
    // e_a = kappa_aa/rho - 1/3 = (m_aa - drho/3 - rho u_a^2 + u_a F_a) / rho
    const float d3 = m000 * (1.0f / 3.0f);
    if (FRC) {
        m.ux = (m100 + 0.5f * Fx) * irho;
        m.uy = (m010 + 0.5f * Fy) * irho;
        m.uz = (m001 + 0.5f * Fz) * irho;
        m.ex = (m200 - d3 - m.rho * m.ux * m.ux + m.ux * Fx) * irho;
        m.ey = (m020 - d3 - m.rho * m.uy * m.uy + m.uy * Fy) * irho;
        m.ez = (m002 - d3 - m.rho * m.uz * m.uz + m.uz * Fz) * irho;
        m.kxy = (m110 - m.rho * m.ux * m.uy + 0.5f * (m.ux * Fy + m.uy * Fx)) * irho;
        m.kxz = (m101 - m.rho * m.ux * m.uz + 0.5f * (m.ux * Fz + m.uz * Fx)) * irho;
        m.kyz = (m011 - m.rho * m.uy * m.uz + 0.5f * (m.uy * Fz + m.uz * Fy)) * irho;
    } else {
        m.ux = m100 * irho;
        m.uy = m010 * irho;
        m.uz = m001 * irho;
        m.ex = (m200 - d3 - m.rho * m.ux * m.ux) * irho;
        m.ey = (m020 - d3 - m.rho * m.uy * m.uy) * irho;
        m.ez = (m002 - d3 - m.rho * m.uz * m.uz) * irho;
        m.kxy = (m110 - m.rho * m.ux * m.uy) * irho;
        m.kxz = (m101 - m.rho * m.ux * m.uz) * irho;
        m.kyz = (m011 - m.rho * m.uy * m.uz) * irho;
    }
    return m;
}

// Norm of the deviatoric non-equilibrium stress per unit density.
__device__ __forceinline__ float q_norm(const CellMoments &m) {
    const float tr3 = (m.ex + m.ey + m.ez) * (1.0f / 3.0f);
    const float a = m.ex - tr3, b = m.ey - tr3, c = m.ez - tr3;
    return fsqrt(a * a + b * b + c * c + 2.0f * (m.kxy * m.kxy + m.kxz * m.kxz + m.kyz * m.kyz));
}

// Smagorinsky shear rate in the closed form of Hou et al. (1996):
// tau = (tau0 + sqrt(tau0^2 + 18 sqrt(2) Cs^2 Q)) / 2.
__device__ __forceinline__ float smag_omega(float Q, float tau0, float cs2_18sqrt2) {
    const float tau = 0.5f * (tau0 + fsqrt(tau0 * tau0 + cs2_18sqrt2 * Q));
    return frcp(tau);
}

// One 1-D inverse pass on a triple of central moments (k0,k1,k2) about u:
// raw moments m0 = k0, m1 = k1 + u k0, m2 = k2 + 2 u k1 + u^2 k0, then the
// populations f- = (m2 - m1)/2, f0 = m0 - m2, f+ = (m2 + m1)/2. The halves
// are taken as fma(1/2, m2, -+m1/2): halving is exact, so these round as
// (m2 -+ m1)/2 do, bit for bit, in one instruction fewer.
__device__ __forceinline__ void inv_triple(float &a, float &b, float &c, float u) {
    const float k0 = a, k1 = b, k2 = c;
    const float m1 = fmaf(u, k0, k1);
    const float m2 = fmaf(u, k1 + m1, k2);
    const float h1 = 0.5f * m1;
    a = fmaf(0.5f, m2, -h1);
    b = k0 - m2;
    c = fmaf(0.5f, m2, h1);
}

// Post-collision deviations d*_i = f*_i - w_i, for unit higher-order rates
// (omega_3..omega_10 = 1; omega_2 arbitrary): the third- to sixth-order
// cumulants are zero after the collision, so the post-collision central
// moments follow from the relaxed second-order ones alone. The target array
// is dk = kappa* - kappa_w(u), where kappa_w(u) are the central moments of
// the weights about u (the product of 1, -u, 1/3 + u^2 per axis); the
// inverse transform of dk is exactly f* - w.
__device__ __forceinline__ void collide_unit_rates(const CellMoments &m, float omega1, float omega2,
                                                   float Fx, float Fy, float Fz, float out[27]) {
    const float r = m.rho, dr = m.drho;
    const float ux = m.ux, uy = m.uy, uz = m.uz;
    const float ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    const float s1 = 1.0f - omega1;
    // second order
    const float dxy = s1 * (m.ex - m.ey);
    const float dxz = s1 * (m.ex - m.ez);
    const float trd = (1.0f - omega2) * (m.ex + m.ey + m.ez);
    const float ex = (trd + dxy + dxz) * (1.0f / 3.0f);
    const float ey = (trd - 2.0f * dxy + dxz) * (1.0f / 3.0f);
    const float ez = (trd + dxy - 2.0f * dxz) * (1.0f / 3.0f);
    const float kxy = s1 * m.kxy, kxz = s1 * m.kxz, kyz = s1 * m.kyz;
    const float Kxx = (1.0f / 3.0f) + ex, Kyy = (1.0f / 3.0f) + ey, Kzz = (1.0f / 3.0f) + ez;
    const float px = (1.0f / 3.0f) + ux2, py = (1.0f / 3.0f) + uy2, pz = (1.0f / 3.0f) + uz2;

    float k[27];
#define K(a, b, c) k[(a) + 3 * (b) + 9 * (c)]
    K(0, 0, 0) = dr;
    K(1, 0, 0) = 0.5f * Fx + ux;
    K(0, 1, 0) = 0.5f * Fy + uy;
    K(0, 0, 1) = 0.5f * Fz + uz;
    K(2, 0, 0) = dr * (1.0f / 3.0f) + r * ex - ux2;
    K(0, 2, 0) = dr * (1.0f / 3.0f) + r * ey - uy2;
    K(0, 0, 2) = dr * (1.0f / 3.0f) + r * ez - uz2;
    K(1, 1, 0) = r * kxy - ux * uy;
    K(1, 0, 1) = r * kxz - ux * uz;
    K(0, 1, 1) = r * kyz - uy * uz;
    // third order: kappa* = 0
    K(2, 1, 0) = uy * px;
    K(2, 0, 1) = uz * px;
    K(1, 2, 0) = ux * py;
    K(0, 2, 1) = uz * py;
    K(1, 0, 2) = ux * pz;
    K(0, 1, 2) = uy * pz;
    K(1, 1, 1) = ux * uy * uz;
    // fourth order: kappa* = rho (K_aa K_bb + 2 k_ab^2), rho (K_aa k_bc + 2 k_ab k_ac)
    K(2, 2, 0) = r * ((ex + ey) * (1.0f / 3.0f) + ex * ey + 2.0f * kxy * kxy) + dr * (1.0f / 9.0f) -
                 (ux2 + uy2) * (1.0f / 3.0f) - ux2 * uy2;
    K(2, 0, 2) = r * ((ex + ez) * (1.0f / 3.0f) + ex * ez + 2.0f * kxz * kxz) + dr * (1.0f / 9.0f) -
                 (ux2 + uz2) * (1.0f / 3.0f) - ux2 * uz2;
    K(0, 2, 2) = r * ((ey + ez) * (1.0f / 3.0f) + ey * ez + 2.0f * kyz * kyz) + dr * (1.0f / 9.0f) -
                 (uy2 + uz2) * (1.0f / 3.0f) - uy2 * uz2;
    K(2, 1, 1) = r * (Kxx * kyz + 2.0f * kxy * kxz) - px * uy * uz;
    K(1, 2, 1) = r * (Kyy * kxz + 2.0f * kxy * kyz) - py * ux * uz;
    K(1, 1, 2) = r * (Kzz * kxy + 2.0f * kxz * kyz) - pz * ux * uy;
    // fifth order: kappa* = 0
    K(2, 2, 1) = uz * px * py;
    K(2, 1, 2) = uy * px * pz;
    K(1, 2, 2) = ux * py * pz;
    // sixth order: rho [Kxx Kyy Kzz + 2 (Kxx kyz^2 + Kyy kxz^2 + Kzz kxy^2) + 8 kxy kxz kyz]
    {
        const float se = ex + ey + ez;
        const float see = ex * ey + ex * ez + ey * ez;
        const float prod_dev = se * (1.0f / 9.0f) + see * (1.0f / 3.0f) + ex * ey * ez;
        const float cross = 2.0f * (Kxx * kyz * kyz + Kyy * kxz * kxz + Kzz * kxy * kxy) + 8.0f * kxy * kxz * kyz;
        const float su = ux2 + uy2 + uz2;
        const float suu = ux2 * uy2 + ux2 * uz2 + uy2 * uz2;
        K(2, 2, 2) = dr * (1.0f / 27.0f) + r * (prod_dev + cross) - su * (1.0f / 9.0f) - suu * (1.0f / 3.0f) -
                     ux2 * uy2 * uz2;
    }
#undef K
    // inverse transform: x lines, then y lines, then z lines
#pragma unroll
    for (int q = 0; q < 9; ++q) inv_triple(k[3 * q], k[3 * q + 1], k[3 * q + 2], ux);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) inv_triple(k[ix + 9 * c], k[ix + 9 * c + 3], k[ix + 9 * c + 6], uy);
#pragma unroll
    for (int p = 0; p < 9; ++p) inv_triple(k[p], k[p + 9], k[p + 18], uz);
#pragma unroll
    for (int i = 0; i < 27; ++i) out[i] = k[i];
}

// ------------------------------------------------------------ general rates
// Collision with arbitrary omega_3..omega_10: the pre-collision cumulants of
// third to sixth order are needed. Central moments of f about u are those of
// the deviations (forward passes on d) plus those of the weights, the
// product of (1, -u, 1/3 + u^2) per axis; cumulants use k = kappa / rho with
// the zero-mean set-partition formulas; after relaxation the moments are
// rebuilt order by order and the weight moments subtracted again before the
// inverse transform, so the output is d* = f* - w.
__device__ __forceinline__ void fwd_triple(float &a, float &b, float &c, float u) {
    const float fm = a, f0 = b, fp = c;
    const float spm = fp + fm, dpm = fp - fm;
    const float k0 = spm + f0;
    b = fmaf(-u, k0, dpm);
    c = fmaf(u * u, k0, fmaf(-2.0f * u, dpm, spm));
    a = k0;
}

__device__ __forceinline__ void collide_general(const float d[27], const CellMoments &m, float omega1, float omega2,
                                                const float *wh, float Fx, float Fy, float Fz, float out[27]) {
    const float ux = m.ux, uy = m.uy, uz = m.uz;
    float k[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = d[i];
#pragma unroll
    for (int p = 0; p < 9; ++p) fwd_triple(k[p], k[p + 9], k[p + 18], uz);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) fwd_triple(k[ix + 9 * c], k[ix + 9 * c + 3], k[ix + 9 * c + 6], uy);
#pragma unroll
    for (int q = 0; q < 9; ++q) fwd_triple(k[3 * q], k[3 * q + 1], k[3 * q + 2], ux);
    // weight moments about u
    const float mx[3] = {1.0f, -ux, 1.0f / 3.0f + ux * ux};
    const float my[3] = {1.0f, -uy, 1.0f / 3.0f + uy * uy};
    const float mz[3] = {1.0f, -uz, 1.0f / 3.0f + uz * uz};
    float kw[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) kw[i] = mx[i % 3] * my[(i / 3) % 3] * mz[i / 9];
    const float rho = m.rho, ir = 1.0f / rho;
    float n[27];  // normalised moments of f (orders >= 2)
#pragma unroll
    for (int i = 0; i < 27; ++i) n[i] = (kw[i] + k[i]) * ir;
#define N(a, b, c) n[(a) + 3 * (b) + 9 * (c)]
    // second order deviations from 1/3 on the diagonal use the accurate forms
    const float exx = m.ex, eyy = m.ey, ezz = m.ez;
    N(2, 0, 0) = 1.0f / 3.0f + exx;
    N(0, 2, 0) = 1.0f / 3.0f + eyy;
    N(0, 0, 2) = 1.0f / 3.0f + ezz;
    N(1, 1, 0) = m.kxy;
    N(1, 0, 1) = m.kxz;
    N(0, 1, 1) = m.kyz;
    // cumulants (orders 4..6 subtract the set-partition products)
    const float c220 = N(2, 2, 0) - (N(2, 0, 0) * N(0, 2, 0) + 2.0f * N(1, 1, 0) * N(1, 1, 0));
    const float c202 = N(2, 0, 2) - (N(2, 0, 0) * N(0, 0, 2) + 2.0f * N(1, 0, 1) * N(1, 0, 1));
    const float c022 = N(0, 2, 2) - (N(0, 2, 0) * N(0, 0, 2) + 2.0f * N(0, 1, 1) * N(0, 1, 1));
    const float c211 = N(2, 1, 1) - (N(2, 0, 0) * N(0, 1, 1) + 2.0f * N(1, 1, 0) * N(1, 0, 1));
    const float c121 = N(1, 2, 1) - (N(0, 2, 0) * N(1, 0, 1) + 2.0f * N(1, 1, 0) * N(0, 1, 1));
    const float c112 = N(1, 1, 2) - (N(0, 0, 2) * N(1, 1, 0) + 2.0f * N(1, 0, 1) * N(0, 1, 1));
    const float c221 = N(2, 2, 1) - (N(2, 0, 0) * N(0, 2, 1) + N(0, 2, 0) * N(2, 0, 1) + 4.0f * N(1, 1, 0) * N(1, 1, 1) +
                                     2.0f * N(1, 0, 1) * N(1, 2, 0) + 2.0f * N(0, 1, 1) * N(2, 1, 0));
    const float c212 = N(2, 1, 2) - (N(2, 0, 0) * N(0, 1, 2) + N(0, 0, 2) * N(2, 1, 0) + 4.0f * N(1, 0, 1) * N(1, 1, 1) +
                                     2.0f * N(1, 1, 0) * N(1, 0, 2) + 2.0f * N(0, 1, 1) * N(2, 0, 1));
    const float c122 = N(1, 2, 2) - (N(0, 2, 0) * N(1, 0, 2) + N(0, 0, 2) * N(1, 2, 0) + 4.0f * N(0, 1, 1) * N(1, 1, 1) +
                                     2.0f * N(1, 1, 0) * N(0, 1, 2) + 2.0f * N(1, 0, 1) * N(0, 2, 1));
    auto s42 = [&](const float *q) {
        return q[2] * q[24] + q[6] * q[20] + q[18] * q[8] +
               4.0f * (q[4] * q[22] + q[10] * q[16] + q[12] * q[14]);
    };
    auto s33 = [&](const float *q) {
        // 4 k111^2 + 2 (k210 k012 + k201 k021 + k120 k102)
        return 4.0f * q[13] * q[13] + 2.0f * (q[5] * q[21] + q[11] * q[15] + q[7] * q[19]);
    };
    auto s222 = [&](const float *q) {
        return q[2] * q[6] * q[18] + 2.0f * (q[2] * q[12] * q[12] + q[6] * q[10] * q[10] + q[18] * q[4] * q[4]) +
               8.0f * q[4] * q[10] * q[12];
    };
    const float c222 = N(2, 2, 2) - s42(n) - s33(n) + 2.0f * s222(n);
    // relaxation (omega_3..omega_10 in wh[0..7])
    const float s1 = 1.0f - omega1;
    float r[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) r[i] = 0.0f;
#define R(a, b, c) r[(a) + 3 * (b) + 9 * (c)]
    {
        const float dxy = s1 * (exx - eyy), dxz = s1 * (exx - ezz), trd = (1.0f - omega2) * (exx + eyy + ezz);
        R(2, 0, 0) = 1.0f / 3.0f + (trd + dxy + dxz) * (1.0f / 3.0f);
        R(0, 2, 0) = 1.0f / 3.0f + (trd - 2.0f * dxy + dxz) * (1.0f / 3.0f);
        R(0, 0, 2) = 1.0f / 3.0f + (trd + dxy - 2.0f * dxz) * (1.0f / 3.0f);
        R(1, 1, 0) = s1 * m.kxy;
        R(1, 0, 1) = s1 * m.kxz;
        R(0, 1, 1) = s1 * m.kyz;
    }
    {
        const float a3 = 1.0f - wh[0], a4 = 1.0f - wh[1];
        // pairs (120, 102), (210, 012), (201, 021): sums with omega_3, differences with omega_4
        const int p0[3] = {1 + 3 * 2, 2 + 3 * 1, 2 + 9 * 1};
        const int p1[3] = {1 + 9 * 2, 3 * 1 + 9 * 2, 3 * 2 + 9 * 1};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float sm = a3 * (n[p0[q]] + n[p1[q]]);
            const float df = a4 * (n[p0[q]] - n[p1[q]]);
            r[p0[q]] = 0.5f * (sm + df);
            r[p1[q]] = 0.5f * (sm - df);
        }
        R(1, 1, 1) = (1.0f - wh[2]) * N(1, 1, 1);
    }
    float C220, C202, C022;
    {
        const float a6 = 1.0f - wh[3], a7 = 1.0f - wh[4];
        const float A = a6 * (c220 - 2.0f * c202 + c022), B = a6 * (c220 + c202 - 2.0f * c022);
        const float S = a7 * (c220 + c202 + c022);
        C220 = (S + A + B) * (1.0f / 3.0f);
        C202 = (S - A) * (1.0f / 3.0f);
        C022 = (S - B) * (1.0f / 3.0f);
    }
    const float a8 = 1.0f - wh[5], a9 = 1.0f - wh[6], a10 = 1.0f - wh[7];
    // rebuild post-collision normalised moments, lower orders first
    R(2, 2, 0) = C220 + R(2, 0, 0) * R(0, 2, 0) + 2.0f * R(1, 1, 0) * R(1, 1, 0);
    R(2, 0, 2) = C202 + R(2, 0, 0) * R(0, 0, 2) + 2.0f * R(1, 0, 1) * R(1, 0, 1);
    R(0, 2, 2) = C022 + R(0, 2, 0) * R(0, 0, 2) + 2.0f * R(0, 1, 1) * R(0, 1, 1);
    R(2, 1, 1) = a8 * c211 + R(2, 0, 0) * R(0, 1, 1) + 2.0f * R(1, 1, 0) * R(1, 0, 1);
    R(1, 2, 1) = a8 * c121 + R(0, 2, 0) * R(1, 0, 1) + 2.0f * R(1, 1, 0) * R(0, 1, 1);
    R(1, 1, 2) = a8 * c112 + R(0, 0, 2) * R(1, 1, 0) + 2.0f * R(1, 0, 1) * R(0, 1, 1);
    R(2, 2, 1) = a9 * c221 + R(2, 0, 0) * R(0, 2, 1) + R(0, 2, 0) * R(2, 0, 1) + 4.0f * R(1, 1, 0) * R(1, 1, 1) +
                 2.0f * R(1, 0, 1) * R(1, 2, 0) + 2.0f * R(0, 1, 1) * R(2, 1, 0);
    R(2, 1, 2) = a9 * c212 + R(2, 0, 0) * R(0, 1, 2) + R(0, 0, 2) * R(2, 1, 0) + 4.0f * R(1, 0, 1) * R(1, 1, 1) +
                 2.0f * R(1, 1, 0) * R(1, 0, 2) + 2.0f * R(0, 1, 1) * R(2, 0, 1);
    R(1, 2, 2) = a9 * c122 + R(0, 2, 0) * R(1, 0, 2) + R(0, 0, 2) * R(1, 2, 0) + 4.0f * R(0, 1, 1) * R(1, 1, 1) +
                 2.0f * R(1, 1, 0) * R(0, 1, 2) + 2.0f * R(1, 0, 1) * R(0, 2, 1);
    R(2, 2, 2) = a10 * c222 + s42(r) + s33(r) - 2.0f * s222(r);
    // kappa* - kappa_w: orders >= 2 as rho r - kw; order 0 and 1 directly
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = rho * r[i] - kw[i];
    k[0] = m.drho;
    k[1] = 0.5f * Fx + ux;
    k[3] = 0.5f * Fy + uy;
    k[9] = 0.5f * Fz + uz;
    // the second-order diagonal in its accurate form: rho (1/3 + e*) - (1/3 + u^2)
    k[2] = m.drho * (1.0f / 3.0f) + rho * (R(2, 0, 0) - 1.0f / 3.0f) - ux * ux;
    k[6] = m.drho * (1.0f / 3.0f) + rho * (R(0, 2, 0) - 1.0f / 3.0f) - uy * uy;
    k[18] = m.drho * (1.0f / 3.0f) + rho * (R(0, 0, 2) - 1.0f / 3.0f) - uz * uz;
#undef N
#undef R
#pragma unroll
    for (int q = 0; q < 9; ++q) inv_triple(k[3 * q], k[3 * q + 1], k[3 * q + 2], ux);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) inv_triple(k[ix + 9 * c], k[ix + 9 * c + 3], k[ix + 9 * c + 6], uy);
#pragma unroll
    for (int p = 0; p < 9; ++p) inv_triple(k[p], k[p + 9], k[p + 18], uz);
#pragma unroll
    for (int i = 0; i < 27; ++i) out[i] = k[i];
}

}  // namespace lbm
