/*
 * Learned eddy-viscosity closure, forward pass, FP64.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper runs an LES (Sec. 1) but names no subgrid model; this closure is
 * an extension beyond the paper: a per-cell network 6 -> 32 -> 32 -> 1 with
 * ReLU hidden layers and a softplus output, fed the invariants of the
 * non-equilibrium stress, that returns an eddy viscosity.
 *
 * Parameter blob (ORC_MLP_NBLOB doubles, row-major matrices):
 *   W1[32][6] b1[32] W2[32][32] b2[32] w3[32] b3 mu[6] sigma[6] nu_scale
 *
 * emulate_bf16 = 1 reproduces the roundings of a bfloat16 matrix-core
 * evaluation: the normalised inputs are formed in float32 as
 * (x - mu) * (1/sigma) and rounded to bfloat16, W1, W2 and the first hidden
 * layer are rounded to bfloat16, the other parameters to float32; the
 * arithmetic itself stays FP64.
 */
#include "orc.h"
#include <math.h>
#include <stdint.h>
#include <string.h>

#define OFF_W1 0
#define OFF_B1 192
#define OFF_W2 224
#define OFF_B2 1248
#define OFF_W3 1280
#define OFF_B3 1312
#define OFF_MU 1313
#define OFF_SG 1319
#define OFF_NS 1325

/* round to float32, then to bfloat16 with round-to-nearest-even */
double orc_bf16_round(double x)
{
    float f = (float)x;
    uint32_t bits;
    memcpy(&bits, &f, 4);
    if ((bits & 0x7f800000u) == 0x7f800000u)
        return (double)f; /* inf / nan unchanged */
    uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7fffu + lsb;
    bits &= 0xffff0000u;
    memcpy(&f, &bits, 4);
    return (double)f;
}

static double fr(double x, int emu) { return emu ? (double)(float)x : x; }
static double br(double x, int emu) { return emu ? orc_bf16_round(x) : x; }

static double softplus(double z)
{
    return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
}

double orc_mlp_nu_t(const double *blob, const double feat[6], int emu)
{
    double xh[6], h1[32], h2[32];
    for (int j = 0; j < 6; ++j) {
        if (emu) {
            float d = (float)feat[j] - (float)blob[OFF_MU + j];
            float is = (float)(1.0 / blob[OFF_SG + j]);
            float v = d * is;
            xh[j] = orc_bf16_round((double)v);
        } else {
            xh[j] = (feat[j] - blob[OFF_MU + j]) / blob[OFF_SG + j];
        }
    }
    for (int o = 0; o < 32; ++o) {
        double s = fr(blob[OFF_B1 + o], emu);
        for (int j = 0; j < 6; ++j)
            s += br(blob[OFF_W1 + 6 * o + j], emu) * xh[j];
        h1[o] = br(s > 0.0 ? s : 0.0, emu);
    }
    for (int o = 0; o < 32; ++o) {
        double s = fr(blob[OFF_B2 + o], emu);
        for (int k = 0; k < 32; ++k)
            s += br(blob[OFF_W2 + 32 * o + k], emu) * h1[k];
        h2[o] = s > 0.0 ? s : 0.0;
    }
    double z = fr(blob[OFF_B3], emu);
    for (int o = 0; o < 32; ++o)
        z += fr(blob[OFF_W3 + o], emu) * h2[o];
    return fr(blob[OFF_NS], emu) * softplus(z);
}

/* omega_1 from the total viscosity: nu0 = (1/omega0 - 1/2)/3 and
 * omega_1 = 1 / (3 (nu0 + nu_t) + 1/2). */
double orc_mlp_omega(const double *blob, const double kappa[ORC_Q], double omega0,
                     int emu)
{
    double feat[6];
    orc_closure_features(kappa, omega0, feat);
    double nut = orc_mlp_nu_t(blob, feat, emu);
    double nu0 = (1.0 / omega0 - 0.5) / 3.0;
    return 1.0 / (3.0 * (nu0 + nut) + 0.5);
}
