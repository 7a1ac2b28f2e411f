/*
 * Single-cell building blocks of the D3Q27 cumulant collision, FP64.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper fixes the velocity set (D3Q27, Sec. 2.1), the lattice Boltzmann
 * update with a collision and a Guo-type force source (Sec. 2.1, eq. (1)),
 * and names the cumulant collision of Geier et al. (2015) without printing
 * its equations (Sec. 2.1). The cumulant algebra below is therefore written
 * from the definition of joint cumulants of the 27-point distribution, with
 * the readings stated at each function.
 */
#include "orc.h"
#include <math.h>
#include <string.h>

#define M(a, b, c) ((a) + 3 * (b) + 9 * (c))

/* one-dimensional weights of the D3Q27 product lattice: w(0)=2/3, w(+-1)=1/6 */
static const double W1D[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};

/* D3Q27 velocity set and weights (Sec. 2.1): all 27 vectors in {-1,0,1}^3;
 * the weights are the tensor product of the 1-D weights, giving 8/27, 2/27,
 * 1/54 and 1/216 for rest, face, edge and corner directions. */
void orc_lattice(int c[ORC_Q][3], double w[ORC_Q])
{
    for (int i = 0; i < ORC_Q; ++i) {
        int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
        c[i][0] = cx;
        c[i][1] = cy;
        c[i][2] = cz;
        w[i] = W1D[cx + 1] * W1D[cy + 1] * W1D[cz + 1];
    }
}

/* One factor of the product equilibrium: the 1-D distribution over {-1,0,1}
 * with zeroth, first and second moments 1, u and u^2 + 1/3. */
static double phi(int c, double u)
{
    if (c == 0)
        return 2.0 / 3.0 - u * u;
    return 0.5 * (1.0 / 3.0 + u * u + c * u);
}

/* Equilibrium (reading: the state the cumulant collision returns when every
 * relaxation rate is 1 and there is no force, i.e. second-order cumulants at
 * c_s^2 and all higher cumulants zero). On D3Q27 this is the product of three
 * 1-D distributions. Used for initialisation and for the inlet. */
void orc_feq(double rho, const double u[3], double f[ORC_Q])
{
    for (int i = 0; i < ORC_Q; ++i) {
        int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
        f[i] = rho * phi(cx, u[0]) * phi(cy, u[1]) * phi(cz, u[2]);
    }
}

/* Central moments by definition:
 *   kappa_abc = sum_i (c_ix-u_x)^a (c_iy-u_y)^b (c_iz-u_z)^c f_i. */
void orc_central_moments_direct(const double f[ORC_Q], const double u[3],
                                double kappa[ORC_Q])
{
    for (int m = 0; m < ORC_Q; ++m) {
        int a = m % 3, b = (m / 3) % 3, c = m / 9;
        double s = 0.0;
        for (int i = 0; i < ORC_Q; ++i) {
            double dx = (i % 3 - 1) - u[0];
            double dy = ((i / 3) % 3 - 1) - u[1];
            double dz = (i / 9 - 1) - u[2];
            s += pow(dx, a) * pow(dy, b) * pow(dz, c) * f[i];
        }
        kappa[m] = s;
    }
}

/* The same central moments, taken one axis at a time: along each lattice line
 * of three values (f-, f0, f+) the zeroth, first and second moments about u
 * are formed and replace the three values in place. Because the velocity and
 * moment indices share the digit layout, after the z, y and x passes the
 * array holds kappa[a + 3b + 9c]. */
static void fwd1d(double *v, int stride, double u)
{
    double fm = v[0], f0 = v[stride], fp = v[2 * stride];
    double k0 = fm + f0 + fp;
    double k1 = (fp - fm) - u * k0;
    double k2 = (fp + fm) - 2.0 * u * (fp - fm) + u * u * k0;
    v[0] = k0;
    v[stride] = k1;
    v[2 * stride] = k2;
}

void orc_central_moments(const double f[ORC_Q], const double u[3],
                         double kappa[ORC_Q])
{
    memcpy(kappa, f, sizeof(double) * ORC_Q);
    for (int p = 0; p < 9; ++p) /* z lines: base p = ix + 3 iy */
        fwd1d(kappa + p, 9, u[2]);
    for (int c = 0; c < 3; ++c) /* y lines: base ix + 9c */
        for (int ix = 0; ix < 3; ++ix)
            fwd1d(kappa + ix + 9 * c, 3, u[1]);
    for (int q = 0; q < 9; ++q) /* x lines: base 3b + 9c */
        fwd1d(kappa + 3 * q, 1, u[0]);
}

/* Inverse of one 1-D pass: central moments (k0,k1,k2) about u give the raw
 * moments m0 = k0, m1 = k1 + u k0, m2 = k2 + 2u k1 + u^2 k0, and the three
 * populations follow from m0 = f-+f0+f+, m1 = f+-f-, m2 = f++f-. */
static void inv1d(double *v, int stride, double u)
{
    double k0 = v[0], k1 = v[stride], k2 = v[2 * stride];
    double m0 = k0;
    double m1 = k1 + u * k0;
    double m2 = k2 + 2.0 * u * k1 + u * u * k0;
    v[0] = 0.5 * (m2 - m1);
    v[stride] = m0 - m2;
    v[2 * stride] = 0.5 * (m2 + m1);
}

void orc_central_to_pops(const double kappa[ORC_Q], const double u[3],
                         double f[ORC_Q])
{
    memcpy(f, kappa, sizeof(double) * ORC_Q);
    for (int q = 0; q < 9; ++q)
        inv1d(f + 3 * q, 1, u[0]);
    for (int c = 0; c < 3; ++c)
        for (int ix = 0; ix < 3; ++ix)
            inv1d(f + ix + 9 * c, 3, u[1]);
    for (int p = 0; p < 9; ++p)
        inv1d(f + p, 9, u[2]);
}

/* Sums of products of normalised moments k that the joint-cumulant
 * expansion of the sixth-order moment needs (pairs with fourth order,
 * triple with triple, and three pairs). */
static double s42(const double *k)
{
    return k[M(2, 0, 0)] * k[M(0, 2, 2)] + k[M(0, 2, 0)] * k[M(2, 0, 2)] +
           k[M(0, 0, 2)] * k[M(2, 2, 0)] +
           4.0 * (k[M(1, 1, 0)] * k[M(1, 1, 2)] + k[M(1, 0, 1)] * k[M(1, 2, 1)] +
                  k[M(0, 1, 1)] * k[M(2, 1, 1)]);
}
static double s33(const double *k)
{
    return 4.0 * k[M(1, 1, 1)] * k[M(1, 1, 1)] +
           2.0 * (k[M(2, 1, 0)] * k[M(0, 1, 2)] + k[M(2, 0, 1)] * k[M(0, 2, 1)] +
                  k[M(1, 2, 0)] * k[M(1, 0, 2)]);
}
static double s222(const double *k)
{
    double kxx = k[M(2, 0, 0)], kyy = k[M(0, 2, 0)], kzz = k[M(0, 0, 2)];
    double kxy = k[M(1, 1, 0)], kxz = k[M(1, 0, 1)], kyz = k[M(0, 1, 1)];
    return kxx * kyy * kzz + 2.0 * (kxx * kyz * kyz + kyy * kxz * kxz + kzz * kxy * kxy) +
           8.0 * kxy * kxz * kyz;
}

/* Fourth- and fifth-order "pair x rest" sums for one index pattern, shared by
 * the forward and inverse maps: for the moment with exponents (a,b,c) these
 * are the partitions of the multiset into one pair and one block of the rest. */
static double pairs4_220(const double *k) /* XXYY */
{
    return k[M(2, 0, 0)] * k[M(0, 2, 0)] + 2.0 * k[M(1, 1, 0)] * k[M(1, 1, 0)];
}
static double pairs4_202(const double *k) /* XXZZ */
{
    return k[M(2, 0, 0)] * k[M(0, 0, 2)] + 2.0 * k[M(1, 0, 1)] * k[M(1, 0, 1)];
}
static double pairs4_022(const double *k) /* YYZZ */
{
    return k[M(0, 2, 0)] * k[M(0, 0, 2)] + 2.0 * k[M(0, 1, 1)] * k[M(0, 1, 1)];
}
static double pairs4_211(const double *k) /* XXYZ */
{
    return k[M(2, 0, 0)] * k[M(0, 1, 1)] + 2.0 * k[M(1, 1, 0)] * k[M(1, 0, 1)];
}
static double pairs4_121(const double *k) /* XYYZ */
{
    return k[M(0, 2, 0)] * k[M(1, 0, 1)] + 2.0 * k[M(1, 1, 0)] * k[M(0, 1, 1)];
}
static double pairs4_112(const double *k) /* XYZZ */
{
    return k[M(0, 0, 2)] * k[M(1, 1, 0)] + 2.0 * k[M(1, 0, 1)] * k[M(0, 1, 1)];
}
static double pairs5_221(const double *k) /* XXYYZ: pair + triple */
{
    return k[M(2, 0, 0)] * k[M(0, 2, 1)] + k[M(0, 2, 0)] * k[M(2, 0, 1)] +
           4.0 * k[M(1, 1, 0)] * k[M(1, 1, 1)] + 2.0 * k[M(1, 0, 1)] * k[M(1, 2, 0)] +
           2.0 * k[M(0, 1, 1)] * k[M(2, 1, 0)];
}
static double pairs5_212(const double *k) /* XXYZZ */
{
    return k[M(2, 0, 0)] * k[M(0, 1, 2)] + k[M(0, 0, 2)] * k[M(2, 1, 0)] +
           4.0 * k[M(1, 0, 1)] * k[M(1, 1, 1)] + 2.0 * k[M(1, 1, 0)] * k[M(1, 0, 2)] +
           2.0 * k[M(0, 1, 1)] * k[M(2, 0, 1)];
}
static double pairs5_122(const double *k) /* XYYZZ */
{
    return k[M(0, 2, 0)] * k[M(1, 0, 2)] + k[M(0, 0, 2)] * k[M(1, 2, 0)] +
           4.0 * k[M(0, 1, 1)] * k[M(1, 1, 1)] + 2.0 * k[M(1, 1, 0)] * k[M(0, 1, 2)] +
           2.0 * k[M(1, 0, 1)] * k[M(0, 2, 1)];
}

static int order_of(int m) { return m % 3 + (m / 3) % 3 + m / 9; }

/* Cumulants from central moments. Reading of the cumulant operator named in
 * Sec. 2.1 (Geier et al. 2015): with k = kappa/rho the normalised central
 * moments, orders two and three equal k, and orders four to six subtract the
 * products over the set partitions of the index multiset into blocks of size
 * at least two (first-order central moments are treated as zero in these
 * products, also when a body force makes them -F/2). Orders 0 and 1 are
 * passed through unnormalised: C[0] = rho and C[first] = kappa[first]. */
void orc_cumulants(const double kappa[ORC_Q], double C[ORC_Q])
{
    double rho = kappa[0];
    double k[ORC_Q];
    for (int m = 0; m < ORC_Q; ++m)
        k[m] = kappa[m] / rho;
    for (int m = 0; m < ORC_Q; ++m)
        C[m] = order_of(m) < 2 ? kappa[m] : k[m];
    C[M(2, 2, 0)] = k[M(2, 2, 0)] - pairs4_220(k);
    C[M(2, 0, 2)] = k[M(2, 0, 2)] - pairs4_202(k);
    C[M(0, 2, 2)] = k[M(0, 2, 2)] - pairs4_022(k);
    C[M(2, 1, 1)] = k[M(2, 1, 1)] - pairs4_211(k);
    C[M(1, 2, 1)] = k[M(1, 2, 1)] - pairs4_121(k);
    C[M(1, 1, 2)] = k[M(1, 1, 2)] - pairs4_112(k);
    C[M(2, 2, 1)] = k[M(2, 2, 1)] - pairs5_221(k);
    C[M(2, 1, 2)] = k[M(2, 1, 2)] - pairs5_212(k);
    C[M(1, 2, 2)] = k[M(1, 2, 2)] - pairs5_122(k);
    C[M(2, 2, 2)] = k[M(2, 2, 2)] - s42(k) - s33(k) + 2.0 * s222(k);
}

/* Inverse of orc_cumulants: rebuild the normalised moments order by order
 * from the (post-collision) cumulants and the already rebuilt lower orders,
 * then scale by rho. C[0] is rho; first-order entries are copied. */
void orc_cumulants_inverse(const double C[ORC_Q], double kappa[ORC_Q])
{
    double rho = C[0];
    double k[ORC_Q];
    for (int m = 0; m < ORC_Q; ++m)
        k[m] = C[m];
    k[M(2, 2, 0)] = C[M(2, 2, 0)] + pairs4_220(k);
    k[M(2, 0, 2)] = C[M(2, 0, 2)] + pairs4_202(k);
    k[M(0, 2, 2)] = C[M(0, 2, 2)] + pairs4_022(k);
    k[M(2, 1, 1)] = C[M(2, 1, 1)] + pairs4_211(k);
    k[M(1, 2, 1)] = C[M(1, 2, 1)] + pairs4_121(k);
    k[M(1, 1, 2)] = C[M(1, 1, 2)] + pairs4_112(k);
    k[M(2, 2, 1)] = C[M(2, 2, 1)] + pairs5_221(k);
    k[M(2, 1, 2)] = C[M(2, 1, 2)] + pairs5_212(k);
    k[M(1, 2, 2)] = C[M(1, 2, 2)] + pairs5_122(k);
    k[M(2, 2, 2)] = C[M(2, 2, 2)] + s42(k) + s33(k) - 2.0 * s222(k);
    for (int m = 0; m < ORC_Q; ++m)
        kappa[m] = order_of(m) < 2 ? C[m] : rho * k[m];
}

/* Relaxation of the cumulants (reading of the cumulant operator of Sec. 2.1;
 * omega[0..9] are the rates omega_1..omega_10):
 *   2nd order: off-diagonal and the two normal-stress differences with
 *              omega_1; the trace towards its equilibrium 1 with omega_2;
 *   3rd order: the three sums C120+C102, C210+C012, C201+C021 with omega_3,
 *              the matching differences with omega_4, C111 with omega_5;
 *   4th order: C220-2C202+C022 and C220+C202-2C022 with omega_6, their sum
 *              with omega_7, C211, C121, C112 with omega_8;
 *   5th order with omega_9, 6th order with omega_10; equilibrium value 0.
 * Orders 0 and 1 are returned unchanged. */
void orc_relax(const double C[ORC_Q], const double omega[10], double Cs[ORC_Q])
{
    double w1 = omega[0], w2 = omega[1], w3 = omega[2], w4 = omega[3];
    double w5 = omega[4], w6 = omega[5], w7 = omega[6], w8 = omega[7];
    double w9 = omega[8], w10 = omega[9];
    memcpy(Cs, C, sizeof(double) * ORC_Q);

    Cs[M(1, 1, 0)] = (1.0 - w1) * C[M(1, 1, 0)];
    Cs[M(1, 0, 1)] = (1.0 - w1) * C[M(1, 0, 1)];
    Cs[M(0, 1, 1)] = (1.0 - w1) * C[M(0, 1, 1)];
    double dxy = C[M(2, 0, 0)] - C[M(0, 2, 0)];
    double dxz = C[M(2, 0, 0)] - C[M(0, 0, 2)];
    double tr = C[M(2, 0, 0)] + C[M(0, 2, 0)] + C[M(0, 0, 2)];
    dxy *= (1.0 - w1);
    dxz *= (1.0 - w1);
    tr += w2 * (1.0 - tr);
    Cs[M(2, 0, 0)] = (tr + dxy + dxz) / 3.0;
    Cs[M(0, 2, 0)] = (tr - 2.0 * dxy + dxz) / 3.0;
    Cs[M(0, 0, 2)] = (tr + dxy - 2.0 * dxz) / 3.0;

    /* third order: pairs (p, q) relaxed as (p+q) with w3 and (p-q) with w4 */
    const int pairs[3][2] = {{M(1, 2, 0), M(1, 0, 2)},
                             {M(2, 1, 0), M(0, 1, 2)},
                             {M(2, 0, 1), M(0, 2, 1)}};
    for (int n = 0; n < 3; ++n) {
        double s = C[pairs[n][0]] + C[pairs[n][1]];
        double d = C[pairs[n][0]] - C[pairs[n][1]];
        s *= (1.0 - w3);
        d *= (1.0 - w4);
        Cs[pairs[n][0]] = 0.5 * (s + d);
        Cs[pairs[n][1]] = 0.5 * (s - d);
    }
    Cs[M(1, 1, 1)] = (1.0 - w5) * C[M(1, 1, 1)];

    double a = C[M(2, 2, 0)] - 2.0 * C[M(2, 0, 2)] + C[M(0, 2, 2)];
    double b = C[M(2, 2, 0)] + C[M(2, 0, 2)] - 2.0 * C[M(0, 2, 2)];
    double s = C[M(2, 2, 0)] + C[M(2, 0, 2)] + C[M(0, 2, 2)];
    a *= (1.0 - w6);
    b *= (1.0 - w6);
    s *= (1.0 - w7);
    Cs[M(2, 2, 0)] = (s + a + b) / 3.0;
    Cs[M(2, 0, 2)] = (s - a) / 3.0;
    Cs[M(0, 2, 2)] = (s - b) / 3.0;
    Cs[M(2, 1, 1)] = (1.0 - w8) * C[M(2, 1, 1)];
    Cs[M(1, 2, 1)] = (1.0 - w8) * C[M(1, 2, 1)];
    Cs[M(1, 1, 2)] = (1.0 - w8) * C[M(1, 1, 2)];

    Cs[M(2, 2, 1)] = (1.0 - w9) * C[M(2, 2, 1)];
    Cs[M(2, 1, 2)] = (1.0 - w9) * C[M(2, 1, 2)];
    Cs[M(1, 2, 2)] = (1.0 - w9) * C[M(1, 2, 2)];
    Cs[M(2, 2, 2)] = (1.0 - w10) * C[M(2, 2, 2)];
}

/* One collision with force (Sec. 2.1, eq. (1) and the moment definitions):
 *   rho = sum f, j = sum c f, u = (j + F/2)/rho  (the printed "F dt/(2 rho)"
 *   is read as F dt/2 inside rho u, the only dimensionally consistent form);
 *   central moments about u -> cumulants -> relaxation -> inverse.
 * Forcing (reading of the Guo model in central-moment form): the velocity
 * shift above makes the pre-collision first-order central moments -F/2; the
 * collision sets them to +F/2, so the momentum grows by exactly F. */
void orc_collide(const double f[ORC_Q], const double F[3],
                 const double omega[10], double fout[ORC_Q])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < ORC_Q; ++i) {
        rho += f[i];
        j[0] += (i % 3 - 1) * f[i];
        j[1] += ((i / 3) % 3 - 1) * f[i];
        j[2] += (i / 9 - 1) * f[i];
    }
    double u[3];
    for (int d = 0; d < 3; ++d)
        u[d] = (j[d] + 0.5 * F[d]) / rho;
    double kappa[ORC_Q], C[ORC_Q], Cs[ORC_Q];
    orc_central_moments(f, u, kappa);
    orc_cumulants(kappa, C);
    orc_relax(C, omega, Cs);
    Cs[M(1, 0, 0)] = 0.5 * F[0];
    Cs[M(0, 1, 0)] = 0.5 * F[1];
    Cs[M(0, 0, 1)] = 0.5 * F[2];
    orc_cumulants_inverse(Cs, kappa);
    orc_central_to_pops(kappa, u, fout);
}

/* Deviatoric part of the normalised non-equilibrium second moment,
 * P = dev(kappa_2/rho - I/3), and its norm Q = sqrt(P:P). */
static double q_norm(const double kappa[ORC_Q], double A[3][3])
{
    double rho = kappa[0];
    A[0][0] = kappa[M(2, 0, 0)] / rho - 1.0 / 3.0;
    A[1][1] = kappa[M(0, 2, 0)] / rho - 1.0 / 3.0;
    A[2][2] = kappa[M(0, 0, 2)] / rho - 1.0 / 3.0;
    A[0][1] = A[1][0] = kappa[M(1, 1, 0)] / rho;
    A[0][2] = A[2][0] = kappa[M(1, 0, 1)] / rho;
    A[1][2] = A[2][1] = kappa[M(0, 1, 1)] / rho;
    double tr3 = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    double q2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double p = A[a][b] - (a == b ? tr3 : 0.0);
            q2 += p * p;
        }
    return sqrt(q2);
}

/* Smagorinsky eddy viscosity in the closed form of Hou et al. (1996), filter
 * width one cell: the LES of the paper (Sec. 1) names no subgrid model, so
 * this is the reading used for the fallback closure. With tau0 = 1/omega0 and
 * Q the norm of the deviatoric non-equilibrium stress per unit density,
 * tau = (tau0 + sqrt(tau0^2 + 18 sqrt(2) Cs^2 Q)) / 2 and omega_1 = 1/tau. */
double orc_smagorinsky_omega(const double kappa[ORC_Q], double omega0, double cs)
{
    double A[3][3];
    double q = q_norm(kappa, A);
    double tau0 = 1.0 / omega0;
    double tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * q));
    return 1.0 / tau;
}

/* Inputs of the learned closure: the three invariants of A = Pi_neq/rho,
 * Q, rho - 1, and the Smagorinsky eddy viscosity for Cs = 0.1. */
void orc_closure_features(const double kappa[ORC_Q], double omega0, double feat[6])
{
    double A[3][3];
    double q = q_norm(kappa, A);
    double i1 = A[0][0] + A[1][1] + A[2][2];
    double trA2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            trA2 += A[a][b] * A[b][a];
    double i2 = 0.5 * (i1 * i1 - trA2);
    double i3 = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double tau0 = 1.0 / omega0;
    double tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * 0.01 * q));
    feat[0] = i1;
    feat[1] = i2;
    feat[2] = i3;
    feat[3] = q;
    feat[4] = kappa[0] - 1.0;
    feat[5] = (tau - tau0) / 3.0;
}
