// Device math of the HWENO-GR scheme (arXiv 2608.10569): gas physics,
// characteristic bases, the scalar unified-stencil HWENO reconstruction and
// the positivity-preserving flux bound.  FP64 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hweno_gen.h"

namespace hw {

// The hardware hands a launch's blocks to the 8 XCDs round-robin, and each
// XCD has its own L2.  With xcd set, XCD x takes the contiguous range x of the
// logical blocks, so blocks of neighbouring rows (which share stencil rows)
// run on the same XCD; with rev each XCD takes its range last first.  A
// bijection of [0, nb).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb, bool rev) {
    const int q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int x = b % NUM_XCD, k = b / NUM_XCD;
    const int len = q + (x < r ? 1 : 0);
    return x * q + (x < r ? x : r) + (rev ? len - 1 - k : k);
}

// ---------------------------------------------------------------------------
// Quadrature (Sec. 2.1: 4-point Legendre-Gauss-Lobatto; Sec. 3.1: 3-point
// Gauss per direction), scaled to the unit cell [-1/2, 1/2].
// ---------------------------------------------------------------------------
constexpr double LGL_T = 0.22360679774997896;   // sqrt(5)/10
constexpr double LGL_W0 = 1.0 / 12.0;           // end points
constexpr double LGL_W1 = 5.0 / 12.0;           // interior points
constexpr double GS = 0.3872983346207417;       // sqrt(15)/10
constexpr double GS2 = 0.15;                    // GS^2
constexpr double GS3 = 0.05809475019311125;     // GS^3
constexpr double GS4 = 0.0225;                  // GS^4
constexpr double GW0 = 5.0 / 18.0;              // outer Gauss weight
constexpr double GW1 = 4.0 / 9.0;               // centre Gauss weight

// Linear weights of the nonlinear combination (eqs. (A.3), (A.6)).
constexpr double G1D_0 = 199.0 / 200.0;
constexpr double G1D_1 = 1.0 / 400.0;
constexpr double G2D_0 = 99.0 / 100.0;
constexpr double G2D_1 = 1.0 / 400.0;

// Scheme constants shared by every kernel of one grid.
struct Consts {
    double gamma, gm1, igm1;    // ratio of specific heats, gamma - 1, 1 / (gamma - 1)
    double Pr, gPr;             // Prandtl number, gamma / Pr
    double mu_ref, mu_exp, T_ref;   // mu(T) = mu_ref (T/T_ref)^mu_exp, T = p/rho
    double eps_pp, eps_weno;
    int linear;                 // 1: omega = gamma (test mode)
    int linear_grad;            // 1: omega = gamma in the gradient reconstruction only
    int dr;                     // 1: viscous gradients by the comparison scheme (HWENO-DR)
    double dx, dy, idx, idy;    // cell sizes and inverses
};

__device__ __forceinline__ double dabs(double x) { return fabs(x); }

// 1/d for normal d of either sign: the hardware reciprocal estimate refined by
// two Newton steps r <- r + r (1 - d r) (within an ulp of the correctly
// rounded reciprocal; about half the instructions of an IEEE division).  Used
// where d is a density, a sound speed or a sum of positive terms.
__device__ __forceinline__ double rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Constants of the gradient reconstruction: linear weights also when only the
// gradients are asked to use them.
__device__ __forceinline__ Consts grad_consts(const Consts& K) {
    Consts G = K;
    G.linear = K.linear | K.linear_grad;
    return G;
}

// mu(T) = mu_ref (T / T_ref)^mu_exp.  VarMu = false builds code that serves
// constant viscosity only (mu_exp = 0 in every instance of a launch): the
// power law, and the registers its code needs, stay out of such kernels.
template <bool VarMu = true>
__device__ __forceinline__ double viscosity(const Consts& K, double rho, double p) {
    if (!VarMu || K.mu_exp == 0.0) return K.mu_ref;
    return K.mu_ref * pow((p / rho) / K.T_ref, K.mu_exp);
}

// ---------------------------------------------------------------------------
// Scalar HWENO, 1D (Appendix A.1).  Input a[5] = {abar0_{i-1}, abar0_i,
// abar0_{i+1}, abar1_{i-1}, abar1_{i+1}}; output: coefficients C[5] (powers
// of xi) of the nonlinear combination of eq. (2.4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void hweno1d(const double* __restrict__ a, const Consts& K,
                                        double* __restrict__ C) {
    double c0[5];
    hweno_gen::p0_1d(a, c0);
    const double s1 = a[1] - a[0];      // p1 slope on {i-1, i}
    const double s2 = a[2] - a[1];      // p2 slope on {i, i+1}
    double w0 = G1D_0, w1 = G1D_1, w2 = G1D_1;
    if (!K.linear) {
        const double b0 = hweno_gen::sobolev_1d(c0);
        const double b1 = s1 * s1, b2 = s2 * s2;
        double tau = 0.5 * (dabs(b0 - b1) + dabs(b0 - b2));
        tau = tau * tau;
        const double t0 = G1D_0 * (1.0 + tau / (b0 + K.eps_weno));
        const double t1 = G1D_1 * (1.0 + tau / (b1 + K.eps_weno));
        const double t2 = G1D_1 * (1.0 + tau / (b2 + K.eps_weno));
        const double tot = t0 + t1 + t2;
        w0 = t0 / tot;
        w1 = t1 / tot;
        w2 = t2 / tot;
    }
    const double r0 = w0 / G1D_0;
    const double d1 = w1 - w0 * G1D_1 / G1D_0;
    const double d2 = w2 - w0 * G1D_1 / G1D_0;
#pragma unroll
    for (int k = 0; k < 5; ++k) C[k] = r0 * c0[k];
    C[0] += (d1 + d2) * a[1];
    C[1] += d1 * s1 + d2 * s2;
}

// Values at the four LGL points (-1/2, -t, t, 1/2) and the scaled moment.
__device__ __forceinline__ void eval1d(const double* __restrict__ C, double* __restrict__ v) {
    const double eh = C[0] + C[2] * 0.25 + C[4] * 0.0625;
    const double oh = C[1] * 0.5 + C[3] * 0.125;
    const double t2 = LGL_T * LGL_T;
    const double et = C[0] + t2 * (C[2] + t2 * C[4]);
    const double ot = LGL_T * (C[1] + t2 * C[3]);
    v[0] = eh - oh;
    v[1] = et - ot;
    v[2] = et + ot;
    v[3] = eh + oh;
}
__device__ __forceinline__ double moment1d(const double* __restrict__ C) {
    return C[1] * (1.0 / 12.0) + C[3] * (1.0 / 80.0);
}
// d/dxi at the four LGL points: with C the combination of eq. (2.4), the
// derivative of eq. (2.5) (the candidates differentiated, the weights kept).
__device__ __forceinline__ void deval1d(const double* __restrict__ C, double* __restrict__ v) {
    const double t2 = LGL_T * LGL_T;
    const double eh = C[1] + 0.75 * C[3];           // even part of p' at |xi| = 1/2
    const double oh = C[2] + 0.5 * C[4];            // odd part
    const double et = C[1] + 3.0 * t2 * C[3];
    const double ot = LGL_T * (2.0 * C[2] + 4.0 * t2 * C[4]);
    v[0] = eh - oh;
    v[1] = et - ot;
    v[2] = et + ot;
    v[3] = eh + oh;
}

// ---------------------------------------------------------------------------
// Scalar HWENO, 2D (Appendix A.2).  Input a[17] (averages of cells 1..9,
// xi-moments of 2,4,6,8, eta-moments of 2,4,6,8; cells row-major from
// (i-1, j-1)); output coefficients C[15] of the combination of eq. (3.4).
// Linear candidates (eq. (A.5)) on S1={2,4,5}, S2={2,5,6}, S3={4,5,8},
// S4={5,6,8}: p_m = abar_5 + sx*xi + sy*eta.
// ---------------------------------------------------------------------------
// monomial index of xi^a eta^b
#define MI(a, b) ((((a) + (b)) * ((a) + (b) + 1)) / 2 + (b))

__device__ __forceinline__ void hweno2d(const double* __restrict__ a, const Consts& K,
                                        double* __restrict__ C) {
    double c0[15];
    hweno_gen::p0_2d(a, c0);
    const double a2 = a[1], a4 = a[3], a5 = a[4], a6 = a[5], a8 = a[7];
    const double sxl = a5 - a4, sxr = a6 - a5, syb = a5 - a2, syt = a8 - a5;
    double w0 = G2D_0, w1 = G2D_1, w2 = G2D_1, w3 = G2D_1, w4 = G2D_1;
    if (!K.linear) {
        const double b0 = hweno_gen::sobolev_2d(c0);
        const double b1 = sxl * sxl + syb * syb;
        const double b2 = sxr * sxr + syb * syb;
        const double b3 = sxl * sxl + syt * syt;
        const double b4 = sxr * sxr + syt * syt;
        double tau = 0.25 * (dabs(b0 - b1) + dabs(b0 - b2) + dabs(b0 - b3) + dabs(b0 - b4));
        tau = tau * tau;
        // five reciprocals 1/(beta_m + eps) from one division (prefix/suffix products)
        const double e = K.eps_weno;
        const double D0 = b0 + e, D1 = b1 + e, D2 = b2 + e, D3 = b3 + e, D4 = b4 + e;
        const double p01 = D0 * D1, p012 = p01 * D2, p0123 = p012 * D3;
        const double s34 = D3 * D4, s234 = D2 * s34;
        const double prod = p0123 * D4;
        double i0, i1, i2, i3, i4;
        if (prod < 1e300) {
            const double inv = rcp(prod);
            i0 = inv * (D1 * s234);
            i1 = inv * (D0 * s234);
            i2 = inv * (p01 * s34);
            i3 = inv * (p012 * D4);
            i4 = inv * p0123;
        } else {   // huge indicators: separate divisions avoid overflow
            i0 = 1.0 / D0;
            i1 = 1.0 / D1;
            i2 = 1.0 / D2;
            i3 = 1.0 / D3;
            i4 = 1.0 / D4;
        }
        const double t0 = G2D_0 * (1.0 + tau * i0);
        const double t1 = G2D_1 * (1.0 + tau * i1);
        const double t2 = G2D_1 * (1.0 + tau * i2);
        const double t3 = G2D_1 * (1.0 + tau * i3);
        const double t4 = G2D_1 * (1.0 + tau * i4);
        const double it = rcp(t0 + t1 + t2 + t3 + t4);
        w0 = t0 * it;
        w1 = t1 * it;
        w2 = t2 * it;
        w3 = t3 * it;
        w4 = t4 * it;
    }
    const double r0 = w0 * (1.0 / G2D_0);
    const double q = w0 * (G2D_1 / G2D_0);
    const double d1 = w1 - q, d2 = w2 - q, d3 = w3 - q, d4 = w4 - q;
#pragma unroll
    for (int k = 0; k < 15; ++k) C[k] = r0 * c0[k];
    C[0] += (d1 + d2 + d3 + d4) * a5;
    C[1] += (d1 + d3) * sxl + (d2 + d4) * sxr;
    C[2] += (d1 + d2) * syb + (d3 + d4) * syt;
}

// Values on the x-faces: out[0..2] at (-1/2, eta_G), out[3..5] at (1/2, eta_G),
// eta_G = (-s, 0, s).
__device__ __forceinline__ void eval_xface(const double* __restrict__ C, double* __restrict__ out) {
    // E_b, O_b: even / odd parts in xi at |xi| = 1/2, for each power b of eta
    const double E0 = C[MI(0, 0)] + 0.25 * C[MI(2, 0)] + 0.0625 * C[MI(4, 0)];
    const double O0 = 0.5 * C[MI(1, 0)] + 0.125 * C[MI(3, 0)];
    const double E1 = C[MI(0, 1)] + 0.25 * C[MI(2, 1)];
    const double O1 = 0.5 * C[MI(1, 1)] + 0.125 * C[MI(3, 1)];
    const double E2 = C[MI(0, 2)] + 0.25 * C[MI(2, 2)];
    const double O2 = 0.5 * C[MI(1, 2)];
    const double E3 = C[MI(0, 3)];
    const double O3 = 0.5 * C[MI(1, 3)];
    const double E4 = C[MI(0, 4)];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double sg = side ? 1.0 : -1.0;
        const double Q0 = E0 + sg * O0, Q1 = E1 + sg * O1, Q2 = E2 + sg * O2;
        const double Q3 = E3 + sg * O3, Q4 = E4;
        const double ev = Q0 + GS2 * Q2 + GS4 * Q4;
        const double od = GS * Q1 + GS3 * Q3;
        out[3 * side + 0] = ev - od;
        out[3 * side + 1] = Q0;
        out[3 * side + 2] = ev + od;
    }
}

// Values on the y-faces: out[0..2] at (xi_G, -1/2), out[3..5] at (xi_G, 1/2).
__device__ __forceinline__ void eval_yface(const double* __restrict__ C, double* __restrict__ out) {
    const double E0 = C[MI(0, 0)] + 0.25 * C[MI(0, 2)] + 0.0625 * C[MI(0, 4)];
    const double O0 = 0.5 * C[MI(0, 1)] + 0.125 * C[MI(0, 3)];
    const double E1 = C[MI(1, 0)] + 0.25 * C[MI(1, 2)];
    const double O1 = 0.5 * C[MI(1, 1)] + 0.125 * C[MI(1, 3)];
    const double E2 = C[MI(2, 0)] + 0.25 * C[MI(2, 2)];
    const double O2 = 0.5 * C[MI(2, 1)];
    const double E3 = C[MI(3, 0)];
    const double O3 = 0.5 * C[MI(3, 1)];
    const double E4 = C[MI(4, 0)];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double sg = side ? 1.0 : -1.0;
        const double Q0 = E0 + sg * O0, Q1 = E1 + sg * O1, Q2 = E2 + sg * O2;
        const double Q3 = E3 + sg * O3, Q4 = E4;
        const double ev = Q0 + GS2 * Q2 + GS4 * Q4;
        const double od = GS * Q1 + GS3 * Q3;
        out[3 * side + 0] = ev - od;
        out[3 * side + 1] = Q0;
        out[3 * side + 2] = ev + od;
    }
}

// Values at the 3x3 tensor Gauss points: out[3*h + g] at (xi_g, eta_h).
__device__ __forceinline__ void eval_vol(const double* __restrict__ C, double* __restrict__ out) {
    // r_a(eta): polynomial in xi with coefficients depending on eta
    double rm[5], r0[5], rp[5];
#pragma unroll
    for (int a = 0; a <= 4; ++a) {
        double ev = C[MI(a, 0)], od = 0.0;
        if (a <= 3) od += GS * C[MI(a, 1)];
        if (a <= 2) ev += GS2 * C[MI(a, 2)];
        if (a <= 1) od += GS3 * C[MI(a, 3)];
        if (a == 0) ev += GS4 * C[MI(0, 4)];
        rm[a] = ev - od;
        r0[a] = C[MI(a, 0)];
        rp[a] = ev + od;
    }
    const double* rows[3] = {rm, r0, rp};
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        const double* r = rows[h];
        const double ev = r[0] + GS2 * r[2] + GS4 * r[4];
        const double od = GS * r[1] + GS3 * r[3];
        out[3 * h + 0] = ev - od;
        out[3 * h + 1] = r[0];
        out[3 * h + 2] = ev + od;
    }
}

// Coefficients (same monomial layout, degree-4 slots zero) of d/dxi and
// d/deta of the quartic C: with C the combination of eq. (3.4), the
// derivatives of eq. (3.5), so the value evaluators above apply to them.
__device__ __forceinline__ void dxi_coeffs(const double* __restrict__ C, double* __restrict__ D) {
#pragma unroll
    for (int q = 0; q < 15; ++q) D[q] = 0.0;
#pragma unroll
    for (int a = 1; a <= 4; ++a)
#pragma unroll
        for (int b = 0; b <= 4 - a; ++b) D[MI(a - 1, b)] = (double)a * C[MI(a, b)];
}
__device__ __forceinline__ void deta_coeffs(const double* __restrict__ C, double* __restrict__ D) {
#pragma unroll
    for (int q = 0; q < 15; ++q) D[q] = 0.0;
#pragma unroll
    for (int b = 1; b <= 4; ++b)
#pragma unroll
        for (int a = 0; a <= 4 - b; ++a) D[MI(a, b - 1)] = (double)b * C[MI(a, b)];
}

// Scaled first moments over the own cell: int p xi, int p eta.
__device__ __forceinline__ double moment_xi(const double* __restrict__ C) {
    return C[MI(1, 0)] * (1.0 / 12.0) + C[MI(1, 2)] * (1.0 / 144.0) + C[MI(3, 0)] * (1.0 / 80.0);
}
__device__ __forceinline__ double moment_eta(const double* __restrict__ C) {
    return C[MI(0, 1)] * (1.0 / 12.0) + C[MI(2, 1)] * (1.0 / 144.0) + C[MI(0, 3)] * (1.0 / 80.0);
}

// ---------------------------------------------------------------------------
// Gas physics (eqs. (2.1), (3.1)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pressure1(const Consts& K, double r, double m, double E) {
    return K.gm1 * (E - 0.5 * (m * m) / r);
}
__device__ __forceinline__ double pressure2(const Consts& K, double r, double m, double n,
                                            double E) {
#pragma clang fp contract(off)   // same rounding in every kernel (see the 2D fluxes)
    return K.gm1 * fma(-0.5 * fma(m, m, n * n), rcp(r), E);
}

// 1D total flux f = f^a - f^d with tau = (4/3) mu u_x, q = -gamma mu e_x / Pr.
__device__ __forceinline__ void flux1(const Consts& K, const double* U, double ux, double ex,
                                      double* f) {
    const double r = U[0], m = U[1], E = U[2];
    const double u = m / r;
    const double p = pressure1(K, r, m, E);
    const double mu = viscosity(K, r, p);
    const double tau = (4.0 / 3.0) * mu * ux;
    const double q = -K.gamma * mu * ex / K.Pr;
    f[0] = m;
    f[1] = m * u + p - tau;
    f[2] = (E + p) * u - (tau * u - q);
}

// PP wave-speed bound of eq. (2.3), taken no smaller than |u| + c.
__device__ __forceinline__ double speed1(const Consts& K, const double* U, double ux, double ex) {
    const double r = U[0], m = U[1], E = U[2];
    const double u = m / r;
    const double p = pressure1(K, r, m, E);
    const double e = p / (K.gm1 * r);
    const double mu = viscosity(K, r, p);
    const double tau = (4.0 / 3.0) * mu * ux;
    const double q = -K.gamma * mu * ex / K.Pr;
    const double r2e = r * r * e;
    const double root = sqrt(r * r * q * q + 2.0 * r2e * (tau - p) * (tau - p));
    const double bpp = fabs(u) + (root + r * fabs(q)) / (2.0 * r2e);
    const double ac = fabs(u) + sqrt(K.gamma * p / r);
    return ac >= bpp ? ac : bpp;
}

// The 2D flux and speed-bound arithmetic below is written with explicit
// fused multiply-adds and no automatic contraction, so that it rounds the
// same way in every kernel it is inlined into (the face fluxes are formed
// by more than one kernel, and their results must agree bit for bit).

// 2D stresses divided by Re (mu(T) in place of 1/Re).
struct Stress { double xx, xy, yy; };
__device__ __forceinline__ Stress stresses(double mu, const double* s) {
#pragma clang fp contract(off)
    Stress t;
    t.xx = mu * fma(4.0 / 3.0, s[0], -(2.0 / 3.0) * s[3]);
    t.xy = mu * (s[1] + s[2]);
    t.yy = mu * fma(4.0 / 3.0, s[3], -(2.0 / 3.0) * s[0]);
    return t;
}

// 2D total flux in direction d (0: f, 1: g); s = (u_x,u_y,v_x,v_y,e_x,e_y).
template <int d, bool VarMu = true>
__device__ __forceinline__ void flux2(const Consts& K, const double* U, const double* s,
                                      double* f) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double u = m * ir, v = n * ir;
    const double p = K.gm1 * fma(-0.5, fma(m, u, n * v), E);
    const double mu = viscosity<VarMu>(K, r, p);
    const Stress t = stresses(mu, s);
    const double kq = K.gPr * mu;
    if (d == 0) {
        f[0] = m;
        f[1] = fma(m, u, p) - t.xx;
        f[2] = fma(n, u, -t.xy);
        f[3] = fma(E + p, u, -fma(t.xx, u, fma(t.xy, v, kq * s[4])));
    } else {
        f[0] = n;
        f[1] = fma(m, v, -t.xy);
        f[2] = fma(n, v, p) - t.yy;
        f[3] = fma(E + p, v, -fma(t.xy, u, fma(t.yy, v, kq * s[5])));
    }
}

// The face fluxes need the six gradients only through three combinations per
// face point: the normal stress and the shear stress divided by mu, and the
// normal derivative of e.  d = 0 (x-face): (4/3 u_x - 2/3 v_y, u_y + v_x,
// e_x); d = 1 (y-face): (4/3 v_y - 2/3 u_x, u_y + v_x, e_y).  Rounded as
// stresses() rounds them, so fluxes from the combinations are the same bits.
template <int d>
__device__ __forceinline__ void stress_combos(const double* s, double* dc) {
#pragma clang fp contract(off)
    dc[0] = d == 0 ? fma(4.0 / 3.0, s[0], -(2.0 / 3.0) * s[3])
                   : fma(4.0 / 3.0, s[3], -(2.0 / 3.0) * s[0]);
    dc[1] = s[1] + s[2];
    dc[2] = s[4 + d];
}

// flux2 at a face point from the three combinations dc of stress_combos.
template <int d, bool VarMu = true>
__device__ __forceinline__ void flux2c(const Consts& K, const double* U, const double* dc,
                                       double* f) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double u = m * ir, v = n * ir;
    const double p = K.gm1 * fma(-0.5, fma(m, u, n * v), E);
    const double mu = viscosity<VarMu>(K, r, p);
    const double tnn = mu * dc[0], txy = mu * dc[1];
    const double kq = K.gPr * mu;
    if (d == 0) {
        f[0] = m;
        f[1] = fma(m, u, p) - tnn;
        f[2] = fma(n, u, -txy);
        f[3] = fma(E + p, u, -fma(tnn, u, fma(txy, v, kq * dc[2])));
    } else {
        f[0] = n;
        f[1] = fma(m, v, -txy);
        f[2] = fma(n, v, p) - tnn;
        f[3] = fma(E + p, v, -fma(txy, u, fma(tnn, v, kq * dc[2])));
    }
}

// speed2 from the three combinations.
template <int d, bool VarMu = true>
__device__ __forceinline__ double speed2c(const Consts& K, const double* U, const double* dc) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double p = K.gm1 * fma(-0.5 * fma(m, m, n * n), ir, E);
    const double mu = viscosity<VarMu>(K, r, p);
    const double tnn = mu * dc[0], txy = mu * dc[1];
    const double kq = K.gPr * mu;
    const double un = (d == 0 ? m : n) * ir;
    const double q = kq * dc[2];
    const double tp = tnn - p;
    const double t2 = fma(tp, tp, txy * txy);
    const double r2e = r * p * K.igm1;
    const double root = sqrt(fma(r * r, q * q, 2.0 * r2e * t2));
    const double bpp = fma(fma(r, fabs(q), root), 0.5 * rcp(r2e), fabs(un));
    const double ac = fabs(un) + sqrt(K.gamma * p * ir);
    return ac >= bpp ? ac : bpp;
}

// The same flux with the direction a run-time value (dy: g instead of f);
// selects instead of branches, so lanes of one wave may take different
// directions without diverging.
template <bool VarMu = true>
__device__ __forceinline__ void flux2_dir(const Consts& K, const double* U, const double* s,
                                          bool dy, double* f) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double u = m * ir, v = n * ir;
    const double p = K.gm1 * fma(-0.5, fma(m, u, n * v), E);
    const double mu = viscosity<VarMu>(K, r, p);
    const Stress t = stresses(mu, s);
    const double kq = K.gPr * mu;
    const double un = dy ? v : u;           // velocity along the direction
    const double tnx = dy ? t.xy : t.xx;    // stress (x, direction)
    const double tny = dy ? t.yy : t.xy;    // stress (y, direction)
    const double qd = dy ? s[5] : s[4];
    f[0] = dy ? n : m;
    f[1] = fma(m, un, (dy ? 0.0 : p)) - tnx;
    f[2] = fma(n, un, (dy ? p : 0.0)) - tny;
    f[3] = fma(E + p, un, -fma(tnx, u, fma(tny, v, kq * qd)));
}

// The two parts of flux2_dir at a volume point, for a volume quadrature
// split between two kernels: the convective flux (and the point's
// viscosity) from the reconstructed state, given u = m / rho and v = n / rho
// as flux2_dir forms them; and the viscous part of components 1..3 from the
// velocities, that viscosity and the six gradients s.  Their sum is
// flux2_dir's flux up to rounding.
template <bool VarMu>
__device__ __forceinline__ void conv2_dir(const Consts& K, double r, double m, double n, double E,
                                          double u, double v, bool dy, double* f, double& mu) {
#pragma clang fp contract(off)
    const double p = K.gm1 * fma(-0.5, fma(m, u, n * v), E);
    mu = viscosity<VarMu>(K, r, p);
    const double un = dy ? v : u;
    f[0] = dy ? n : m;
    f[1] = fma(m, un, (dy ? 0.0 : p));
    f[2] = fma(n, un, (dy ? p : 0.0));
    f[3] = (E + p) * un;
}

__device__ __forceinline__ void visc2_dir(const Consts& K, double u, double v, double mu,
                                          const double* s, bool dy, double* f) {
#pragma clang fp contract(off)
    const Stress t = stresses(mu, s);
    const double kq = K.gPr * mu;
    const double tnx = dy ? t.xy : t.xx;
    const double tny = dy ? t.yy : t.xy;
    const double qd = dy ? s[5] : s[4];
    f[0] = -tnx;
    f[1] = -tny;
    f[2] = -fma(tnx, u, fma(tny, v, kq * qd));
}

// PP wave-speed bound of eq. (3.3) in direction d, no smaller than |u_d| + c.
template <int d, bool VarMu = true>
__device__ __forceinline__ double speed2(const Consts& K, const double* U, const double* s) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double p = K.gm1 * fma(-0.5 * fma(m, m, n * n), ir, E);
    const double mu = viscosity<VarMu>(K, r, p);
    const Stress t = stresses(mu, s);
    const double kq = K.gPr * mu;
    const double un = (d == 0 ? m : n) * ir;
    const double q = kq * s[4 + d];
    const double tp = (d == 0 ? t.xx : t.yy) - p;
    const double t2 = fma(tp, tp, t.xy * t.xy);
    const double r2e = r * p * K.igm1;      // rho^2 e with e = p / ((gamma - 1) rho)
    const double root = sqrt(fma(r * r, q * q, 2.0 * r2e * t2));
    const double bpp = fma(fma(r, fabs(q), root), 0.5 * rcp(r2e), fabs(un));
    const double ac = fabs(un) + sqrt(K.gamma * p * ir);
    return ac >= bpp ? ac : bpp;
}

// ---------------------------------------------------------------------------
// Characteristic bases (Sec. 2.1 / 3.1): eigenvectors of the convective
// Jacobian at a cell average.  Right eigenvectors as columns of R; L = R^-1.
// ---------------------------------------------------------------------------
struct Eig1 { double R[3][3], L[3][3]; };
__device__ __forceinline__ void eig1(const Consts& K, const double* Ub, Eig1& e) {
    const double r = Ub[0], u = Ub[1] / r;
    const double p = pressure1(K, r, Ub[1], Ub[2]);
    const double c = sqrt(K.gamma * p / r);
    const double H = (Ub[2] + p) / r;
    const double b1 = K.gm1 / (c * c), b2 = 0.5 * b1 * u * u, ic = 1.0 / c;
    e.R[0][0] = 1.0;        e.R[0][1] = 1.0;         e.R[0][2] = 1.0;
    e.R[1][0] = u - c;      e.R[1][1] = u;           e.R[1][2] = u + c;
    e.R[2][0] = H - u * c;  e.R[2][1] = 0.5 * u * u; e.R[2][2] = H + u * c;
    e.L[0][0] = 0.5 * (b2 + u * ic); e.L[0][1] = -0.5 * (b1 * u + ic); e.L[0][2] = 0.5 * b1;
    e.L[1][0] = 1.0 - b2;            e.L[1][1] = b1 * u;               e.L[1][2] = -b1;
    e.L[2][0] = 0.5 * (b2 - u * ic); e.L[2][1] = 0.5 * (ic - b1 * u);  e.L[2][2] = 0.5 * b1;
}

// Row k of L and row c of R of the x- (b = 0) or y-Jacobian (b = 1).
__device__ __forceinline__ void eig2_rows(const Consts& K, const double* Ub, int b, int k,
                                          double* Lrow, double* Rrow) {
    const double ir = rcp(Ub[0]);
    const double u = Ub[1] * ir, v = Ub[2] * ir;
    const double q2 = u * u + v * v;
    const double p = K.gm1 * (Ub[3] - 0.5 * Ub[0] * q2);
    const double c2 = K.gamma * p * ir;
    const double c = sqrt(c2);
    const double ic = rcp(c);
    const double H = (Ub[3] + p) * ir;
    const double b1 = K.gm1 * ic * ic, b2 = 0.5 * b1 * q2;
    const double un = b ? v : u;       // normal velocity
    const double ut = b ? u : v;       // tangential velocity
    // In (rho, m_n, m_t, E) ordering the two Jacobians have identical
    // eigenvectors; (rho, m, n, E) puts the normal momentum in slot 1 for
    // b = 0 and in slot 2 for b = 1.  Row k of L in the normal/tangential
    // ordering:
    double L0, Ln, Lt, L3;
    switch (k) {
        case 0: L0 = 0.5 * (b2 + un * ic); Ln = -0.5 * (b1 * un + ic);
                Lt = -0.5 * b1 * ut;       L3 = 0.5 * b1; break;
        case 1: L0 = 1.0 - b2; Ln = b1 * un; Lt = b1 * ut; L3 = -b1; break;
        case 2: L0 = -ut; Ln = 0.0; Lt = 1.0; L3 = 0.0; break;
        default: L0 = 0.5 * (b2 - un * ic); Ln = 0.5 * (ic - b1 * un);
                 Lt = -0.5 * b1 * ut;       L3 = 0.5 * b1; break;
    }
    Lrow[0] = L0;
    Lrow[1] = b ? Lt : Ln;
    Lrow[2] = b ? Ln : Lt;
    Lrow[3] = L3;
    // Row of R for conserved component k; columns (fields 0..3):
    // (1, un-c, ut, H-un c), (1, un, ut, q2/2), (0, 0, 1, ut), (1, un+c, ut, H+un c)
    if (k == 0) {
        Rrow[0] = 1.0; Rrow[1] = 1.0; Rrow[2] = 0.0; Rrow[3] = 1.0;
    } else if (k == 3) {
        Rrow[0] = H - un * c; Rrow[1] = 0.5 * q2; Rrow[2] = ut; Rrow[3] = H + un * c;
    } else {
        const bool nrm = (k == 1) == (b == 0);   // the normal momentum's row
        Rrow[0] = nrm ? un - c : ut;
        Rrow[1] = nrm ? un : ut;
        Rrow[2] = nrm ? 0.0 : 1.0;
        Rrow[3] = nrm ? un + c : ut;
    }
}

// ---------------------------------------------------------------------------
// Order-preserving maps of doubles to unsigned 64-bit keys (for atomic
// max / min of doubles of any sign).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dkey(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double dkey_inv(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double x;
    __builtin_memcpy(&x, &b, 8);
    return x;
}

}  // namespace hw
