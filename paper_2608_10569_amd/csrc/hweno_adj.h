// Reverse mode of the scalar unified-stencil HWENO reconstruction
// (Appendix A, eqs. (A.1)-(A.6)): given the adjoint of the combined
// polynomial's coefficients, the adjoint of the input moments.  The
// nonlinear weights are differentiated (|x| has derivative sign(x), 0 at 0).
#pragma once

#include "hweno_device.h"
#include "hweno_gen_adj.h"

namespace hw {

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// ab[17] = (d C / d a)^T Cb for the 2D reconstruction hweno2d(a) -> C.
__device__ inline void hweno2d_vjp(const double* __restrict__ a, const Consts& K,
                                   const double* __restrict__ Cb, double* __restrict__ ab) {
    double c0[15];
    hweno_gen::p0_2d(a, c0);
    const double a2 = a[1], a4 = a[3], a5 = a[4], a6 = a[5], a8 = a[7];
    const double sxl = a5 - a4, sxr = a6 - a5, syb = a5 - a2, syt = a8 - a5;
    double w[5] = {G2D_0, G2D_1, G2D_1, G2D_1, G2D_1};
    double b[5], im[5], tau = 0.0, sig = 0.0, T = 1.0;
    if (!K.linear) {
        b[0] = hweno_gen::sobolev_2d(c0);
        b[1] = sxl * sxl + syb * syb;
        b[2] = sxr * sxr + syb * syb;
        b[3] = sxl * sxl + syt * syt;
        b[4] = sxr * sxr + syt * syt;
        sig = 0.25 * (fabs(b[0] - b[1]) + fabs(b[0] - b[2]) + fabs(b[0] - b[3]) + fabs(b[0] - b[4]));
        tau = sig * sig;
        double t[5];
        T = 0.0;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            im[m] = 1.0 / (b[m] + K.eps_weno);
            t[m] = (m ? G2D_1 : G2D_0) * (1.0 + tau * im[m]);
            T += t[m];
        }
#pragma unroll
        for (int m = 0; m < 5; ++m) w[m] = t[m] / T;
    }
    const double r0 = w[0] * (1.0 / G2D_0);
    const double q = w[0] * (G2D_1 / G2D_0);
    const double d1 = w[1] - q, d2 = w[2] - q, d3 = w[3] - q, d4 = w[4] - q;
    // backward through C = r0 c0 + linear-candidate terms
    double cb0[15];
    double r0b = 0.0;
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        cb0[k] = r0 * Cb[k];
        r0b += Cb[k] * c0[k];
    }
    const double d1b = Cb[0] * a5 + Cb[1] * sxl + Cb[2] * syb;
    const double d2b = Cb[0] * a5 + Cb[1] * sxr + Cb[2] * syb;
    const double d3b = Cb[0] * a5 + Cb[1] * sxl + Cb[2] * syt;
    const double d4b = Cb[0] * a5 + Cb[1] * sxr + Cb[2] * syt;
    double a5b = Cb[0] * (d1 + d2 + d3 + d4);
    double sxlb = Cb[1] * (d1 + d3), sxrb = Cb[1] * (d2 + d4);
    double sybb = Cb[2] * (d1 + d2), sytb = Cb[2] * (d3 + d4);
    if (!K.linear) {
        double wb[5];
        wb[0] = r0b * (1.0 / G2D_0) - (G2D_1 / G2D_0) * (d1b + d2b + d3b + d4b);
        wb[1] = d1b;
        wb[2] = d2b;
        wb[3] = d3b;
        wb[4] = d4b;
        double ws = 0.0;
#pragma unroll
        for (int m = 0; m < 5; ++m) ws += wb[m] * w[m];
        double taub = 0.0, bb[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const double tb = (wb[m] - ws) / T;
            const double g = m ? G2D_1 : G2D_0;
            taub += tb * g * im[m];
            bb[m] = -tb * g * tau * im[m] * im[m];
        }
        const double sigb = 2.0 * sig * taub;
#pragma unroll
        for (int m = 1; m < 5; ++m) {
            const double s = 0.25 * sigb * sgn(b[0] - b[m]);
            bb[0] += s;
            bb[m] -= s;
        }
        double g[15];
        adj::sobolev_2d_grad(c0, g);
#pragma unroll
        for (int k = 0; k < 15; ++k) cb0[k] += bb[0] * g[k];
        sxlb += 2.0 * sxl * (bb[1] + bb[3]);
        sxrb += 2.0 * sxr * (bb[2] + bb[4]);
        sybb += 2.0 * syb * (bb[1] + bb[2]);
        sytb += 2.0 * syt * (bb[3] + bb[4]);
    }
    adj::p0_2d_T(cb0, ab);
    ab[3] -= sxlb;
    ab[5] += sxrb;
    ab[1] -= sybb;
    ab[7] += sytb;
    ab[4] += a5b + sxlb - sxrb + sybb - sytb;
}

// ab[5] = (d C / d a)^T Cb for the 1D reconstruction hweno1d(a) -> C.
__device__ inline void hweno1d_vjp(const double* __restrict__ a, const Consts& K,
                                   const double* __restrict__ Cb, double* __restrict__ ab) {
    double c0[5];
    hweno_gen::p0_1d(a, c0);
    const double s1 = a[1] - a[0], s2 = a[2] - a[1];
    double w[3] = {G1D_0, G1D_1, G1D_1};
    double b[3], im[3], tau = 0.0, sig = 0.0, T = 1.0;
    if (!K.linear) {
        b[0] = hweno_gen::sobolev_1d(c0);
        b[1] = s1 * s1;
        b[2] = s2 * s2;
        sig = 0.5 * (fabs(b[0] - b[1]) + fabs(b[0] - b[2]));
        tau = sig * sig;
        double t[3];
        T = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            im[m] = 1.0 / (b[m] + K.eps_weno);
            t[m] = (m ? G1D_1 : G1D_0) * (1.0 + tau * im[m]);
            T += t[m];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) w[m] = t[m] / T;
    }
    const double r0 = w[0] / G1D_0;
    const double q = w[0] * G1D_1 / G1D_0;
    const double d1 = w[1] - q, d2 = w[2] - q;
    double cb0[5], r0b = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        cb0[k] = r0 * Cb[k];
        r0b += Cb[k] * c0[k];
    }
    const double d1b = Cb[0] * a[1] + Cb[1] * s1;
    const double d2b = Cb[0] * a[1] + Cb[1] * s2;
    double a1b = Cb[0] * (d1 + d2);
    double s1b = Cb[1] * d1, s2b = Cb[1] * d2;
    if (!K.linear) {
        double wb[3] = {r0b / G1D_0 - (G1D_1 / G1D_0) * (d1b + d2b), d1b, d2b};
        const double ws = wb[0] * w[0] + wb[1] * w[1] + wb[2] * w[2];
        double taub = 0.0, bb[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double tb = (wb[m] - ws) / T;
            const double g = m ? G1D_1 : G1D_0;
            taub += tb * g * im[m];
            bb[m] = -tb * g * tau * im[m] * im[m];
        }
        const double sigb = 2.0 * sig * taub;
#pragma unroll
        for (int m = 1; m < 3; ++m) {
            const double s = 0.5 * sigb * sgn(b[0] - b[m]);
            bb[0] += s;
            bb[m] -= s;
        }
        double g[5];
        adj::sobolev_1d_grad(c0, g);
#pragma unroll
        for (int k = 0; k < 5; ++k) cb0[k] += bb[0] * g[k];
        s1b += 2.0 * s1 * bb[1];
        s2b += 2.0 * s2 * bb[2];
    }
    adj::p0_1d_T(cb0, ab);
    ab[0] -= s1b;
    ab[1] += a1b + s1b - s2b;
    ab[2] += s2b;
}

// Adjoint of the own-cell moments (transpose of moment_xi / moment_eta / moment1d).
__device__ __forceinline__ void moment_xi_T(double yb, double* Cb) {
    Cb[MI(1, 0)] += yb * (1.0 / 12.0);
    Cb[MI(1, 2)] += yb * (1.0 / 144.0);
    Cb[MI(3, 0)] += yb * (1.0 / 80.0);
}
__device__ __forceinline__ void moment_eta_T(double yb, double* Cb) {
    Cb[MI(0, 1)] += yb * (1.0 / 12.0);
    Cb[MI(2, 1)] += yb * (1.0 / 144.0);
    Cb[MI(0, 3)] += yb * (1.0 / 80.0);
}
__device__ __forceinline__ void moment1d_T(double yb, double* Cb) {
    Cb[1] += yb * (1.0 / 12.0);
    Cb[3] += yb * (1.0 / 80.0);
}

}  // namespace hw
