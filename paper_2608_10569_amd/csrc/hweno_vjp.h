// Interfaces of the reverse-mode kernels: adjoint inputs, adjoint workspace
// and thin wrappers over the generated vector-Jacobian products.
#pragma once

#include "hweno_adj.h"
#include "hweno_kernels.h"

namespace hw {

struct AdjIn {
    const double* Rb;   // residual adjoint, D1 interior layout (12 or 6 per cell)
    const double* Vb;   // modified-moment adjoint, interior layout (8 or 3 per cell)
    double rs, vs;      // scale factors applied to Rb and Vb as they are read
};

// Adjoint workspace (component-major over the ghosted grid, like Grid2/Grid1).
struct AdjWs {
    double* xfb;        // 24 / 12: face-trace adjoints
    double* yfb;        // 24
    double* xvb;        // 36: volume-value adjoints
    double* yvb;        // 36
    double* gfb;        // 72 / 8: face-gradient adjoints
    double* rbc;        // 102 / 10: weak-moment contributions to the 3x3 stencil
    double* rbb;        // 18 / 4: gathered weak-moment adjoints
    double* uc;         // 136 / 15: state contributions to the stencil
    double* rcb;        // 128: cotangents of the 16 characteristic outputs per (b, k)
    double* rrb;        // 32: R-bar rows per (b, k)
    double* rlim;       // 4: the limiter's share of the cell-average adjoint
    double* ubb;        // 12 / 6: gathered state adjoint (ghosted)
    double* mupart;     // block partials of the mu adjoint
    double* rbm;        // 12 / cell (interior): a masked grid's residual seed, solid cells zeroed
    double* vbm;        // 8 / cell (interior): its modified-moment seed likewise
    // masked grids: the mirror list grouped by source (fluid cells that are
    // the mirror source of a listed solid cell, ghosted index; the listed
    // entries of source u are sord[sstart[u] .. sstart[u + 1]), ascending)
    const int* ssrcu;
    const int* sstart;
    const int* sord;
    int nsrc;
    int mu_off1, mu_off2;
    unsigned rev;       // bit k: adjoint kernel k takes its blocks last first (per XCD)
};

__device__ __forceinline__ double g_ld(const double* p, long long idx) { return p[idx]; }

template <int d>
__device__ __forceinline__ void flux2_vjp(const Consts& K, const double* U, const double* s,
                                          double mu, const double* fb, double* Ub, double* sb,
                                          double& mub) {
    if (d == 0) adj::flux2_vjp_0(K, U, s, mu, fb, Ub, sb, mub);
    else adj::flux2_vjp_1(K, U, s, mu, fb, Ub, sb, mub);
}

// adjoint of speed2<d> = max(|u_n| + c, beta_PP) (ties to the first branch)
template <int d>
__device__ __forceinline__ void speed2_vjp(const Consts& K, const double* U, const double* s,
                                           double mu, double yb, double* Ub, double* sb,
                                           double& mub) {
    const double r = U[0];
    const double p = pressure2(K, r, U[1], U[2], U[3]);
    const double e = p / (K.gm1 * r);
    const Stress t = stresses(mu, s);
    const double kq = K.gamma * mu / K.Pr;
    const double un = (d == 0 ? U[1] : U[2]) / r;
    const double q = kq * s[4 + d];
    const double t2 = d == 0 ? (t.xx - p) * (t.xx - p) + t.xy * t.xy
                             : t.xy * t.xy + (t.yy - p) * (t.yy - p);
    const double r2e = r * r * e;
    const double bpp = fabs(un) + (sqrt(r * r * q * q + 2.0 * r2e * t2) + r * fabs(q)) / (2.0 * r2e);
    const double ac = fabs(un) + sqrt(K.gamma * p / r);
    const double sgu = sgn(un);
    if (ac >= bpp) {
        if (d == 0) adj::speed2_ac_vjp_0(K, U, sgu, yb, Ub);
        else adj::speed2_ac_vjp_1(K, U, sgu, yb, Ub);
    } else {
        if (d == 0) adj::speed2_bpp_vjp_0(K, U, s, mu, sgu, sgn(q), yb, Ub, sb, mub);
        else adj::speed2_bpp_vjp_1(K, U, s, mu, sgu, sgn(q), yb, Ub, sb, mub);
    }
}

// mu(T) = mu_ref (T / T_ref)^mu_exp, T = p / rho (eq. (3.1) with the power
// law), at a point as the forward fluxes form it.
__device__ __forceinline__ double point_mu(const Consts& K, const double* U) {
#pragma clang fp contract(off)
    const double r = U[0], m = U[1], n = U[2], E = U[3];
    const double ir = rcp(r);
    const double u = m * ir, v = n * ir;
    const double p = K.gm1 * fma(-0.5, fma(m, u, n * v), E);
    return viscosity<true>(K, r, p);
}

// Adjoint of the dependence of mu(T) on the state at a point: Ub += mub *
// dmu/dU with dmu/dT = mu_exp mu / T and T = (gamma - 1)(E / rho - |u|^2 / 2);
// returns dmu/dmu_ref = (T / T_ref)^mu_exp, which carries mub into the
// adjoint of mu_ref.
__device__ __forceinline__ double mu_T_vjp(const Consts& K, const double* U, double mub,
                                           double* Ub) {
    if (K.mu_exp == 0.0) return 1.0;
    const double r = U[0], ir = 1.0 / r;
    const double u = U[1] * ir, v = U[2] * ir;
    const double q2 = u * u + v * v;
    const double T = K.gm1 * (U[3] * ir - 0.5 * q2);
    const double f = pow(T / K.T_ref, K.mu_exp);
    const double gT = mub * K.mu_ref * f * K.mu_exp / T;   // mub * dmu/dT
    Ub[0] += gT * (0.5 * K.gm1 * q2 - T) * ir;
    Ub[1] -= gT * K.gm1 * u * ir;
    Ub[2] -= gT * K.gm1 * v * ir;
    Ub[3] += gT * K.gm1 * ir;
    return f;
}

// Adjoint workspace of a 1D grid (component-major over the ghosted cells).
struct AdjWs1 {
    double* base;       // start of the zero-filled region (ptsb .. mupart)
    long long count;    // doubles in that region
    double* ptsb;       // 12: adjoints of the limited LGL values (p*3 + c)
    double* grb;        // 8: adjoints of the LGL gradients (p*2 + w)
    double* mupart;     // NX + nx + 1: mu-adjoint partials of the faces, then of the cells
    double* rbc;        // 10: weak-moment adjoints from the gradient stencil (w*5 + s)
    double* uc;         // 15: state adjoints from the reconstruction stencil (s*3 + c)
    double* ub;         // 6: gathered state adjoint
};

// Adjoint of the 1D LF speed speed1 (the branch of the forward point; ties
// to |u| + c), accumulated into Ub, uxb, exb, mub.
__device__ __forceinline__ void speed1_vjp(const Consts& K, const double* U, double ux, double ex,
                                           double mu, double yb, double* Ub, double& uxb,
                                           double& exb, double& mub) {
    const double r = U[0], u = U[1] / r;
    const double p = pressure1(K, r, U[1], U[2]);
    const double e = p / (K.gm1 * r);
    const double tau = (4.0 / 3.0) * mu * ux;
    const double q = -K.gamma * mu * ex / K.Pr;
    const double r2e = r * r * e;
    const double root = sqrt(r * r * q * q + 2.0 * r2e * (tau - p) * (tau - p));
    const double bpp = fabs(u) + (root + r * fabs(q)) / (2.0 * r2e);
    const double ac = fabs(u) + sqrt(K.gamma * p / r);
    if (ac >= bpp) adj::speed1_ac_vjp(K, U, sgn(u), yb, Ub);
    else adj::speed1_bpp_vjp(K, U, ux, ex, mu, sgn(u), sgn(q), yb, Ub, uxb, exb, mub);
}

// mu(T) of a 1D point as flux1 and speed1 form it, and the adjoint of its
// dependence on (rho, m, E) (T = (gamma - 1)(E / rho - u^2 / 2)); the return
// value carries mub into the adjoint of mu_ref.
__device__ __forceinline__ double point_mu1(const Consts& K, const double* U) {
    return viscosity<true>(K, U[0], pressure1(K, U[0], U[1], U[2]));
}
__device__ __forceinline__ double mu_T_vjp1(const Consts& K, const double* U, double mub,
                                            double* Ub) {
    if (K.mu_exp == 0.0) return 1.0;
    const double ir = 1.0 / U[0], u = U[1] * ir;
    const double T = K.gm1 * (U[2] * ir - 0.5 * u * u);
    const double f = pow(T / K.T_ref, K.mu_exp);
    const double gT = mub * K.mu_ref * f * K.mu_exp / T;
    Ub[0] += gT * (0.5 * K.gm1 * u * u - T) * ir;
    Ub[1] -= gT * K.gm1 * u * ir;
    Ub[2] += gT * K.gm1 * ir;
    return f;
}

hipError_t launch_vjp1(const Grid1& g, const AdjIn& A, AdjWs1 W, const double* S, double* Ubar,
                       double* mu_out, int mu_acc, hipStream_t st);

long long adj_mu_partials2(const Grid2& g);
// mu_acc = 0: *mu_out = mu-bar; 1: *mu_out += mu-bar (device scalar).
// add != nullptr: add_a * add[t] joins the cell-average adjoints (the first
// 4 nx ny entries of Ubar) of the fluid cells, as an axpy after the call would.
// Masked grids: the seeds of solid cells are taken as zero (they carry no
// residual), pass != nullptr adds pass[t] to every component of the
// solid cells (a stage leaves them at its filled input), and the adjoint of
// the mirror fill of the solid cells ends the call.
hipError_t launch_vjp2(const Grid2& g, const AdjIn& A, AdjWs W, const double* S, double* Ubar,
                       double* mu_out, int mu_acc, hipStream_t st, const double* add = nullptr,
                       double add_a = 0.0, const double* pass = nullptr);
// y[0:n] += a x[0:n]
hipError_t launch_axpy(double* y, const double* x, double a, long long n, hipStream_t st);
// y[0:n] = a u[0:n] + b y[0:n] + x[0:n]
hipError_t launch_lin3(double* y, const double* u, double a, double b, const double* x, long long n,
                       hipStream_t st);

}  // namespace hw
