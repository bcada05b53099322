// 1D HWENO-GR residual and SSP-RK3 stage update (Sec. 2 of arXiv 2608.10569).
// Same stage structure as the 2D pipeline, one thread per cell:
//   ghost -> recon (eq. (2.4), characteristic fields, PP limiter on the four
//   LGL values) -> rbar (eqs. (2.6)-(2.8)) -> grad (eq. (2.9), volume-flux
//   quadrature) -> flux (eq. (2.3)) -> update (eqs. (2.2), (2.12)).
// The comparison scheme HWENO-DR (eq. (2.5)) takes its gradients and volume
// fluxes from the reconstruction kernel and skips rbar and grad.

#include "hweno_kernels.h"

namespace hw {

namespace {

constexpr int HALO = 4;

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ unsigned long long wsum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ void k_ghost1(Grid1 g, double* S) {
    const int t = threadIdx.x;
    if (t >= 2 * HALO) return;
    const int right = t >= HALO;
    const int d = (t % HALO) + 1;
    const Side& sd = g.side[right];
    const long long N = g.NX;
    int di, si;
    if (!right) {
        di = HALO - d;
        si = sd.kind == 0 ? HALO + g.nx - d : (sd.kind == 1 ? HALO : HALO + d - 1);
    } else {
        di = HALO + g.nx - 1 + d;
        si = sd.kind == 0 ? HALO + d - 1 : (sd.kind == 1 ? HALO + g.nx - 1 : HALO + g.nx - d);
    }
    if (sd.kind == 2) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            S[c * N + di] = sd.inflow[c];
            S[(3 + c) * N + di] = 0.0;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q * N + di] = sd.sign[q] * S[q * N + si];
}

// Characteristic reconstruction + PP limiter on cells 1 .. NX-2.  DR: the
// comparison scheme's viscous gradients as well (eq. (2.5)): each field's
// combination differentiated with its weights kept, transformed back to
// (rho, m, E)_x and converted to (u_x, e_x) with the limited point values,
// which enter the flux there; then the volume-flux quadrature, so that the
// weak-moment and gradient kernels are not needed.
template <bool DR>
__global__ void k_recon1(Grid1 g, const double* __restrict__ S) {
    const Consts& K = g.K;
    const long long N = g.NX;
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i <= g.NX - 2;
    double amax = -INFINITY;
    unsigned long long act = 0;
    if (valid) {
        double ub[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) ub[c] = S[c * N + i];
        Eig1 e;
        eig1(K, ub, e);
        double P[4][3] = {{0.0}}, vh[3] = {0.0, 0.0, 0.0};
        double dP[4][3] = {{0.0}};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double l = e.L[k][c];
                a[0] += l * S[c * N + i - 1];
                a[1] += l * S[c * N + i];
                a[2] += l * S[c * N + i + 1];
                a[3] += l * S[(3 + c) * N + i - 1];
                a[4] += l * S[(3 + c) * N + i + 1];
            }
            double C[5], v[4];
            hweno1d(a, K, C);
            eval1d(C, v);
            const double mo = moment1d(C);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int p = 0; p < 4; ++p) P[p][c] += e.R[c][k] * v[p];
                vh[c] += e.R[c][k] * mo;
            }
            if constexpr (DR) {
                double dv[4];
                deval1d(C, dv);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int p = 0; p < 4; ++p) dP[p][c] += e.R[c][k] * (dv[p] * K.idx);
            }
        }
        // positivity limiter on the four LGL values (all four are rescaled)
        const double rbar = ub[0];
        const double pbar = pressure1(K, ub[0], ub[1], ub[2]);
        const double eps = fmin(fmin(K.eps_pp, rbar), pbar);
        double rmin = P[0][0];
#pragma unroll
        for (int p = 1; p < 4; ++p) rmin = fmin(rmin, P[p][0]);
        const double th1 = rmin < eps ? (rbar - eps) / (rbar - rmin) : 1.0;
        double th2 = 1.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            P[p][0] = rbar + th1 * (P[p][0] - rbar);
            const double pt = pressure1(K, P[p][0], P[p][1], P[p][2]);
            if (pt < eps) th2 = fmin(th2, (pbar - eps) / (pbar - pt));
        }
        double su = 0.0, se = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                P[p][c] = ub[c] + th2 * (P[p][c] - ub[c]);
                g.pts[(p * 3 + c) * N + i] = P[p][c];
            }
            const double wq = (p == 0 || p == 3) ? LGL_W0 : LGL_W1;
            const double u = P[p][1] / P[p][0];
            su += wq * u;
            se += wq * (P[p][2] / P[p][0] - 0.5 * u * u);
        }
        g.wb[0 * N + i] = su;
        g.wb[1 * N + i] = se;
        const bool inter = i >= HALO && i < HALO + g.nx;
        if constexpr (DR) {
            double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const double r = P[p][0], u = P[p][1] / r;
                const double ux = (dP[p][1] - u * dP[p][0]) / r;
                const double ex = (dP[p][2] - (P[p][2] / r) * dP[p][0]) / r - u * ux;
                g.gr[(p * 2 + 0) * N + i] = ux;
                g.gr[(p * 2 + 1) * N + i] = ex;
                double f[3];
                flux1(K, P[p], ux, ex, f);
                const double wq = (p == 0 || p == 3) ? LGL_W0 : LGL_W1;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += wq * f[c];
            }
            if (inter) {
#pragma unroll
                for (int c = 0; c < 3; ++c) g.vf[c * N + i] = acc[c];
            }
        }
        if (inter) {
#pragma unroll
            for (int c = 0; c < 3; ++c) g.vk[c * N + i] = vh[c];
#pragma unroll
            for (int p = 0; p < 4; p += 3) {
                const double pr = pressure1(K, P[p][0], P[p][1], P[p][2]);
                amax = fmax(amax, fabs(P[p][1] / P[p][0]) + sqrt(K.gamma * pr / P[p][0]));
            }
            act = (th1 < 1.0 || th2 < 1.0) ? 1ull : 0ull;
        }
    }
    amax = wmax(amax);
    act = wsum(act);
    if ((threadIdx.x & 63) == 0) {
        if (amax > -INFINITY) atomicMax(&g.red->alpha_key, dkey(amax));
        if (act) atomicAdd(&g.red->pp_cells, act);
    }
}

__device__ __forceinline__ void prim_ue(const Grid1& g, long long i, int p, double* w) {
    const long long N = g.NX;
    const double r = g.pts[(p * 3 + 0) * N + i];
    const double u = g.pts[(p * 3 + 1) * N + i] / r;
    w[0] = u;
    w[1] = g.pts[(p * 3 + 2) * N + i] / r - 0.5 * u * u;
}

// Weak-derivative moments on cells 2 .. NX-3.
__global__ void k_rbar1(Grid1 g) {
    const int i = 2 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > g.NX - 3) return;
    const long long N = g.NX;
    double a[2], b[2], c[2], d[2];
    prim_ue(g, i - 1, 3, a);
    prim_ue(g, i, 0, b);
    prim_ue(g, i, 3, c);
    prim_ue(g, i + 1, 0, d);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double hm = 0.5 * (a[w] + b[w]);
        const double hp = 0.5 * (c[w] + d[w]);
        g.rb[(w * 2 + 0) * N + i] = (hp - hm) * g.K.idx;
        g.rb[(w * 2 + 1) * N + i] = (0.5 * (hp + hm) - g.wb[w * N + i]) * g.K.idx;
    }
}

// Gradient reconstruction on cells 3 .. NX-4 and the volume-flux quadrature.
__global__ void k_grad1(Grid1 g) {
    const int i = 3 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > g.NX - 4) return;
    const long long N = g.NX;
    double gr[4][2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double* r0 = g.rb + (w * 2 + 0) * N;
        const double* r1 = g.rb + (w * 2 + 1) * N;
        const double a[5] = {r0[i - 1], r0[i], r0[i + 1], r1[i - 1], r1[i + 1]};
        double C[5], v[4];
        hweno1d(a, grad_consts(g.K), C);
        eval1d(C, v);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            gr[p][w] = v[p];
            g.gr[(p * 2 + w) * N + i] = v[p];
        }
    }
    if (i >= HALO && i < HALO + g.nx) {
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double U[3], f[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) U[c] = g.pts[(p * 3 + c) * N + i];
            flux1(g.K, U, gr[p][0], gr[p][1], f);
            const double wq = (p == 0 || p == 3) ? LGL_W0 : LGL_W1;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += wq * f[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) g.vf[c * N + i] = acc[c];
    }
}

// Face fluxes at i + 1/2 for i = HALO-1 .. HALO+nx-1.
__global__ void k_flux1(Grid1 g) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double beta = -INFINITY;
    if (f <= g.nx) {
        const long long N = g.NX;
        const int i = HALO - 1 + f;
        double Um[3], Up[3], fm[3], fp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Um[c] = g.pts[(3 * 3 + c) * N + i];
            Up[c] = g.pts[(0 * 3 + c) * N + i + 1];
        }
        const double umx = g.gr[(3 * 2 + 0) * N + i], emx = g.gr[(3 * 2 + 1) * N + i];
        const double upx = g.gr[(0 * 2 + 0) * N + i + 1], epx = g.gr[(0 * 2 + 1) * N + i + 1];
        flux1(g.K, Um, umx, emx, fm);
        flux1(g.K, Up, upx, epx, fp);
        beta = fmax(speed1(g.K, Um, umx, emx), speed1(g.K, Up, upx, epx));
#pragma unroll
        for (int c = 0; c < 3; ++c) g.fh[c * N + i] = 0.5 * (fm[c] + fp[c] - beta * (Up[c] - Um[c]));
    }
    beta = wmax(beta);
    if ((threadIdx.x & 63) == 0 && beta > -INFINITY) atomicMax(&g.red->beta_key, dkey(beta));
}

__global__ void k_update1(Grid1 g, int stage, const double* __restrict__ S0,
                          const double* __restrict__ Sin, double* __restrict__ Sout,
                          double* __restrict__ Rout, double* __restrict__ Vout,
                          const double* __restrict__ src) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double rmin = INFINITY, pmin = INFINITY;
    unsigned long long bad = 0;
    if (t < g.nx) {
        const long long N = g.NX;
        const int i = t + HALO;
        double F1[3], F2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double fr = g.fh[c * N + i], fl = g.fh[c * N + i - 1];
            F1[c] = -(fr - fl) * g.K.idx;
            F2[c] = -(fl + fr) * (0.5 * g.K.idx) + g.vf[c * N + i] * g.K.idx;
        }
        if (src) {   // prescribed source moments (layout of R)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                F1[c] += src[c * g.nx + t];
                F2[c] += src[(3 + c) * g.nx + t];
            }
        }
        if (stage == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Rout[c * g.nx + t] = F1[c];
                Rout[(3 + c) * g.nx + t] = F2[c];
                Vout[c * g.nx + t] = g.vk[c * N + i];
            }
        } else {
            const double dt = g.red->dt;
            double nw[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double in0 = Sin[c * N + i];
                const double in1 = g.vk[c * N + i];
                if (stage == 1) {
                    nw[c] = in0 + dt * F1[c];
                    nw[3 + c] = in1 + dt * F2[c];
                    g.vn[c * N + i] = in1;
                } else {
                    const double a = stage == 2 ? 0.75 : 1.0 / 3.0;
                    const double bb = stage == 2 ? 0.25 : 2.0 / 3.0;
                    nw[c] = a * S0[c * N + i] + bb * (in0 + dt * F1[c]);
                    nw[3 + c] = a * g.vn[c * N + i] + bb * (in1 + dt * F2[c]);
                }
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) Sout[q * N + i] = nw[q];
            const double p = pressure1(g.K, nw[0], nw[1], nw[2]);
            rmin = nw[0];
            pmin = p;
            bool ok = nw[0] > 0.0 && p > 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) ok = ok && isfinite(nw[q]);
            bad = ok ? 0ull : 1ull;
        }
    }
    if (stage > 0) {
        rmin = wmin(rmin);
        pmin = wmin(pmin);
        bad = wsum(bad);
        if ((threadIdx.x & 63) == 0) {
            if (rmin < INFINITY) atomicMin(&g.red->min_rho_key, dkey(rmin));
            if (pmin < INFINITY) atomicMin(&g.red->min_p_key, dkey(pmin));
            if (bad) atomicAdd(&g.red->bad[stage], (unsigned int)bad);
        }
    }
}

__global__ void k_check1(Grid1 g, const double* __restrict__ S) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bad = 0;
    if (t < g.nx) {
        const long long N = g.NX;
        const int i = t + HALO;
        double q[6];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            q[k] = S[k * N + i];
            ok = ok && isfinite(q[k]);
        }
        ok = ok && q[0] > 0.0 && pressure1(g.K, q[0], q[1], q[2]) > 0.0;
        bad = ok ? 0ull : 1ull;
    }
    bad = wsum(bad);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(&g.red->bad[0], (unsigned int)bad);
}

__global__ void k_copy_in1(Grid1 g, const double* __restrict__ U, double* __restrict__ S) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nx * 6) return;
    const int q = t / g.nx, i = t % g.nx;
    S[(long long)q * g.NX + i + HALO] = U[t];
}

__global__ void k_copy_out1(Grid1 g, const double* __restrict__ S, double* __restrict__ U) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nx * 6) return;
    const int q = t / g.nx, i = t % g.nx;
    U[t] = S[(long long)q * g.NX + i + HALO];
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_check1(const Grid1& g, const double* S, hipStream_t st) {
    k_check1<<<nb(g.nx, 128), 128, 0, st>>>(g, S);
    return hipGetLastError();
}

hipError_t launch_copy_in1(const Grid1& g, const double* U, double* S, hipStream_t st) {
    k_copy_in1<<<nb((long long)g.nx * 6, 256), 256, 0, st>>>(g, U, S);
    return hipGetLastError();
}

hipError_t launch_copy_out1(const Grid1& g, const double* S, double* U, hipStream_t st) {
    k_copy_out1<<<nb((long long)g.nx * 6, 256), 256, 0, st>>>(g, S, U);
    return hipGetLastError();
}

hipError_t launch_ghost1(const Grid1& g, double* S, hipStream_t st, Timer* tm) {
    tbeg(tm, KC_GHOST, st);
    k_ghost1<<<1, 64, 0, st>>>(g, S);
    tend(tm, st);
    return hipGetLastError();
}

hipError_t launch_residual1(const Grid1& g, const double* S, hipStream_t st, Timer* tm) {
    tbeg(tm, KC_RECON, st);
    if (g.K.dr) k_recon1<true><<<nb(g.NX - 2, 128), 128, 0, st>>>(g, S);
    else k_recon1<false><<<nb(g.NX - 2, 128), 128, 0, st>>>(g, S);
    tend(tm, st);
    if (g.K.dr) {   // the gradients and volume fluxes came with the reconstruction
        tbeg(tm, KC_FLUX, st);
        k_flux1<<<nb(g.nx + 1, 128), 128, 0, st>>>(g);
        tend(tm, st);
        return hipGetLastError();
    }
    tbeg(tm, KC_RBAR, st);
    k_rbar1<<<nb(g.NX - 4, 128), 128, 0, st>>>(g);
    tend(tm, st);
    tbeg(tm, KC_GRAD, st);
    k_grad1<<<nb(g.NX - 6, 128), 128, 0, st>>>(g);
    tend(tm, st);
    tbeg(tm, KC_FLUX, st);
    k_flux1<<<nb(g.nx + 1, 128), 128, 0, st>>>(g);
    tend(tm, st);
    return hipGetLastError();
}

hipError_t launch_update1(const Grid1& g, int stage, const double* S0, const double* Sin,
                          double* Sout, double* R, double* Vhat, hipStream_t st, Timer* tm,
                          const double* src) {
    tbeg(tm, KC_UPDATE, st);
    k_update1<<<nb(g.nx, 128), 128, 0, st>>>(g, stage, S0, Sin, Sout, R, Vhat, src);
    tend(tm, st);
    return hipGetLastError();
}

}  // namespace hw
