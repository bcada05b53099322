// Reverse mode (vector-Jacobian product) of the 1D HWENO-GR residual (Sec. 2,
// eqs. (2.2)-(2.9)): the adjoints of the forward kernels of hweno1d.hip in
// reverse order, one thread per face or cell.  The forward intermediates
// (limited LGL values, weak moments, gradients) are those of the residual the
// caller has just evaluated; the reconstruction is recomputed.  Branches of
// the forward point are kept (limiter thetas and their argmin points, the LF
// maximum and its side, |.| in the weights); ties go to the lowest index.
// Every sum is a fixed-order gather, so the results are bitwise reproducible.
//   k_adj1_flux    face fluxes (eq. (2.3))
//   k_adj1_grad    volume-flux quadrature and gradient reconstruction (eq. (2.9))
//   k_adj1_wmom    weak-derivative moments (eqs. (2.6)-(2.8)) -> LGL values
//   k_adj1_recon   PP limiter, back-transform, scalar HWENO, projection, basis
//   k_adj1_gather  state adjoint from the 3-cell stencils
//   k_adj1_ghost   ghost fill (Remark 4.1)

#include "hweno_vjp.h"

namespace hw {

namespace {

constexpr int HALO = 4;
constexpr int NT1 = 256;

__device__ __forceinline__ double lgl_w(int p) { return (p == 0 || p == 3) ? LGL_W0 : LGL_W1; }

// Seed of component q (0..5: F1 then F2) of the residual of ghosted cell i
// (zero outside the interior).
__device__ __forceinline__ double rseed(const AdjIn& A, const Grid1& g, int q, int i) {
    if (i < HALO || i >= HALO + g.nx) return 0.0;
    return A.rs * A.Rb[q * g.nx + (i - HALO)];
}

__global__ void k_fill1(double* p, long long n) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        p[k] = 0.0;
}

// Face i + 1/2, i = HALO-1 .. HALO+nx-1: fhat = 1/2 (f(U-) + f(U+) - beta (U+ - U-)),
// beta = max(speed1(U-), speed1(U+)).
template <bool VarMu>
__global__ __launch_bounds__(NT1) void k_adj1_flux(Grid1 g, AdjIn A, AdjWs1 W) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > g.nx) return;
    const Consts& K = g.K;
    const long long N = g.NX;
    const int i = HALO - 1 + f;
    double Um[3], Up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Um[c] = g.pts[(9 + c) * N + i];
        Up[c] = g.pts[c * N + i + 1];
    }
    const double umx = g.gr[6 * N + i], emx = g.gr[7 * N + i];
    const double upx = g.gr[0 * N + i + 1], epx = g.gr[1 * N + i + 1];
    // F1 = -(fr - fl) / dx and F2 = -(fl + fr) / (2 dx) + vf / dx of the cells
    // on both sides of the face
    double fb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        fb[c] = (-rseed(A, g, c, i) - 0.5 * rseed(A, g, 3 + c, i)) * K.idx +
                (rseed(A, g, c, i + 1) - 0.5 * rseed(A, g, 3 + c, i + 1)) * K.idx;
    const double spm = speed1(K, Um, umx, emx), spp = speed1(K, Up, upx, epx);
    const double beta = spm >= spp ? spm : spp;
    const double mum = VarMu ? point_mu1(K, Um) : K.mu_ref;
    const double mup = VarMu ? point_mu1(K, Up) : K.mu_ref;
    double Umb[3] = {0.0, 0.0, 0.0}, Upb[3] = {0.0, 0.0, 0.0};
    double umxb = 0.0, emxb = 0.0, upxb = 0.0, epxb = 0.0, mubm = 0.0, mubp = 0.0;
    double hf[3], betab = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        hf[c] = 0.5 * fb[c];
        Umb[c] += 0.5 * beta * fb[c];
        Upb[c] -= 0.5 * beta * fb[c];
        betab -= 0.5 * fb[c] * (Up[c] - Um[c]);
    }
    adj::flux1_vjp(K, Um, umx, emx, mum, hf, Umb, umxb, emxb, mubm);
    adj::flux1_vjp(K, Up, upx, epx, mup, hf, Upb, upxb, epxb, mubp);
    if (spm >= spp) speed1_vjp(K, Um, umx, emx, mum, betab, Umb, umxb, emxb, mubm);
    else speed1_vjp(K, Up, upx, epx, mup, betab, Upb, upxb, epxb, mubp);
    double mub = mubm + mubp;
    if constexpr (VarMu) mub = mubm * mu_T_vjp1(K, Um, mubm, Umb) + mubp * mu_T_vjp1(K, Up, mubp, Upb);
    // the face owns the minus side's point 3 and the plus side's point 0
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        W.ptsb[(9 + c) * N + i] += Umb[c];
        W.ptsb[c * N + i + 1] += Upb[c];
    }
    W.grb[6 * N + i] += umxb;
    W.grb[7 * N + i] += emxb;
    W.grb[0 * N + i + 1] += upxb;
    W.grb[1 * N + i + 1] += epxb;
    W.mupart[f] = mub;
}

// Cells 3 .. NX-4: the volume-flux quadrature (interior cells), then the
// gradient reconstruction from the weak moments (eq. (2.9)).
template <bool VarMu>
__global__ __launch_bounds__(NT1) void k_adj1_grad(Grid1 g, AdjIn A, AdjWs1 W) {
    const int i = 3 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > g.NX - 4) return;
    const Consts& K = g.K;
    const long long N = g.NX;
    double mub = 0.0;
    if (i >= HALO && i < HALO + g.nx) {
        double vb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) vb[c] = rseed(A, g, 3 + c, i) * K.idx;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double U[3], f[3], Ub[3] = {0.0, 0.0, 0.0}, uxb = 0.0, exb = 0.0, mubq = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                U[c] = g.pts[(p * 3 + c) * N + i];
                f[c] = lgl_w(p) * vb[c];
            }
            const double mu = VarMu ? point_mu1(K, U) : K.mu_ref;
            adj::flux1_vjp(K, U, g.gr[(p * 2) * N + i], g.gr[(p * 2 + 1) * N + i], mu, f, Ub, uxb,
                           exb, mubq);
            if constexpr (VarMu) mub += mubq * mu_T_vjp1(K, U, mubq, Ub);
            else mub += mubq;
#pragma unroll
            for (int c = 0; c < 3; ++c) W.ptsb[(p * 3 + c) * N + i] += Ub[c];
            W.grb[(p * 2) * N + i] += uxb;
            W.grb[(p * 2 + 1) * N + i] += exb;
        }
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double* r0 = g.rb + (w * 2 + 0) * N;
        const double* r1 = g.rb + (w * 2 + 1) * N;
        const double a[5] = {r0[i - 1], r0[i], r0[i + 1], r1[i - 1], r1[i + 1]};
        double yb[4], Cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, ab[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < 4; ++p) yb[p] = W.grb[(p * 2 + w) * N + i];
        adj::lgl_T(yb, Cb);
        hweno1d_vjp(a, grad_consts(K), Cb, ab);
#pragma unroll
        for (int s = 0; s < 5; ++s) W.rbc[(w * 5 + s) * N + i] = ab[s];
    }
    W.mupart[g.nx + 1 + i] = mub;
}

// Cells 1 .. NX-2: adjoints of this cell's LGL values through the weak
// moments of the cells j-1, j, j+1 (cells 2 .. NX-3 carry weak moments):
// r0 = (hp - hm) / dx, r1 = ((hp + hm) / 2 - wbar) / dx, with the interface
// averages hm = (w(j-1, 3) + w(j, 0)) / 2, hp = (w(j, 3) + w(j+1, 0)) / 2 of
// w = (u, e) and wbar the LGL quadrature of w.
__global__ __launch_bounds__(NT1) void k_adj1_wmom(Grid1 g, AdjWs1 W) {
    const int j = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (j > g.NX - 2) return;
    const long long N = g.NX;
    const double idx = g.K.idx;
    auto RC = [&](int w, int s, int ii) -> double {
        return (ii >= 3 && ii <= g.NX - 4) ? W.rbc[(w * 5 + s) * N + ii] : 0.0;
    };
    // adjoints of hp, hm and wbar of cell ii (zero outside 2 .. NX-3)
    auto hbar = [&](int ii, int w, double& hp, double& hm, double& wbb) {
        hp = hm = wbb = 0.0;
        if (ii < 2 || ii > g.NX - 3) return;
        const double b0 = RC(w, 0, ii + 1) + RC(w, 1, ii) + RC(w, 2, ii - 1);
        const double b1 = RC(w, 3, ii + 1) + RC(w, 4, ii - 1);
        hp = (b0 + 0.5 * b1) * idx;
        hm = (-b0 + 0.5 * b1) * idx;
        wbb = -b1 * idx;
    };
    double pb[4][2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        double hpj, hmj, wbj, hpl, hml, wbl, hpr, hmr, wbr;
        hbar(j, w, hpj, hmj, wbj);
        hbar(j - 1, w, hpl, hml, wbl);
        hbar(j + 1, w, hpr, hmr, wbr);
#pragma unroll
        for (int p = 0; p < 4; ++p) pb[p][w] = lgl_w(p) * wbj;
        pb[0][w] += 0.5 * hmj + 0.5 * hpl;
        pb[3][w] += 0.5 * hpj + 0.5 * hmr;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double U[3], Ub[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 3; ++c) U[c] = g.pts[(p * 3 + c) * N + j];
        adj::prim1_vjp(U, pb[p], Ub);
#pragma unroll
        for (int c = 0; c < 3; ++c) W.ptsb[(p * 3 + c) * N + j] += Ub[c];
    }
}

// Cells 1 .. NX-2: the reconstruction recomputed as k_recon1 forms it, then
// the adjoints of the limiter, the back-transform, the three scalar
// reconstructions, the projection and the characteristic basis.  Writes the
// cell's contributions to the state adjoints of its stencil: uc slot s = 0, 1,
// 2 the averages of cells i-1, i, i+1 (slot 1 with the cell's own basis and
// limiter terms), s = 3, 4 the moments of cells i-1, i+1.
__global__ __launch_bounds__(NT1) void k_adj1_recon(Grid1 g, AdjIn A, AdjWs1 W, const double* __restrict__ S) {
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > g.NX - 2) return;
    const Consts& K = g.K;
    const long long N = g.NX;
    double ub[3], st[5][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ub[c] = S[c * N + i];
        st[0][c] = S[c * N + i - 1];
        st[1][c] = S[c * N + i];
        st[2][c] = S[c * N + i + 1];
        st[3][c] = S[(3 + c) * N + i - 1];
        st[4][c] = S[(3 + c) * N + i + 1];
    }
    Eig1 e;
    eig1(K, ub, e);
    // ---- forward recompute ----
    double a[3][5], v[3][4], mo[3];
    double P0[4][3] = {{0.0}}, vh[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int s = 0; s < 5; ++s) a[k][s] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double l = e.L[k][c];
#pragma unroll
            for (int s = 0; s < 5; ++s) a[k][s] += l * st[s][c];
        }
        double C[5];
        hweno1d(a[k], K, C);
        eval1d(C, v[k]);
        mo[k] = moment1d(C);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int p = 0; p < 4; ++p) P0[p][c] += e.R[c][k] * v[k][p];
            vh[c] += e.R[c][k] * mo[k];
        }
    }
    const double rbar = ub[0];
    const double pbar = pressure1(K, ub[0], ub[1], ub[2]);
    const double e1 = K.eps_pp <= rbar ? K.eps_pp : rbar;
    const int esrc1 = K.eps_pp <= rbar ? 0 : 1;
    const double eps = e1 <= pbar ? e1 : pbar;
    const int esrc = e1 <= pbar ? esrc1 : 2;
    double rmin = P0[0][0];
    int p1 = 0;
#pragma unroll
    for (int p = 1; p < 4; ++p)
        if (P0[p][0] < rmin) {
            rmin = P0[p][0];
            p1 = p;
        }
    const bool low1 = rmin < eps;
    const double th1 = low1 ? (rbar - eps) / (rbar - rmin) : 1.0;
    double P1[4][3];
    double tmin = INFINITY;
    int p2 = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        P1[p][0] = rbar + th1 * (P0[p][0] - rbar);
        P1[p][1] = P0[p][1];
        P1[p][2] = P0[p][2];
        const double pt = pressure1(K, P1[p][0], P1[p][1], P1[p][2]);
        const double t = pt < eps ? (pbar - eps) / (pbar - pt) : 1.0;
        if (t < tmin) {
            tmin = t;
            p2 = p;
        }
    }
    const bool low2 = tmin < 1.0;
    const double th2 = low2 ? tmin : 1.0;
    // ---- limiter adjoint: P = ub + th2 (P1 - ub) ----
    double ubb[3] = {0.0, 0.0, 0.0}, P1b[4][3], th2b = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double pb = W.ptsb[(p * 3 + c) * N + i];
            P1b[p][c] = th2 * pb;
            ubb[c] += (1.0 - th2) * pb;
            th2b += pb * (P1[p][c] - ub[c]);
        }
    }
    double rbb = 0.0, pbb = 0.0, epsb = 0.0;
    if (low2) {
        const double pt = pressure1(K, P1[p2][0], P1[p2][1], P1[p2][2]);
        const double den = pbar - pt;
        pbb += th2b * (eps - pt) / (den * den);
        epsb -= th2b / den;
        adj::pres1_vjp(K, P1[p2], th2b * (pbar - eps) / (den * den), P1b[p2]);
    }
    // P1[p][0] = rbar + th1 (P0[p][0] - rbar)
    double P0b[4][3], th1b = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        P0b[p][0] = th1 * P1b[p][0];
        P0b[p][1] = P1b[p][1];
        P0b[p][2] = P1b[p][2];
        rbb += (1.0 - th1) * P1b[p][0];
        th1b += P1b[p][0] * (P0[p][0] - rbar);
    }
    if (low1) {
        const double den = rbar - rmin;
        rbb += th1b * (eps - rmin) / (den * den);
        epsb -= th1b / den;
        P0b[p1][0] += th1b * (rbar - eps) / (den * den);
    }
    if (esrc == 1) rbb += epsb;
    if (esrc == 2) pbb += epsb;
    ubb[0] += rbb;
    if (pbb != 0.0) adj::pres1_vjp(K, ub, pbb, ubb);
    // ---- back-transform adjoint: P0[p][c] = sum_k R[c][k] v_k[p], vh[c] = sum_k R[c][k] mo_k ----
    double vhb[3] = {0.0, 0.0, 0.0};
    if (A.Vb && i >= HALO && i < HALO + g.nx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vhb[c] = A.vs * A.Vb[c * g.nx + (i - HALO)];
    }
    double lb[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rb[9];
    double ucs[5][3] = {{0.0}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double acc = vhb[c] * mo[k];
#pragma unroll
            for (int p = 0; p < 4; ++p) acc += P0b[p][c] * v[k][p];
            rb[c * 3 + k] = acc;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double vb[4], mob = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc += e.R[c][k] * P0b[p][c];
            vb[p] = acc;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) mob += e.R[c][k] * vhb[c];
        // ---- scalar reconstruction and projection adjoints ----
        double Cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, ab[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        adj::lgl_T(vb, Cb);
        moment1d_T(mob, Cb);
        hweno1d_vjp(a[k], K, Cb, ab);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                acc += ab[s] * st[s][c];
                ucs[s][c] += e.L[k][c] * ab[s];
            }
            lb[k * 3 + c] = acc;
        }
    }
    adj::eig1_vjp(K, ub, lb, rb, ubb);
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) W.uc[(s * 3 + c) * N + i] = ucs[s][c] + (s == 1 ? ubb[c] : 0.0);
}

// Cells 0 .. NX-1: state adjoint gathered from the stencils of the cells
// that reconstruct (1 .. NX-2).
__global__ __launch_bounds__(NT1) void k_adj1_gather(Grid1 g, AdjWs1 W) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.NX) return;
    const long long N = g.NX;
    auto UC = [&](int s, int c, int ii) -> double {
        return (ii >= 1 && ii <= g.NX - 2) ? W.uc[(s * 3 + c) * N + ii] : 0.0;
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        W.ub[c * N + j] = UC(2, c, j - 1) + UC(1, c, j) + UC(0, c, j + 1);
        W.ub[(3 + c) * N + j] = UC(4, c, j - 1) + UC(3, c, j + 1);
    }
}

// Ghost fill adjoint, one thread in a fixed order: each ghost cell's adjoint
// goes to the interior cell it copies (with the wall signs); inflow ghosts
// hold a constant state and pass nothing on.
__global__ void k_adj1_ghost(Grid1 g, AdjWs1 W) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const long long N = g.NX;
    for (int right = 0; right < 2; ++right) {
        const Side& sd = g.side[right];
        for (int d = 1; d <= HALO; ++d) {
            int di, si;
            if (!right) {
                di = HALO - d;
                si = sd.kind == 0 ? HALO + g.nx - d : (sd.kind == 1 ? HALO : HALO + d - 1);
            } else {
                di = HALO + g.nx - 1 + d;
                si = sd.kind == 0 ? HALO + d - 1 : (sd.kind == 1 ? HALO + g.nx - 1 : HALO + g.nx - d);
            }
            for (int q = 0; q < 6; ++q) {
                if (sd.kind != 2) W.ub[q * N + si] += sd.sign[q] * W.ub[q * N + di];
                W.ub[q * N + di] = 0.0;
            }
        }
    }
}

__global__ void k_adj1_out(Grid1 g, AdjWs1 W, double* __restrict__ Ubar) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * g.nx) return;
    const int q = t / g.nx, x = t % g.nx;
    Ubar[t] = W.ub[(long long)q * g.NX + HALO + x];
}

// mu-bar = sum of the partials in a fixed order (one block).
__global__ void k_mu_sum1(const double* __restrict__ part, int n, double* out, int acc) {
    __shared__ double sh[NT1];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += NT1) s += part[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = NT1 / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = acc ? *out + sh[0] : sh[0];
}

unsigned nb1(long long n) { return (unsigned)((n + NT1 - 1) / NT1); }

}  // namespace

hipError_t launch_vjp1(const Grid1& g, const AdjIn& A, AdjWs1 W, const double* S, double* Ubar,
                       double* mu_out, int mu_acc, hipStream_t st) {
    k_fill1<<<nb1(W.count) < 1024 ? nb1(W.count) : 1024, NT1, 0, st>>>(W.base, W.count);
    if (g.K.mu_exp != 0.0) {   // mu(T): the viscosity's dependence on the state too
        k_adj1_flux<true><<<nb1(g.nx + 1), NT1, 0, st>>>(g, A, W);
        k_adj1_grad<true><<<nb1(g.NX - 6), NT1, 0, st>>>(g, A, W);
    } else {
        k_adj1_flux<false><<<nb1(g.nx + 1), NT1, 0, st>>>(g, A, W);
        k_adj1_grad<false><<<nb1(g.NX - 6), NT1, 0, st>>>(g, A, W);
    }
    k_adj1_wmom<<<nb1(g.NX - 2), NT1, 0, st>>>(g, W);
    k_adj1_recon<<<nb1(g.NX - 2), NT1, 0, st>>>(g, A, W, S);
    k_adj1_gather<<<nb1(g.NX), NT1, 0, st>>>(g, W);
    k_adj1_ghost<<<1, 64, 0, st>>>(g, W);
    k_adj1_out<<<nb1(6LL * g.nx), NT1, 0, st>>>(g, W, Ubar);
    k_mu_sum1<<<1, NT1, 0, st>>>(W.mupart, g.NX + g.nx + 1, mu_out, mu_acc);
    return hipGetLastError();
}

}  // namespace hw
