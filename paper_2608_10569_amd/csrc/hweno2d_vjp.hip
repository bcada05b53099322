// Reverse mode (vector-Jacobian product) of the 2D HWENO-GR residual of
// arXiv 2608.10569 (eq. (3.2) with eqs. (3.3)-(3.9)): given the adjoints of
// the residual R and of the modified moments, the adjoint of the input state
// and of the viscosity mu_ref.
//
// The forward pipeline is recomputed first (its intermediates stay in the
// workspace); the adjoint kernels then run in reverse order.  Every adjoint
// slot has exactly one writer and cross-cell sums are gathers in a fixed
// order, so the result is deterministic (no floating-point atomics).
// Branches (limiter thetas, LF-speed maximum, |.| in the weights) follow the
// forward point; ties go to the lowest index in the order of the oracle.
//
//   k_adj_flux<d>  face-flux adjoint (eq. (3.3)) -> trace / face-gradient adjoints
//   k_adj_grad     volume-flux + gradient-reconstruction adjoint (eq. (3.9))
//   k_adj_rgather  gather of the weak-moment adjoints from the 3x3 stencils
//   k_adj_wmom     weak-moment adjoint (eqs. (3.6)-(3.8)) -> trace / volume adjoints
//   k_adj_recon_a  forward recompute; limiter and back-transform adjoints
//   k_adj_recon_b  scalar HWENO, eigen-system and projection adjoints
//   k_adj_ugather  gather of the state adjoint from the 3x3 stencils
//   k_adj_ghost_out adjoint of the ghost fill (Remark 4.1), written to the output
//   k_mu_sum       fixed-order sum of the mu-adjoint block partials

#include "hweno_adj.h"
#include "hweno_vjp.h"

namespace hw {

namespace {

constexpr int HALO = 4;

__device__ __forceinline__ double gw(int g) { return g == 1 ? GW1 : GW0; }
__device__ __forceinline__ double gx(int g) { return g == 0 ? -GS : (g == 1 ? 0.0 : GS); }

__device__ __forceinline__ bool interior(const Grid2& g, int j, int i) {
    return j >= HALO && j < HALO + g.ny && i >= HALO && i < HALO + g.nx;
}

// Whether face f (0 left, 1 right, 2 bottom, 3 top) of cell (j, i) is one of
// the faces k_adj_flux visits (the faces of the interior cells): its trace
// and gradient adjoints are then assigned there, and later kernels add to
// them; the other slots the later kernels assign (or read as zero), so the
// adjoint workspace needs no clearing.
__device__ __forceinline__ bool flux_face(const Grid2& g, int j, int i, int f) {
    if (f < 2) {
        if (j < HALO || j >= HALO + g.ny) return false;
        return f == 0 ? (i >= HALO && i <= HALO + g.nx) : (i >= HALO - 1 && i <= HALO + g.nx - 1);
    }
    if (i < HALO || i >= HALO + g.nx) return false;
    return f == 2 ? (j >= HALO && j <= HALO + g.ny) : (j >= HALO - 1 && j <= HALO + g.ny - 1);
}

// Solid cell of a masked grid (interior index t)
__device__ __forceinline__ bool solid_cell(const Grid2& g, long long t) {
    return g.solid && g.solid[t];
}

// residual adjoint of interior cell (j, i): F1, F2, F3 component c (on a
// masked grid the seeds come with the solid cells' zeroed, k_mask_seeds)
__device__ __forceinline__ double rbar(const AdjIn& A, const Grid2& g, int m, int c, int j, int i) {
    const long long nint = (long long)g.nx * g.ny;
    return A.rs * A.Rb[(m * 4 + c) * nint + (long long)(j - HALO) * g.nx + (i - HALO)];
}

// Logical index of this block: XCD-aware (each XCD takes a contiguous range
// of the launch, so neighbouring rows of a stencil share an L2), last first
// where bit k of W.rev is set (k: 0, 1 face fluxes x, y; 2 gradients; 3
// weak-moment gather; 4 weak moments; 5, 7 the two reconstruction kernels;
// 6 state gather).
// The mu partials are stored by it, so their fixed summation order is
// unchanged.
__device__ __forceinline__ int lblock(const AdjWs& W, int k) {
    return xcd_block((int)blockIdx.x, (int)gridDim.x, (W.rev >> k) & 1u);
}

// fixed-order block sum of the mu adjoint: one partial per (logical) block;
// a butterfly within each wavefront, then the wavefronts' sums in order
template <int NT>
__device__ __forceinline__ void mu_partial(double v, double* part, int lb) {
    static_assert(NT % 64 == 0, "whole wavefronts");
    __shared__ double sh[NT / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += sh[w];
        part[lb] = s;
    }
}

// ---------------------------------------------------------------------------
// Face fluxes: fhat = 1/2 (f(u-,s-) + f(u+,s+) - beta (u+ - u-)), beta the
// max over the face's 3 Gauss points x 2 sides of max(|u_n| + c, beta_PP).
// Block: 3 Gauss points x 64 faces.
// ---------------------------------------------------------------------------
constexpr int AF = 64;

template <int d, bool VarMu>
__global__ __launch_bounds__(3 * AF) void k_adj_flux(Grid2 g, AdjIn A, AdjWs W) {
    __shared__ double shs[2][3 * AF];     // speeds of the two sides
    __shared__ double shb[3 * AF];        // beta-bar partial sums
    const Consts& K = g.K;
    const int nfi = d == 0 ? g.nx + 1 : g.nx;
    const int nfj = d == 0 ? g.ny : g.ny + 1;
    const int G = threadIdx.x / AF;
    const int fl = threadIdx.x % AF;
    const int lb = lblock(W, d);
    const long long t = (long long)lb * AF + fl;
    const bool valid = t < (long long)nfi * nfj;
    const long long N = g.ncell;
    int j = HALO, i = HALO;
    if (valid) {
        const int fj = (int)(t / nfi), fi = (int)(t % nfi);
        j = d == 0 ? HALO + fj : HALO - 1 + fj;
        i = d == 0 ? HALO - 1 + fi : HALO + fi;
    }
    const long long cm = (long long)j * g.NX + i;
    const long long cp = d == 0 ? cm + 1 : cm + g.NX;
    const int jp = d == 0 ? j : j + 1, ip = d == 0 ? i + 1 : i;
    const double* F = d == 0 ? g.xf : g.yf;
    const int pg = d == 0 ? 0 : 6;
    double Um[4], Up[4], sm[6], sp[6];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        Um[c] = F[((3 + G) * 4 + c) * N + cm];
        Up[c] = F[(G * 4 + c) * N + cp];
    }
#pragma unroll
    for (int z = 0; z < 6; ++z) {
        sm[z] = g.gf[((pg + 3 + G) * 6 + z) * N + cm];
        sp[z] = g.gf[((pg + G) * 6 + z) * N + cp];
    }
    const double spm = speed2<d>(K, Um, sm), spp = speed2<d>(K, Up, sp);
    shs[0][threadIdx.x] = valid ? spm : -INFINITY;
    shs[1][threadIdx.x] = valid ? spp : -INFINITY;
    // adjoint of fhat at this Gauss point from the two adjacent residuals
    double fb[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        const double w = gw(G), x = gx(G);
        const bool im = interior(g, j, i), ipn = interior(g, jp, ip);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double v = 0.0;
            if (d == 0) {
                if (im) v += -w * K.idx * rbar(A, g, 0, c, j, i) - 0.5 * w * K.idx * rbar(A, g, 1, c, j, i)
                             - w * x * K.idx * rbar(A, g, 2, c, j, i);
                if (ipn) v += w * K.idx * rbar(A, g, 0, c, jp, ip) - 0.5 * w * K.idx * rbar(A, g, 1, c, jp, ip)
                              + w * x * K.idx * rbar(A, g, 2, c, jp, ip);
            } else {
                if (im) v += -w * K.idy * rbar(A, g, 0, c, j, i) - w * x * K.idy * rbar(A, g, 1, c, j, i)
                             - 0.5 * w * K.idy * rbar(A, g, 2, c, j, i);
                if (ipn) v += w * K.idy * rbar(A, g, 0, c, jp, ip) + w * x * K.idy * rbar(A, g, 1, c, jp, ip)
                              - 0.5 * w * K.idy * rbar(A, g, 2, c, jp, ip);
            }
            fb[c] = v;
        }
    }
    __syncthreads();
    // beta and its argmax in the order (minus side G = 0,1,2, plus side G = 0,1,2)
    double beta = -INFINITY;
    int arg = 0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double v = shs[side][q * AF + fl];
            if (v > beta) {
                beta = v;
                arg = side * 3 + q;
            }
        }
    }
    double Umb[4] = {0.0, 0.0, 0.0, 0.0}, Upb[4] = {0.0, 0.0, 0.0, 0.0};
    double smb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, spb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mub = 0.0, betab = 0.0;
    // the viscosity at the point on each side: mu_ref, or mu(T) of that
    // side's state, whose adjoint (mbm, mbp) is chained through T below
    const double mum = VarMu ? point_mu(K, Um) : K.mu_ref;
    const double mup = VarMu ? point_mu(K, Up) : K.mu_ref;
    double mubm = 0.0, mubp = 0.0;
    double& mbm = VarMu ? mubm : mub;
    double& mbp = VarMu ? mubp : mub;
    if (valid) {
        double hf[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            hf[c] = 0.5 * fb[c];
            Umb[c] += 0.5 * beta * fb[c];
            Upb[c] -= 0.5 * beta * fb[c];
            betab -= 0.5 * fb[c] * (Up[c] - Um[c]);
        }
        flux2_vjp<d>(K, Um, sm, mum, hf, Umb, smb, mbm);
        flux2_vjp<d>(K, Up, sp, mup, hf, Upb, spb, mbp);
    }
    shb[threadIdx.x] = betab;
    __syncthreads();
    if (valid && arg % 3 == G) {
        const double bsum = shb[fl] + shb[AF + fl] + shb[2 * AF + fl];
        if (arg < 3) speed2_vjp<d>(K, Um, sm, mum, bsum, Umb, smb, mbm);
        else speed2_vjp<d>(K, Up, sp, mup, bsum, Upb, spb, mbp);
    }
    if constexpr (VarMu) {
        if (valid) mub = mubm * mu_T_vjp(K, Um, mubm, Umb) + mubp * mu_T_vjp(K, Up, mubp, Upb);
    }
    if (valid) {
        double* XB = d == 0 ? W.xfb : W.yfb;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            XB[((3 + G) * 4 + c) * N + cm] = Umb[c];
            XB[(G * 4 + c) * N + cp] = Upb[c];
        }
#pragma unroll
        for (int z = 0; z < 6; ++z) {
            W.gfb[((pg + 3 + G) * 6 + z) * N + cm] = smb[z];
            W.gfb[((pg + G) * 6 + z) * N + cp] = spb[z];
        }
    }
    mu_partial<3 * AF>(valid ? mub : 0.0, W.mupart + (d == 0 ? 0 : W.mu_off1), lb);
}

// ---------------------------------------------------------------------------
// Gradient reconstruction (and, on interior cells, the volume fluxes).
// Block: 32 cells x 6 gradient components s = 2 w + l.
// ---------------------------------------------------------------------------
constexpr int AG = 32;

template <bool VarMu>
__global__ __launch_bounds__(6 * AG) void k_adj_grad(Grid2 g, AdjIn A, AdjWs W) {
    __shared__ double shv[6 * 9 * AG];       // forward volume gradients
    __shared__ double shvb[2][6 * 9 * AG];   // their adjoints from f and from g
    const Consts& K = g.K;
    const int tid = threadIdx.x;
    const int cl = tid % AG;
    const int s = tid / AG;
    const int w = s >> 1, l = s & 1;
    const int wc = g.NX - 6;
    const long long nreg = (long long)wc * (g.NY - 6);
    const int lb = lblock(W, 2);
    const long long cid = (long long)lb * AG + cl;
    const bool valid = cid < nreg;
    int j = 3, i = 3;
    if (valid) {
        j = 3 + (int)(cid / wc);
        i = 3 + (int)(cid % wc);
    }
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    const double* R0 = g.rb + ((l * 3 + w) * 3 + 0) * N;
    const double* R1 = g.rb + ((l * 3 + w) * 3 + 1) * N;
    const double* R2 = g.rb + ((l * 3 + w) * 3 + 2) * N;
    double a[17];
#pragma unroll
    for (int q = 0; q < 9; ++q) a[q] = R0[cell + (long long)(q / 3 - 1) * g.NX + (q % 3 - 1)];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = 2 * e + 1;
        const long long nb = cell + (long long)(q / 3 - 1) * g.NX + (q % 3 - 1);
        a[9 + e] = R1[nb];
        a[13 + e] = R2[nb];
    }
    double C[15], vo[9];
    hweno2d(a, grad_consts(K), C);
    eval_vol(C, vo);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        shv[(s * 9 + q) * AG + cl] = vo[q];
        shvb[0][(s * 9 + q) * AG + cl] = 0.0;
        shvb[1][(s * 9 + q) * AG + cl] = 0.0;
    }
    __syncthreads();
    const bool inter = valid && interior(g, j, i);
    double mub = 0.0;
    if (inter) {
        // volume flux: vf = sum_q w_q f(U_q, s_q); vf-bar = F2-bar/dx (f), F3-bar/dy (g).
        // The 18 point adjoints over the cell's 6 threads: direction dv = s / 3,
        // points 3 (s % 3) .. 3 (s % 3) + 2
        const int dv = s / 3, q0 = 3 * (s % 3);
        double fb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            fb[c] = dv == 0 ? rbar(A, g, 1, c, j, i) * K.idx : rbar(A, g, 2, c, j, i) * K.idy;
        const double* V = dv == 0 ? g.xv : g.yv;
        double* VB = dv == 0 ? W.xvb : W.yvb;
        for (int q = q0; q < q0 + 3; ++q) {
            const double wq = gw(q / 3) * gw(q % 3);
            double Uq[4], sq[6], Uqb[4] = {0.0, 0.0, 0.0, 0.0}, sqb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            double f[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Uq[c] = V[(q * 4 + c) * N + cell];
                f[c] = wq * fb[c];
            }
#pragma unroll
            for (int z = 0; z < 6; ++z) sq[z] = shv[(z * 9 + q) * AG + cl];
            const double muq = VarMu ? point_mu(K, Uq) : K.mu_ref;
            double mubq = 0.0;
            double& mb = VarMu ? mubq : mub;
            if (dv == 0) flux2_vjp<0>(K, Uq, sq, muq, f, Uqb, sqb, mb);
            else flux2_vjp<1>(K, Uq, sq, muq, f, Uqb, sqb, mb);
            if constexpr (VarMu) mub += mubq * mu_T_vjp(K, Uq, mubq, Uqb);
#pragma unroll
            for (int c = 0; c < 4; ++c) VB[(q * 4 + c) * N + cell] = Uqb[c];
#pragma unroll
            for (int z = 0; z < 6; ++z) shvb[dv][(z * 9 + q) * AG + cl] = sqb[z];
        }
    }
    __syncthreads();
    // adjoint of this component's 21 point values
    double yb[21];
#pragma unroll
    for (int p = 0; p < 12; ++p)
        yb[p] = flux_face(g, j, i, p / 3) ? g_ld(W.gfb, (p * 6 + s) * N + cell) : 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q)
        yb[12 + q] = shvb[0][(s * 9 + q) * AG + cl] + shvb[1][(s * 9 + q) * AG + cl];
    double Cb[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) Cb[k] = 0.0;
    adj::xface_T(yb, Cb);
    adj::yface_T(yb + 6, Cb);
    adj::vol_T(yb + 12, Cb);
    double ab[17];
    hweno2d_vjp(a, grad_consts(K), Cb, ab);
    if (valid) {
#pragma unroll
        for (int k = 0; k < 17; ++k) W.rbc[(s * 17 + k) * N + cell] = ab[k];
    }
    mu_partial<6 * AG>(mub, W.mupart + W.mu_off2, lb);
}

// ---------------------------------------------------------------------------
// Gather of the weak-moment adjoints: cell X is slot k of the 3x3 stencil of
// cell X - off(k).  Cells of halo ring 2.
// ---------------------------------------------------------------------------
__global__ void k_adj_rgather(Grid2 g, AdjWs W) {
    const int wc = g.NX - 4;
    const long long nreg = (long long)wc * (g.NY - 4);
    const long long cid = (long long)lblock(W, 3) * blockDim.x + threadIdx.x;
    if (cid >= nreg) return;
    const int j = 2 + (int)(cid / wc), i = 2 + (int)(cid % wc);
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    for (int s = 0; s < 6; ++s) {
        const int w = s >> 1, l = s & 1;
        double m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int ox = k % 3 - 1, oy = k / 3 - 1;
            const int yj = j - oy, yi = i - ox;
            if (yj < 3 || yj > g.NY - 4 || yi < 3 || yi > g.NX - 4) continue;   // not in ring 1
            const long long Y = (long long)yj * g.NX + yi;
            m0 += W.rbc[(s * 17 + k) * N + Y];
            if (k & 1) {
                const int e = k >> 1;     // k = 1, 3, 5, 7 -> edge slot 0..3
                m1 += W.rbc[(s * 17 + 9 + e) * N + Y];
                m2 += W.rbc[(s * 17 + 13 + e) * N + Y];
            }
        }
        W.rbb[((l * 3 + w) * 3 + 0) * N + cell] = m0;
        W.rbb[((l * 3 + w) * 3 + 1) * N + cell] = m1;
        W.rbb[((l * 3 + w) * 3 + 2) * N + cell] = m2;
    }
}

// ---------------------------------------------------------------------------
// Weak-moment adjoint (eqs. (3.6)-(3.8)) on cells X of ring 3 (every cell
// with a reconstruction): its four faces' interface averages take adjoints
// from the weak moments of both adjacent cells; half goes to each trace.
// The wbar adjoint goes to the volume values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_ring2(const Grid2& g, int j, int i) {
    return j >= 2 && j <= g.NY - 3 && i >= 2 && i <= g.NX - 3;
}

// Six independent tasks per cell, one per wavefront of the block: tasks 0..3
// the four faces (left, right, bottom, top), tasks 4..5 the volume values of
// the x and y bases.  Every task owns the cotangent slots it adds to.
constexpr int WM_CELLS = 64;

__global__ __launch_bounds__(6 * WM_CELLS) void k_adj_wmom(Grid2 g, AdjWs W) {
    const int task = threadIdx.x / WM_CELLS;
    const int wc = g.NX - 2;
    const long long nreg = (long long)wc * (g.NY - 2);
    const long long cid = (long long)lblock(W, 4) * WM_CELLS + threadIdx.x % WM_CELLS;
    if (cid >= nreg) return;
    const int j = 1 + (int)(cid / wc), i = 1 + (int)(cid % wc);
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    const double idx = g.K.idx, idy = g.K.idy;
    auto RB = [&](int jj, int ii, int l, int w, int mom) -> double {
        if (!in_ring2(g, jj, ii)) return 0.0;
        return W.rbb[((l * 3 + w) * 3 + mom) * N + (long long)jj * g.NX + ii];
    };
    if (task < 4) {
        // face `task`: 0 left (x, this cell is the plus side), 1 right (minus
        // side), 2 bottom (y, plus side), 3 top (minus side)
        const int face = task;
        const int dir = face >> 1;
        const bool hi = face & 1;
        const int oj = dir == 1 ? (hi ? 1 : -1) : 0, oi = dir == 0 ? (hi ? 1 : -1) : 0;
        const double* F = dir == 0 ? g.xf : g.yf;
        double* FB = dir == 0 ? W.xfb : W.yfb;
        const double ih = dir == 0 ? idx : idy;
        double W0b[3], W1b[3];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            // contributions of this cell (face on its hi side or lo side) and of the neighbour
            const double own0 = RB(j, i, dir, w, 0);
            const double ownm = RB(j, i, dir, w, dir == 0 ? 1 : 2);      // the (W0+ + W0-)/2 moment
            const double own1 = RB(j, i, dir, w, dir == 0 ? 2 : 1);      // the transverse moment
            const double nb0 = RB(j + oj, i + oi, dir, w, 0);
            const double nbm = RB(j + oj, i + oi, dir, w, dir == 0 ? 1 : 2);
            const double nb1 = RB(j + oj, i + oi, dir, w, dir == 0 ? 2 : 1);
            if (hi) {   // this cell's upper face = neighbour's lower face
                W0b[w] = (own0 + 0.5 * ownm) * ih + (-nb0 + 0.5 * nbm) * ih;
                W1b[w] = own1 * ih - nb1 * ih;
            } else {
                W0b[w] = (-own0 + 0.5 * ownm) * ih + (nb0 + 0.5 * nbm) * ih;
                W1b[w] = -own1 * ih + nb1 * ih;
            }
        }
#pragma unroll
        for (int G = 0; G < 3; ++G) {
            const int p = (hi ? 3 : 0) + G;
            double U[4], wb[3], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) U[c] = F[(p * 4 + c) * N + cell];
#pragma unroll
            for (int w = 0; w < 3; ++w) wb[w] = 0.5 * gw(G) * (W0b[w] + gx(G) * W1b[w]);
            adj::prim2_vjp(U, wb, Ub);
            const bool add = flux_face(g, j, i, dir * 2 + (hi ? 1 : 0));
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double& x = FB[(p * 4 + c) * N + cell];
                x = add ? x + Ub[c] : Ub[c];
            }
        }
    } else if (!in_ring2(g, j, i)) {
        // no weak moments here: the volume-value adjoints are zero
        double* VB = task == 4 ? W.xvb : W.yvb;
        for (int q = 0; q < 36; ++q) VB[q * N + cell] = 0.0;
    } else {
        // wbar adjoint of this cell's own weak moments, to its volume values
        // (added to the volume-flux adjoints on interior cells)
        const int dir = task - 4;
        const bool add = interior(g, j, i);
        const double* V = dir == 0 ? g.xv : g.yv;
        double* VB = dir == 0 ? W.xvb : W.yvb;
        double wbb[3];
#pragma unroll
        for (int w = 0; w < 3; ++w)
            wbb[w] = -RB(j, i, dir, w, dir == 0 ? 1 : 2) * (dir == 0 ? idx : idy);
        for (int q = 0; q < 9; ++q) {
            const double wq = gw(q / 3) * gw(q % 3);
            double U[4], wb[3], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) U[c] = V[(q * 4 + c) * N + cell];
#pragma unroll
            for (int w = 0; w < 3; ++w) wb[w] = wq * wbb[w];
            adj::prim2_vjp(U, wb, Ub);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double& x = VB[(q * 4 + c) * N + cell];
                x = add ? x + Ub[c] : Ub[c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Characteristic reconstruction adjoint, in two kernels over the same cells.
// Block: 16 cells x 8 threads (b = basis, k = characteristic field /
// conservative component).
//   k_adj_recon_a: forward recompute (scalar HWENO, back-transform, limiter),
//     adjoint of the limiter and of the back-transform: the cotangents of
//     the 16 characteristic outputs of every (cell, b, k), the R-bar rows and
//     the limiter's share of the cell-average adjoint go to the workspace;
//   k_adj_recon_b: the scalar HWENO adjoint, the eigen-system adjoint and the
//     projection adjoint.
// Split, each kernel keeps fewer values live and less LDS per block than the
// one kernel before it (256 VGPRs plus spill space, 75 KB of LDS, one wave
// per SIMD).
// ---------------------------------------------------------------------------
constexpr int AC = 16;

__device__ __forceinline__ int pt_index(int b, int o) { return o < 6 ? b * 6 + o : 12 + b * 9 + (o - 6); }

__global__ __launch_bounds__(8 * AC) void k_adj_recon_a(Grid2 g, AdjIn A, AdjWs W,
                                                        const double* __restrict__ S) {
    __shared__ double shc[8 * 16 * AC];   // characteristic point values (b, f, o)
    // conservative point values (b, c, o); once the limiter adjoint has read
    // them, the adjoints of the conservative values
    __shared__ double shu[8 * 16 * AC];
    __shared__ double shr[8 * AC];        // reductions (value)
    __shared__ int shi[8 * AC];           // reductions (index)
    __shared__ double shx[8 * AC];        // second reduction value
    // limiter adjoints: slots 0..7 per-thread cell-average part (b*4+c), 8 P1 density,
    // 9..12 P2 components, 13..16 cell-level part (rbar, pbar, eps)
    __shared__ double shp[17 * AC];
    __shared__ int shpi[2 * AC];
    const Consts& K = g.K;
    const int tid = threadIdx.x;
    const int cl = tid % AC;
    const int bk = tid / AC;
    const int b = bk >> 2, k = bk & 3;
    const int wc = g.NX - 2;
    const long long nreg = (long long)wc * (g.NY - 2);
    const long long cid = (long long)lblock(W, 5) * AC + cl;
    const bool valid = cid < nreg;
    int j = 1, i = 1;
    if (valid) {
        j = 1 + (int)(cid / wc);
        i = 1 + (int)(cid % wc);
    }
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    auto C_ = [&](int bb, int f, int o) -> double& { return shc[((bb * 4 + f) * 16 + o) * AC + cl]; };
    auto U_ = [&](int bb, int c, int o) -> double& { return shu[((bb * 4 + c) * 16 + o) * AC + cl]; };
    auto B_ = [&](int bb, int c, int o) -> double& { return shu[((bb * 4 + c) * 16 + o) * AC + cl]; };

    // ---- forward recompute (as the forward reconstruction kernel) ----
    double ub[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) ub[c] = S[c * N + cell];
    double Lr[4], Rr[4];
    eig2_rows(K, ub, b, k, Lr, Rr);
    // projected stencil data of field k (recomputed before the scalar adjoint
    // instead of being kept live through the limiter)
    auto project = [&](const double* Lrow, double* a) {
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) acc += Lrow[c] * S[c * N + nb];
            a[s] = acc;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int s = 2 * e + 1;
            const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ax += Lrow[c] * S[(4 + c) * N + nb];
                ay += Lrow[c] * S[(8 + c) * N + nb];
            }
            a[9 + e] = ax;
            a[13 + e] = ay;
        }
    };
    {
        double a[17];
        project(Lr, a);
        double C[15], out[16];
        hweno2d(a, K, C);
        if (b == 0) eval_xface(C, out);
        else eval_yface(C, out);
        eval_vol(C, out + 6);
        out[15] = b == 0 ? moment_xi(C) : moment_eta(C);
#pragma unroll
        for (int o = 0; o < 16; ++o) C_(b, k, o) = out[o];
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) acc += Rr[f] * C_(b, f, o);
        U_(b, k, o) = acc;
    }
    __syncthreads();
    // limiter forward: rho_min (argmin in the point order), theta1, then theta2
    const double rbar = ub[0];
    const double pbar = pressure2(K, ub[0], ub[1], ub[2], ub[3]);
    const double e1 = K.eps_pp <= rbar ? K.eps_pp : rbar;
    const int esrc1 = K.eps_pp <= rbar ? 0 : 1;
    const double eps = e1 <= pbar ? e1 : pbar;
    const int esrc = e1 <= pbar ? esrc1 : 2;
    {
        double v = INFINITY;
        int ix = 1 << 30;
        for (int o = k; o < 15; o += 4) {
            const double r = U_(b, 0, o);
            const int id = pt_index(b, o);
            if (r < v || (r == v && id < ix)) { v = r; ix = id; }
        }
        shr[bk * AC + cl] = v;
        shi[bk * AC + cl] = ix;
    }
    __syncthreads();
    double rmin = INFINITY;
    int irmin = 1 << 30;
    for (int q = 0; q < 8; ++q) {
        const double v = shr[q * AC + cl];
        const int id = shi[q * AC + cl];
        if (v < rmin || (v == rmin && id < irmin)) { rmin = v; irmin = id; }
    }
    const bool low1 = rmin < eps;
    const double th1 = low1 ? (rbar - eps) / (rbar - rmin) : 1.0;
    __syncthreads();
    {
        double v = INFINITY;
        int ix = 1 << 30;
        for (int o = k; o < 15; o += 4) {
            const double rt = rbar + th1 * (U_(b, 0, o) - rbar);
            const double pt = pressure2(K, rt, U_(b, 1, o), U_(b, 2, o), U_(b, 3, o));
            const double t = pt < eps ? (pbar - eps) / (pbar - pt) : 1.0;
            const int id = pt_index(b, o);
            if (t < v || (t == v && id < ix)) { v = t; ix = id; }
        }
        shr[bk * AC + cl] = v;
        shi[bk * AC + cl] = ix;
    }
    __syncthreads();
    double tmin = INFINITY;
    int itmin = 1 << 30;
    for (int q = 0; q < 8; ++q) {
        const double v = shr[q * AC + cl];
        const int id = shi[q * AC + cl];
        if (v < tmin || (v == tmin && id < itmin)) { tmin = v; itmin = id; }
    }
    const double th2 = tmin <= 1.0 ? tmin : 1.0;
    const bool low2 = tmin < 1.0;

    // ---- adjoint of the outputs of this thread's component k ----
    const bool inter = valid && interior(g, j, i);
    double Ub[16];
    double th1b = 0.0, th2b = 0.0, ubb0 = 0.0;
    {
        const double* FB = b == 0 ? W.xfb : W.yfb;
        const double* VB = b == 0 ? W.xvb : W.yvb;
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            const double lb = valid ? FB[(o * 4 + k) * N + cell] : 0.0;
            const double x = U_(b, k, o);
            if (k == 0) {
                const double ut = rbar + th1 * (x - rbar);
                Ub[o] = th2 * th1 * lb;
                ubb0 += lb * (1.0 - th2 * th1);
                th2b += lb * (ut - rbar);
                th1b += th2 * lb * (x - rbar);
            } else {
                Ub[o] = th2 * lb;
                ubb0 += lb * (1.0 - th2);
                th2b += lb * (x - ub[k]);
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) Ub[6 + q] = valid ? VB[(q * 4 + k) * N + cell] : 0.0;
        const long long nint = (long long)g.nx * g.ny;
        Ub[15] = (inter && A.Vb)
                     ? A.vs * A.Vb[(b * 4 + k) * nint + (long long)(j - HALO) * g.nx + (i - HALO)]
                     : 0.0;
    }
    shr[bk * AC + cl] = th1b;
    shx[bk * AC + cl] = th2b;
    shp[bk * AC + cl] = ubb0;            // this thread's cell-average adjoint, component k
    __syncthreads();
    if (bk == 0) {
        // cell-level limiter adjoint: thetas -> rbar, pbar, eps and the argmin points
        double T1b = 0.0, T2b = 0.0;
        for (int q = 0; q < 8; ++q) {
            T1b += shr[q * AC + cl];
            T2b += shx[q * AC + cl];
        }
        double rbb = 0.0, pbb = 0.0, epsb = 0.0;
        double P2b[4] = {0.0, 0.0, 0.0, 0.0}, P1b = 0.0;
        int b2 = 0, o2 = 0, b1 = 0, o1 = 0;
        auto unidx = [&](int id, int& bb, int& oo) {
            if (id < 12) { bb = id / 6; oo = id % 6; }
            else { bb = (id - 12) / 9; oo = 6 + (id - 12) % 9; }
        };
        if (low2) {
            unidx(itmin, b2, o2);
            const double rho = U_(b2, 0, o2);
            double Ut[4] = {rbar + th1 * (rho - rbar), U_(b2, 1, o2), U_(b2, 2, o2), U_(b2, 3, o2)};
            const double pt = pressure2(K, Ut[0], Ut[1], Ut[2], Ut[3]);
            const double den = pbar - pt;
            pbb += T2b * (eps - pt) / (den * den);
            epsb += -T2b / den;
            const double ptb = T2b * (pbar - eps) / (den * den);
            double Utb[4] = {0.0, 0.0, 0.0, 0.0};
            adj::pres2_vjp(K, Ut, ptb, Utb);
            rbb += Utb[0] * (1.0 - th1);
            P2b[0] = Utb[0] * th1;
            P2b[1] = Utb[1];
            P2b[2] = Utb[2];
            P2b[3] = Utb[3];
            T1b += Utb[0] * (rho - rbar);
        }
        if (low1) {
            unidx(irmin, b1, o1);
            const double den = rbar - rmin;
            rbb += T1b * (eps - rmin) / (den * den);
            epsb += -T1b / den;
            P1b = T1b * (rbar - eps) / (den * den);
        }
        if (esrc == 1) rbb += epsb;
        double ubar_b[4] = {rbb, 0.0, 0.0, 0.0};
        if (esrc == 2) pbb += epsb;
        if (pbb != 0.0) adj::pres2_vjp(K, ub, pbb, ubar_b);
#pragma unroll
        for (int c = 0; c < 4; ++c) shp[(13 + c) * AC + cl] = ubar_b[c];
        // point adjoints: P2 (4 components) and P1 (density), marked by index
        shp[8 * AC + cl] = P1b;
        shpi[0 * AC + cl] = low1 ? (b1 * 16 + o1) : -1;
        shpi[1 * AC + cl] = low2 ? (b2 * 16 + o2) : -1;
#pragma unroll
        for (int c = 0; c < 4; ++c) shp[(9 + c) * AC + cl] = P2b[c];
    }
    __syncthreads();
    {
        const int p1 = shpi[0 * AC + cl], p2 = shpi[1 * AC + cl];
        if (p1 >= 0 && k == 0 && p1 / 16 == b) Ub[p1 % 16] += shp[8 * AC + cl];
        if (p2 >= 0 && p2 / 16 == b) Ub[p2 % 16] += shp[(9 + k) * AC + cl];
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) B_(b, k, o) = Ub[o];
    __syncthreads();
    // ---- back-transform adjoint: char-bar_f = sum_c R[c][f] Ub_c; R-bar row k ----
    double Rb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < 16; ++o) {
#pragma unroll
        for (int f = 0; f < 4; ++f) Rb[f] += Ub[o] * C_(b, f, o);
    }
    // column k of R (eigenvector of field k), formed from the cell average
    double Rk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double Lt[4], Rt[4];
        eig2_rows(K, ub, b, c, Lt, Rt);
        Rk[c] = Rt[k];
    }
    double cb[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += Rk[c] * B_(b, c, o);
        cb[o] = acc;
    }
    // ---- to the workspace: cotangents of the characteristic outputs, the
    // R-bar row, and (thread b = 0, k = c) the limiter's cell-average part
    // of component c ----
    if (valid) {
#pragma unroll
        for (int o = 0; o < 16; ++o) W.rcb[(bk * 16 + o) * N + cell] = cb[o];
#pragma unroll
        for (int f = 0; f < 4; ++f) W.rrb[(bk * 4 + f) * N + cell] = Rb[f];
        if (b == 0)
            W.rlim[k * N + cell] = shp[(0 * 4 + k) * AC + cl] + shp[(1 * 4 + k) * AC + cl] +
                                   shp[(13 + k) * AC + cl];
    }
}

// Scalar HWENO, eigen-system and projection adjoints of (cell, b, k), from
// the cotangents k_adj_recon_a left in the workspace.
__global__ __launch_bounds__(8 * AC, 2) void k_adj_recon_b(Grid2 g, AdjWs W,
                                                        const double* __restrict__ S) {
    __shared__ double sha[8 * 17 * AC];   // adjoints of the projected inputs (b, k, s)
    __shared__ double shL[8 * 4 * AC];    // rows of L (b, k, c)
    __shared__ double shq[8 * 4 * AC];    // eigen-system part of the cell-average adjoint
    const Consts& K = g.K;
    const int tid = threadIdx.x;
    const int cl = tid % AC;
    const int bk = tid / AC;
    const int b = bk >> 2, k = bk & 3;
    const int wc = g.NX - 2;
    const long long nreg = (long long)wc * (g.NY - 2);
    const long long cid = (long long)lblock(W, 7) * AC + cl;
    const bool valid = cid < nreg;
    int j = 1, i = 1;
    if (valid) {
        j = 1 + (int)(cid / wc);
        i = 1 + (int)(cid % wc);
    }
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    double ub[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) ub[c] = S[c * N + cell];
    double Lr[4], Rr[4];
    eig2_rows(K, ub, b, k, Lr, Rr);
#pragma unroll
    for (int f = 0; f < 4; ++f) shL[(bk * 4 + f) * AC + cl] = Lr[f];
    double cb[16], Rb[4];
#pragma unroll
    for (int o = 0; o < 16; ++o) cb[o] = valid ? W.rcb[(bk * 16 + o) * N + cell] : 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) Rb[f] = valid ? W.rrb[(bk * 4 + f) * N + cell] : 0.0;
    // ---- scalar reconstruction adjoint ----
    double Cb[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) Cb[q] = 0.0;
    if (b == 0) adj::xface_T(cb, Cb);
    else adj::yface_T(cb, Cb);
    adj::vol_T(cb + 6, Cb);
    if (b == 0) moment_xi_T(cb[15], Cb);
    else moment_eta_T(cb[15], Cb);
    double ab[17];
    {
        double a[17];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) acc += Lr[c] * S[c * N + nb];
            a[s] = acc;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int s = 2 * e + 1;
            const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ax += Lr[c] * S[(4 + c) * N + nb];
                ay += Lr[c] * S[(8 + c) * N + nb];
            }
            a[9 + e] = ax;
            a[13 + e] = ay;
        }
        hweno2d_vjp(a, K, Cb, ab);
    }
#pragma unroll
    for (int s = 0; s < 17; ++s) sha[(bk * 17 + s) * AC + cl] = ab[s];
    // L-bar row k: sum_s ab[s] * stencil value (component c)
    double Lb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) Lb[c] += ab[s] * S[c * N + nb];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = 2 * e + 1;
        const long long nb = cell + (long long)(s / 3 - 1) * g.NX + (s % 3 - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            Lb[c] += ab[9 + e] * S[(4 + c) * N + nb] + ab[13 + e] * S[(8 + c) * N + nb];
    }
    double ubp[4] = {0.0, 0.0, 0.0, 0.0};
    if (b == 0) adj::eig2_vjp_0(K, ub, k, Lb, Rb, ubp);
    else adj::eig2_vjp_1(K, ub, k, Lb, Rb, ubp);
    // cell-average adjoint of this thread: eigen part (4 comps) -> LDS for the owner threads
#pragma unroll
    for (int c = 0; c < 4; ++c) shq[((b * 4 + k) * 4 + c) * AC + cl] = ubp[c];
    __syncthreads();
    // ---- projection adjoint, thread (b, c): sum_k L[k][c] ab_k[s] ----
    if (valid) {
        const int c = k;
        double* UC = W.uc + (long long)b * 68 * N;
#pragma unroll
        for (int s = 0; s < 17; ++s) {
            double acc = 0.0;
#pragma unroll
            for (int f = 0; f < 4; ++f) acc += shL[((b * 4 + f) * 4 + c) * AC + cl] * sha[((b * 4 + f) * 17 + s) * AC + cl];
            if (s == 4) {
                // own cell average: eigenvector dependence (both fields' rows of this basis)
#pragma unroll
                for (int f = 0; f < 4; ++f) acc += shq[((b * 4 + f) * 4 + c) * AC + cl];
                // limiter: per-component pass-through of theta and the cell-level part
                if (b == 0) acc += W.rlim[c * N + cell];
            }
            UC[(s * 4 + c) * N + cell] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// State adjoint on the ghosted grid: cell X is slot k of the stencil of
// cell X - off(k) (averages: all 9 slots; moments: the 4 edge slots).
// ---------------------------------------------------------------------------
__global__ void k_adj_ugather(Grid2 g, AdjWs W) {
    const long long t = (long long)lblock(W, 6) * blockDim.x + threadIdx.x;
    if (t >= g.ncell) return;
    const int j = (int)(t / g.NX), i = (int)(t % g.NX);
    const long long N = g.ncell;
    double acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = 0.0;
    for (int b = 0; b < 2; ++b) {
        const double* UC = W.uc + (long long)b * 68 * N;
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            const int ox = s % 3 - 1, oy = s / 3 - 1;
            const int yj = j - oy, yi = i - ox;
            if (yj < 1 || yj > g.NY - 2 || yi < 1 || yi > g.NX - 2) continue;
            const long long Y = (long long)yj * g.NX + yi;
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += UC[(s * 4 + c) * N + Y];
            if (s & 1) {
                const int e = s >> 1;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[4 + c] += UC[((9 + e) * 4 + c) * N + Y];
                    acc[8 + c] += UC[((13 + e) * 4 + c) * N + Y];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) W.ubb[q * N + t] = acc[q];
}

// ---------------------------------------------------------------------------
// Adjoint of the ghost fill: the y sweep is undone first (its sources include
// the x-ghost columns), then the x sweep.  Each source cell gathers the
// ghost cells copied from it, in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ghost_src(int kind, int side, int d, int n) {
    if (kind == 2) return -1;                 // inflow: constant
    if (side == 0) return kind == 0 ? HALO + n - d : (kind == 1 ? HALO : HALO + d - 1);
    return kind == 0 ? HALO + d - 1 : (kind == 1 ? HALO + n - 1 : HALO + n - d);
}

// Component q of the adjoint at cell (r, i) of an interior row once the y
// sweep is undone: its own value plus the ghost rows copied from it.
__device__ __forceinline__ double ghost_y_gather(const Grid2& g, const AdjWs& W, int q, int r,
                                                 int i) {
    const long long N = g.ncell;
    double v = W.ubb[q * N + (long long)r * g.NX + i];
    for (int side = 0; side < 2; ++side) {
        const Side& sd = g.side[2 + side];
        for (int d = 1; d <= HALO; ++d) {
            if (ghost_src(sd.kind, side, d, g.ny) != r) continue;
            const int gj = side == 0 ? HALO - d : HALO + g.ny - 1 + d;
            v += sd.sign[q] * W.ubb[q * N + (long long)gj * g.NX + i];
        }
    }
    return v;
}

// Both sweeps undone for interior cell (j, c0), component q, written to the
// caller's interior array: the y sweep's gather at the cell, then the x
// ghost columns copied from it, each with its own y sweep's gather (the
// corner ghost cells reach the interior through the x-ghost columns).
__global__ void k_adj_ghost_out(Grid2 g, AdjWs W, double* __restrict__ Ubar,
                                const double* __restrict__ add, double add_a,
                                const double* __restrict__ pass) {
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nint * 12) return;
    const int q = (int)(t / nint);
    const long long r = t % nint;
    const int j = HALO + (int)(r / g.nx), c0 = HALO + (int)(r % g.nx);
    // a stage's direct term: fluid cells (averages) or, on a masked grid,
    // solid cells (every component: a stage leaves them at its filled input)
    const bool sol = solid_cell(g, r);
    // every ghost cell copies one of the HALO cells next to a side
    if (c0 >= 2 * HALO && c0 < g.nx && j >= 2 * HALO && j < g.ny) {
        double v = W.ubb[q * g.ncell + (long long)j * g.NX + c0];
        if (sol) {
            if (pass) v += pass[t];
        } else if (add && q < 4) {
            v += add_a * add[t];
        }
        Ubar[t] = v;
        return;
    }
    double v = ghost_y_gather(g, W, q, j, c0);
    for (int side = 0; side < 2; ++side) {
        const Side& sd = g.side[side];
        for (int d = 1; d <= HALO; ++d) {
            if (ghost_src(sd.kind, side, d, g.nx) != c0) continue;
            const int gi = side == 0 ? HALO - d : HALO + g.nx - 1 + d;
            v += sd.sign[q] * ghost_y_gather(g, W, q, j, gi);
        }
    }
    if (sol) {
        if (pass) v += pass[t];
    } else if (add && q < 4) {
        v += add_a * add[t];
    }
    Ubar[t] = v;
}

// Seeds of a masked grid with the solid cells' entries zeroed (solid cells
// carry no residual and no modified moments): the residual seed into rbm (12
// per cell), the modified-moment seed (if any) into vbm (8 per cell).
__global__ void k_mask_seeds(Grid2 g, AdjWs W, const double* __restrict__ Rb,
                             const double* __restrict__ Vb) {
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nint * 20) return;
    const int q = (int)(t / nint);
    const long long r = t % nint;
    const bool sol = g.solid[r] != 0;
    if (q < 12) W.rbm[t] = sol ? 0.0 : Rb[t];
    else if (Vb) W.vbm[t - 12 * nint] = sol ? 0.0 : Vb[t - 12 * nint];
}

// Adjoint of the mirror fill of a masked grid's solid cells (k_solid2):
// each mirror source gathers sign * adjoint of the solid cells copied from it
// (in the list's order), then every listed solid cell's adjoint is zero (its
// value was overwritten).  Ubar in the interior layout.
__global__ void k_adj_solid_gather(Grid2 g, AdjWs W, double* __restrict__ Ubar) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)W.nsrc * 12) return;
    const int u = (int)(t / 12), q = (int)(t % 12);
    const int m = q / 4, c = q % 4;
    const long long nint = (long long)g.nx * g.ny;
    auto interior = [&](int gi) -> long long {
        return (long long)(gi / g.NX - HALO) * g.nx + (gi % g.NX - HALO);
    };
    const long long s = interior(W.ssrcu[u]);
    double acc = Ubar[q * nint + s];
    for (int k = W.sstart[u]; k < W.sstart[u + 1]; ++k) {
        const int e = W.sord[k];
        const int dir = g.sdir[e];
        const bool vel = g.solid_wall == 4 ? (c == 1 || c == 2) : (c == 1 + dir);
        const bool mom = m == 1 + dir;
        const double sg = (vel != mom) ? -1.0 : 1.0;
        acc += sg * Ubar[q * nint + interior(g.sdst[e])];
    }
    Ubar[q * nint + s] = acc;
}

__global__ void k_adj_solid_zero(Grid2 g, double* __restrict__ Ubar) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)g.nsolid * 12) return;
    const int e = (int)(t / 12), q = (int)(t % 12);
    const int gi = g.sdst[e];
    const long long nint = (long long)g.nx * g.ny;
    Ubar[q * nint + (long long)(gi / g.NX - HALO) * g.nx + (gi % g.NX - HALO)] = 0.0;
}

// mu-bar = fixed-order sum of the block partials (added to *out if acc)
__global__ __launch_bounds__(256) void k_mu_sum(const double* part, int n, double* out, int acc) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    // each thread sums its partials q = t, t + 256, ... in order; the loads
    // of eight of them are issued together
    double s = 0.0;
    int q = t;
    for (; q + 7 * 256 < n; q += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[q + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < n; q += 256) s += part[q];
    sh[t] = s;
    __syncthreads();
    // pairwise tree in a fixed order
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *out = acc ? *out + sh[0] : sh[0];
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

__global__ void k_lin3(double* __restrict__ y, const double* __restrict__ u, double a, double b,
                       const double* __restrict__ x, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = a * u[t] + b * y[t] + x[t];
}

inline unsigned nb2(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

long long adj_mu_partials2(const Grid2& g) {
    return (long long)nb2((long long)(g.nx + 1) * g.ny, AF) + nb2((long long)g.nx * (g.ny + 1), AF) +
           nb2((long long)(g.NX - 6) * (g.NY - 6), AG);
}

hipError_t launch_vjp2(const Grid2& g, const AdjIn& A0, AdjWs W, const double* S, double* Ubar,
                       double* mu_out, int mu_acc, hipStream_t st, const double* add,
                       double add_a, const double* pass) {
    const unsigned bx = nb2((long long)(g.nx + 1) * g.ny, AF);
    const unsigned by = nb2((long long)g.nx * (g.ny + 1), AF);
    const unsigned bg = nb2((long long)(g.NX - 6) * (g.NY - 6), AG);
    W.mu_off1 = bx;
    W.mu_off2 = bx + by;
    // the reconstruction adjoint walks its blocks last first, opposite to the
    // weak-moment adjoint before it (1.5 % of a step adjoint on 256^2; the
    // other kernels showed no gain)
    W.rev = 1u << 5;
    AdjIn A = A0;
    if (g.solid) {   // masked grid: the solid cells' seeds zeroed once, for every kernel
        k_mask_seeds<<<nb2((long long)g.nx * g.ny * 20, 256), 256, 0, st>>>(g, W, A0.Rb, A0.Vb);
        A.Rb = W.rbm;
        A.Vb = A0.Vb ? W.vbm : nullptr;
    }
    if (g.K.mu_exp != 0.0) {   // mu(T): the viscosity's dependence on the state too
        k_adj_flux<0, true><<<bx, 3 * AF, 0, st>>>(g, A, W);
        k_adj_flux<1, true><<<by, 3 * AF, 0, st>>>(g, A, W);
        k_adj_grad<true><<<bg, 6 * AG, 0, st>>>(g, A, W);
    } else {
        k_adj_flux<0, false><<<bx, 3 * AF, 0, st>>>(g, A, W);
        k_adj_flux<1, false><<<by, 3 * AF, 0, st>>>(g, A, W);
        k_adj_grad<false><<<bg, 6 * AG, 0, st>>>(g, A, W);
    }
    k_adj_rgather<<<nb2((long long)(g.NX - 4) * (g.NY - 4), 256), 256, 0, st>>>(g, W);
    k_adj_wmom<<<nb2((long long)(g.NX - 2) * (g.NY - 2), WM_CELLS), 6 * WM_CELLS, 0, st>>>(g, W);
    const unsigned brec = nb2((long long)(g.NX - 2) * (g.NY - 2), AC);
    k_adj_recon_a<<<brec, 8 * AC, 0, st>>>(g, A, W, S);
    k_adj_recon_b<<<brec, 8 * AC, 0, st>>>(g, W, S);
    k_adj_ugather<<<nb2(g.ncell, 256), 256, 0, st>>>(g, W);
    k_adj_ghost_out<<<nb2((long long)g.nx * g.ny * 12, 256), 256, 0, st>>>(g, W, Ubar, add, add_a,
                                                                            pass);
    if (g.nsolid > 0) {   // masked grid: the mirror fill, undone
        if (W.nsrc > 0)
            k_adj_solid_gather<<<nb2((long long)W.nsrc * 12, 256), 256, 0, st>>>(g, W, Ubar);
        k_adj_solid_zero<<<nb2((long long)g.nsolid * 12, 256), 256, 0, st>>>(g, Ubar);
    }
    k_mu_sum<<<1, 256, 0, st>>>(W.mupart, (int)(bx + by + bg), mu_out, mu_acc);
    return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, long long n, hipStream_t st) {
    if (n > 0) k_axpy<<<nb2(n, 256), 256, 0, st>>>(y, x, a, n);
    return hipGetLastError();
}

hipError_t launch_lin3(double* y, const double* u, double a, double b, const double* x, long long n,
                       hipStream_t st) {
    if (n > 0) k_lin3<<<nb2(n, 256), 256, 0, st>>>(y, u, a, b, x, n);
    return hipGetLastError();
}

}  // namespace hw
