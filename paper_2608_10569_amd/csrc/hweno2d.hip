// 2D HWENO-GR residual and SSP-RK3 stage update (Sec. 3 of arXiv 2608.10569)
// as a pipeline of HIP kernels over a ghosted structure-of-arrays grid.
//
//   ghost            : halo of width 4 (Remark 4.1)
//   recon            : characteristic HWENO in the x- and y-bases (eq. (3.4)),
//                      positivity limiter on the face values, wbar, hat-v/w,
//                      CFL wave speed                 [cells of halo ring 3]
//   rbar             : interface averages, face moments, weak-derivative
//                      moments (eqs. (3.6)-(3.8))      [halo ring 2]
//   grad             : gradient HWENO (eq. (3.9)) at 12 face + 9 volume points,
//                      volume-flux quadratures         [halo ring 1]
//   rgrad            : rbar + grad in one kernel per tile of cells, the weak
//                      moments of the tile and its ring kept in LDS (a tile
//                      choice)
//   flux_x, flux_y   : PP Lax-Friedrichs fluxes at face Gauss points (eq. (3.3))
//   update           : assembly of eq. (3.2) and the stage combination of the
//                      SSP-RK3 scheme with modified moments (eq. (2.12))
//   fluxup           : flux_x + flux_y + update in one kernel per tile of
//                      cells, the face fluxes kept in LDS (a tile choice)
//
// Every other intermediate lives in HBM, laid out component-major over the
// ghosted grid so that consecutive lanes touch consecutive cells.

#include <hip/hip_ext.h>

#include <mutex>

#include "hweno_kernels.h"

namespace hw {

namespace {

constexpr int HALO = 4;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-level reductions: wave shuffles, then LDS across the block's waves;
// thread 0 issues at most one atomic, and only when it can change the slot.
// (red_max / red_add with a scratch pointer use the caller's LDS, NT / 64
// free slots no thread reads or writes until the block ends.)
template <int NT>
__device__ __forceinline__ void red_max(unsigned long long* slot, double v, double* sh) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) v = fmax(v, sh[w]);
        const unsigned long long k = dkey(v);
        if (v > -INFINITY && k > *(volatile HW_GLOBAL unsigned long long*)slot) atomicMax(slot, k);
    }
}
template <int NT>
__device__ __forceinline__ void red_max(unsigned long long* slot, double v) {
    __shared__ double sh[NT / 64];
    red_max<NT>(slot, v, sh);
}
// Two minima in one pass (one LDS array per value: a second red_min call
// right after the first could overwrite slots thread 0 is still reading).
template <int NT>
__device__ __forceinline__ void red_min2(unsigned long long* sa, double a, unsigned long long* sb,
                                         double b) {
    __shared__ double sh[2][NT / 64];
    a = wave_min(a);
    b = wave_min(b);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = a;
        sh[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            a = fmin(a, sh[0][w]);
            b = fmin(b, sh[1][w]);
        }
        const unsigned long long ka = dkey(a), kb = dkey(b);
        if (a < INFINITY && ka < *(volatile HW_GLOBAL unsigned long long*)sa) atomicMin(sa, ka);
        if (b < INFINITY && kb < *(volatile HW_GLOBAL unsigned long long*)sb) atomicMin(sb, kb);
    }
}
template <int NT>
__device__ __forceinline__ void red_add(unsigned long long* slot, unsigned long long v,
                                        unsigned long long* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) v += sh[w];
        if (v) atomicAdd(slot, v);
    }
}
template <int NT>
__device__ __forceinline__ void red_add(unsigned long long* slot, unsigned long long v) {
    __shared__ unsigned long long sh[NT / 64];
    red_add<NT>(slot, v, sh);
}
template <int NT>
__device__ __forceinline__ void red_add32(unsigned int* slot, unsigned int v) {
    __shared__ unsigned long long sh[NT / 64];
    unsigned long long s = wave_sum((unsigned long long)v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) s += sh[w];
        if (s) atomicAdd(slot, (unsigned int)s);
    }
}

// Slot of the instance that owns this block and the block's index within it
// (uniform per block: binary search of the launch's block prefix table).
struct Loc {
    int p, b;
};
__device__ __forceinline__ Loc locate(const Batch& B) {
    const int nb = (int)gridDim.x;
    const int bid = B.xcd ? xcd_block((int)blockIdx.x, nb, B.rev)
                          : (B.rev ? nb - 1 - (int)blockIdx.x : (int)blockIdx.x);
    int lo = 0, hi = B.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.start[mid] <= bid) lo = mid;
        else hi = mid;
    }
    return Loc{lo, bid - B.start[lo]};
}

// ---------------------------------------------------------------------------
// Ghost cells (Remark 4.1).  The x rule fills the ghost columns of interior
// rows and the y rule every column of the ghost rows; a corner cell takes the
// y rule applied to the value the x rule gives the ghost cell of its source
// row (what an x sweep followed by a y sweep would leave), so one launch
// fills the whole halo.
// ---------------------------------------------------------------------------
// Source of ghost index gi (0..HALO-1 below the interior, HALO+n.. above)
// along a direction with n interior cells: the periodic image, the boundary
// cell (outflow) or the mirror cell (walls).
__device__ __forceinline__ int ghost_src(int kind, int gi, int n) {
    if (gi < HALO) {
        const int d = HALO - gi;   // distance from the boundary
        return kind == 0 ? HALO + n - d : (kind == 1 ? HALO : HALO + d - 1);
    }
    const int d = gi - (HALO + n - 1);
    return kind == 0 ? HALO + d - 1 : (kind == 1 ? HALO + n - 1 : HALO + n - d);
}

// Inflow: the prescribed average of boundary cell k (of n along the side;
// the stage's profile when the fill names a stage), zero moments.
__device__ __forceinline__ void inflow_values(const Side& sd, int k, int n, int stage, double* v) {
    const double* st = (stage >= 0 && sd.prof_stage) ? sd.prof_stage + 4 * (stage * n + k)
                       : sd.prof                      ? sd.prof + 4 * k
                                                      : sd.inflow;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        v[c] = st[c];
        v[4 + c] = 0.0;
        v[8 + c] = 0.0;
    }
}

// Value the x rule of side sd gives ghost column i of interior row j.
__device__ __forceinline__ void x_ghost(const Grid2& g, const Side& sd, const double* S, int j,
                                        int i, int stage, double* v) {
    if (sd.kind == 2) {
        inflow_values(sd, j - HALO, g.ny, stage, v);
        return;
    }
    const long long src = (long long)j * g.NX + ghost_src(sd.kind, i, g.nx);
#pragma unroll
    for (int q = 0; q < 12; ++q) v[q] = sd.sign[q] * S[q * g.ncell + src];
}

// Walls inside the grid (masked domains): solid cell = mirror image of a fluid
// cell across the nearest wall face, with the box walls' parities (Remark 4.1);
// a cell listed with source -1 holds the prescribed state with zero first
// moments instead, as the ghost cells of an inflow side do.
__global__ void k_solid2(const Grid2* gp, int sidx) {
    const Grid2& g = *gp;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nsolid) return;
    double* S = g.S[sidx];
    const long long N = g.ncell;
    const long long d = g.sdst[t], s = g.ssrc[t];
    if (s < 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            S[c * N + d] = g.fixed_state[c];
            S[(4 + c) * N + d] = 0.0;
            S[(8 + c) * N + d] = 0.0;
        }
        return;
    }
    const int dir = g.sdir[t];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bool vel = g.solid_wall == 4 ? (c == 1 || c == 2) : (c == 1 + dir);
            const bool mom = m == 1 + dir;
            const double sg = (vel != mom) ? -1.0 : 1.0;
            S[(m * 4 + c) * N + d] = sg * S[(m * 4 + c) * N + s];
        }
    }
}

// Threads 0 .. 2 HALO ny - 1: ghost columns of the interior rows; then the
// 2 HALO ghost rows, every column.
__global__ void k_ghost2(Batch bt, int sidx, int stage) {
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    double* S = gsrc.S[sidx];
    const int t = lc.b * blockDim.x + threadIdx.x;
    const int nxg = g.ny * 2 * HALO;
    if (t >= nxg + g.NX * 2 * HALO) return;
    double v[12];
    long long dst;
    if (t < nxg) {
        const int j = HALO + t / (2 * HALO);
        const int gi = t % (2 * HALO);
        const int i = gi < HALO ? gi : g.nx + gi;
        x_ghost(g, gsrc.side[gi >= HALO], S, j, i, stage, v);
        dst = (long long)j * g.NX + i;
    } else {
        const int u = t - nxg;
        const int i = u % g.NX;
        const int gj = u / g.NX;
        const int j = gj < HALO ? gj : g.ny + gj;
        const Side& sd = gsrc.side[2 + (gj >= HALO)];
        if (sd.kind == 2) {
            // ghost columns take the profile's end states
            inflow_values(sd, min(max(i - HALO, 0), g.nx - 1), g.nx, stage, v);
        } else {
            const int sj = ghost_src(sd.kind, j, g.ny);
            if (i < HALO || i >= HALO + g.nx) {
                x_ghost(g, gsrc.side[i >= HALO], S, sj, i, stage, v);
            } else {
#pragma unroll
                for (int q = 0; q < 12; ++q) v[q] = S[q * g.ncell + (long long)sj * g.NX + i];
            }
#pragma unroll
            for (int q = 0; q < 12; ++q) v[q] = sd.sign[q] * v[q];
        }
        dst = (long long)j * g.NX + i;
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) S[q * g.ncell + dst] = v[q];
}

// ---------------------------------------------------------------------------
// Characteristic reconstruction + positivity limiter.
// Block: 32 cells x 8 threads; thread (b, k) projects onto characteristic
// field k of basis b (0: x-Jacobian, 1: y-Jacobian), reconstructs it, and
// after an LDS exchange owns conservative component k of basis b.
// DR (the comparison scheme HWENO-DR, eq. (3.5)): the thread also
// differentiates its field's combination in xi and eta at the basis's face
// and volume points (weights kept), the derivatives go back to conservative
// variables through the same exchange, and the viscous gradients
// s = (u_x, u_y, v_x, v_y, e_x, e_y) are formed with the point values that
// enter the flux there (limited face traces; each basis's unlimited volume
// values for its own volume flux).  The kernel then writes the face
// gradients and the volume-flux quadratures itself, in place of the
// weak-moment and gradient kernels.
// ---------------------------------------------------------------------------
template <int RC_CELLS, bool DR = false, bool VarMu = false, bool FULL = false>
__global__ __launch_bounds__(8 * RC_CELLS) void k_recon2(Batch bt, int si) {
    // one block = RC_CELLS consecutive cells of one row; the 3-row stencil
    // tile of all 12 fields is staged in LDS first, then the same memory holds
    // the exchange of the 16 outputs of every (basis, field) thread
    constexpr int TW = RC_CELLS + 2;                 // tile width (columns)
    constexpr int TILE = 12 * 3 * TW;
    constexpr int SH = 8 * 16 * RC_CELLS;
    __shared__ double sh[SH > TILE ? SH : TILE];
    // the per-thread reductions use the exchange's moment slots (o = 15),
    // which are never read back
    double* const red = sh + 15 * RC_CELLS;
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const double* __restrict__ S = gsrc.S[si];
    const Consts& K = g.K;
    const int tid = threadIdx.x;
    const int cl = tid & (RC_CELLS - 1);
    // 32 cells: wavefront w holds field k = w of both bases (lanes 0..31 the
    // x-basis, 32..63 the y-basis), so k is uniform per wavefront
    const int k = RC_CELLS == 32 ? __builtin_amdgcn_readfirstlane(tid >> 6) : (tid / RC_CELLS) & 3;
    const int b = RC_CELLS == 32 ? (tid >> 5) & 1 : (tid / RC_CELLS) >> 2;
    const int bk = b * 4 + k;
    // region: rows 1..NY-2, columns 1..NX-2, in row segments of RC_CELLS
    const int segs = (g.NX - 2 + RC_CELLS - 1) / RC_CELLS;
    const int j = 1 + lc.b / segs;
    const int i0 = 1 + (lc.b % segs) * RC_CELLS;
    const int i = i0 + cl;
    const bool valid = i <= g.NX - 2;
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    // stencil tile: rows j-1..j+1, columns i0-1..i0+RC_CELLS (clamped to the
    // grid); tile row R = 3 c + r holds field c of grid row j-1+r.  All of a
    // thread's loads are issued before the first LDS write.
    if constexpr (RC_CELLS == 32) {
        // wavefront wv loads tile rows 9 wv .. 9 wv + 8, lane = column: the row
        // base is wave-uniform and the lane offset is fixed
        const int lane = tid & 63;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int gi = min(i0 - 1 + lane, g.NX - 1);
        const bool col_ok = lane < TW;
        double v[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int R = 9 * wv + q, c = R / 3, r = R - 3 * c;
            if (col_ok) v[q] = S[c * N + (long long)(j - 1 + r) * g.NX + gi];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (col_ok) sh[(9 * wv + q) * TW + lane] = v[q];
    } else {
        constexpr int NT = 8 * RC_CELLS;
        constexpr int NIT = (TILE + NT - 1) / NT;
        double v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tid + it * NT;
            if (t < TILE) {
                const int R = t / TW, col = t - R * TW;
                const int c = R / 3, r = R - 3 * c;
                const int gi = min(i0 - 1 + col, g.NX - 1);
                v[it] = S[c * N + (long long)(j - 1 + r) * g.NX + gi];
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tid + it * NT;
            if (t < TILE) sh[t] = v[it];
        }
    }
    __syncthreads();
    auto T = [&](int c, int oy, int ox) -> double {
        return sh[(c * 3 + 1 + oy) * TW + cl + 1 + ox];
    };

    double ub[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) ub[c] = T(c, 0, 0);
    double Lr[4], Rr[4];
    eig2_rows(K, ub, b, k, Lr, Rr);

    double a[17];
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += Lr[c] * T(c, s / 3 - 1, s % 3 - 1);
        a[s] = acc;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = 2 * e + 1;   // cells 2, 4, 6, 8
        double ax = 0.0, ay = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ax += Lr[c] * T(4 + c, s / 3 - 1, s % 3 - 1);
            ay += Lr[c] * T(8 + c, s / 3 - 1, s % 3 - 1);
        }
        a[9 + e] = ax;
        a[13 + e] = ay;
    }
    __syncthreads();   // the tile is dead; sh holds the output exchange from here
    double C[15];
    hweno2d(a, K, C);
    double out[16];
    if (b == 0) eval_xface(C, out);
    else eval_yface(C, out);
    eval_vol(C, out + 6);
    out[15] = b == 0 ? moment_xi(C) : moment_eta(C);
#pragma unroll
    for (int o = 0; o < 16; ++o) sh[(bk * 16 + o) * RC_CELLS + cl] = out[o];
    __syncthreads();
    // back to conservative component k of basis b
    double U[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) acc += Rr[f] * sh[((b * 4 + f) * 16 + o) * RC_CELLS + cl];
        U[o] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 16; ++o) sh[(bk * 16 + o) * RC_CELLS + cl] = U[o];
    __syncthreads();

    // positivity limiter: theta over 6 face + 9 volume points of both bases
    auto comp = [&](int bb, int c, int o) { return sh[((bb * 4 + c) * 16 + o) * RC_CELLS + cl]; };
    double rmin = INFINITY;
    for (int o = k; o < 15; o += 4) rmin = fmin(rmin, comp(b, 0, o));
    red[bk * 16 * RC_CELLS + cl] = rmin;
    __syncthreads();
    rmin = red[cl];
#pragma unroll
    for (int q = 1; q < 8; ++q) rmin = fmin(rmin, red[q * 16 * RC_CELLS + cl]);
    const double rbar = ub[0];
    const double pbar = pressure2(K, ub[0], ub[1], ub[2], ub[3]);
    const double eps = fmin(fmin(K.eps_pp, rbar), pbar);
    const double th1 = rmin < eps ? (rbar - eps) / (rbar - rmin) : 1.0;
    double tmin = 1.0;
    for (int o = k; o < 15; o += 4) {
        const double rt = rbar + th1 * (comp(b, 0, o) - rbar);
        const double pt = pressure2(K, rt, comp(b, 1, o), comp(b, 2, o), comp(b, 3, o));
        if (pt < eps) tmin = fmin(tmin, (pbar - eps) / (pbar - pt));
    }
    __syncthreads();   // every thread has read the rho minima
    red[bk * 16 * RC_CELLS + cl] = tmin;
    __syncthreads();
    double th2 = red[cl];
#pragma unroll
    for (int q = 1; q < 8; ++q) th2 = fmin(th2, red[q * 16 * RC_CELLS + cl]);

    const bool inter = valid && j >= HALO && j < HALO + g.ny && i >= HALO && i < HALO + g.nx;
    if (valid) {
        double* F = (b == 0 ? g.xf : g.yf) + k * N + cell;
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            const double ut = k == 0 ? rbar + th1 * (U[o] - rbar) : U[o];
            F[o * 4 * N] = ub[k] + th2 * (ut - ub[k]);
        }
    }
    // HWENO-GR: wbar of (u, v, e) from this basis' unlimited volume values,
    // and the compact volume data of the gradient kernel's volume flux: the
    // Gauss sum of this basis' convective flux and the velocities (and
    // viscosities) at the points.  Thread k takes the volume points q = k,
    // k+4, k+8; the partial sums meet in LDS.  (HWENO-DR forms its volume
    // fluxes below and needs none of this.)
    if constexpr (!DR) {
        double su = 0.0, sv = 0.0, se = 0.0;
        double fs[4] = {0.0, 0.0, 0.0, 0.0};
        double* VC = g.vc + (long long)b * VC_B * N + cell;
        for (int q = k; q < 9; q += 4) {
            const int o = 6 + q;
            const double w = (q / 3 == 1 ? GW1 : GW0) * (q % 3 == 1 ? GW1 : GW0);
            const double r = comp(b, 0, o), m = comp(b, 1, o), n = comp(b, 2, o);
            const double E = comp(b, 3, o);
            const double ir = rcp(r);
            const double u = m * ir, v = n * ir;
            const double e = E * ir - 0.5 * (u * u + v * v);
            su += w * u;
            sv += w * v;
            se += w * e;
            double fc[4], mu;
            conv2_dir<VarMu>(K, r, m, n, E, u, v, b == 1, fc, mu);
#pragma unroll
            for (int c = 0; c < 4; ++c) fs[c] += w * fc[c];
            if (valid) {
                VC[(4 + q) * N] = u;
                VC[(13 + q) * N] = v;
                if constexpr (VarMu) VC[(22 + q) * N] = mu;
            }
        }
        __syncthreads();   // theta2 and the volume slots of sh are read
        // the partial sums go to the thread's own volume slots 6..12
        sh[(bk * 16 + 10) * RC_CELLS + cl] = su;
        sh[(bk * 16 + 11) * RC_CELLS + cl] = sv;
        sh[(bk * 16 + 12) * RC_CELLS + cl] = se;
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[(bk * 16 + 6 + c) * RC_CELLS + cl] = fs[c];
        __syncthreads();
        if (valid && k == 0) {
            double tu = 0.0, tv = 0.0, te = 0.0;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                tu += sh[((b * 4 + f) * 16 + 10) * RC_CELLS + cl];
                tv += sh[((b * 4 + f) * 16 + 11) * RC_CELLS + cl];
                te += sh[((b * 4 + f) * 16 + 12) * RC_CELLS + cl];
            }
            g.wb[(b * 3 + 0) * N + cell] = tu;
            g.wb[(b * 3 + 1) * N + cell] = tv;
            g.wb[(b * 3 + 2) * N + cell] = te;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int f = 0; f < 4; ++f) acc += sh[((b * 4 + f) * 16 + 6 + c) * RC_CELLS + cl];
                VC[c * N] = acc;
            }
        }
        if constexpr (FULL) {   // the reverse mode reads the full volume values
            if (valid) {
                double* V = (b == 0 ? g.xv : g.yv) + k * N + cell;
#pragma unroll
                for (int q = 0; q < 9; ++q) V[q * 4 * N] = U[6 + q];
            }
        }
    }
    if (inter) g.vk[(b * 4 + k) * N + cell] = U[15];
    // CFL wave speed over the limited face traces of interior cells; thread k
    // takes the face points o = k, k+4
    double amax = -INFINITY;
    if (inter) {
        for (int o = k; o < 6; o += 4) {
            double Ul[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double x = comp(b, c, o);
                const double ut = c == 0 ? rbar + th1 * (x - rbar) : x;
                Ul[c] = ub[c] + th2 * (ut - ub[c]);
            }
            const double ir = rcp(Ul[0]);
            const double u = Ul[1] * ir, v = Ul[2] * ir;
            const double p = K.gm1 * (Ul[3] - 0.5 * (Ul[1] * u + Ul[2] * v));
            const double sp = fmax(fabs(u), fabs(v)) + sqrt(K.gamma * p * ir);
            amax = fmax(amax, sp);
        }
    }
    if constexpr (DR) {
        // thread k converts the points o = k, k+4, k+8, k+12 of basis b:
        // gather the four components of the point values (limited on the
        // faces) and of their two derivatives from the exchange
        double P[4][4], Dx[4][4], Dy[4][4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int o = k + 4 * s4;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (o < 15) {
                    const double x = comp(b, c, o);
                    const double ut = c == 0 ? rbar + th1 * (x - rbar) : x;
                    P[s4][c] = o < 6 ? ub[c] + th2 * (ut - ub[c]) : x;
                } else {
                    P[s4][c] = 1.0;
                }
            }
        }
        // the derivatives of this field's combination in xi, then eta, at the
        // 15 points; back to conservative component k through the exchange
        // (as the values), then a second exchange hands each thread the four
        // components at its points
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
            double dv[15];
            {
                double D[15];
                if (dir == 0) dxi_coeffs(C, D);
                else deta_coeffs(C, D);
                if (b == 0) eval_xface(D, dv);
                else eval_yface(D, dv);
                eval_vol(D, dv + 6);
            }
            __syncthreads();
#pragma unroll
            for (int o = 0; o < 15; ++o) sh[(bk * 16 + o) * RC_CELLS + cl] = dv[o];
            __syncthreads();
            const double h = dir == 0 ? K.idx : K.idy;
#pragma unroll
            for (int o = 0; o < 15; ++o) {
                double acc = 0.0;
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    acc += Rr[f] * sh[((b * 4 + f) * 16 + o) * RC_CELLS + cl];
                dv[o] = acc * h;
            }
            __syncthreads();
#pragma unroll
            for (int o = 0; o < 15; ++o) sh[(bk * 16 + o) * RC_CELLS + cl] = dv[o];
            __syncthreads();
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int o = min(k + 4 * s4, 14);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double x = sh[((b * 4 + c) * 16 + o) * RC_CELLS + cl];
                    if (dir == 0) Dx[s4][c] = x;
                    else Dy[s4][c] = x;
                }
            }
        }
        // faces of interior cells read the gradients of the cells on both
        // sides; volume fluxes are needed in interior cells only
        const bool ring = valid && j >= HALO - 1 && j <= HALO + g.ny && i >= HALO - 1 &&
                          i <= HALO + g.nx;
        double vfs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int o = k + 4 * s4;
            if (o >= 15 || !ring) continue;
            const double ir = rcp(P[s4][0]);
            const double u = P[s4][1] * ir, v = P[s4][2] * ir, eo = P[s4][3] * ir;
            double sg[6];
#pragma unroll
            for (int dir = 0; dir < 2; ++dir) {
                const double* D = dir == 0 ? Dx[s4] : Dy[s4];
                const double ul = (D[1] - u * D[0]) * ir;
                const double vl = (D[2] - v * D[0]) * ir;
                const double el = (D[3] - eo * D[0]) * ir - u * ul - v * vl;
                sg[0 + dir] = ul;
                sg[2 + dir] = vl;
                sg[4 + dir] = el;
            }
            if (o < 6) {
                const int p = b * 6 + o;
                double dc[3];
                if (b == 0) stress_combos<0>(sg, dc);
                else stress_combos<1>(sg, dc);
#pragma unroll
                for (int z = 0; z < 3; ++z) g.gf[(p * 3 + z) * N + cell] = dc[z];
            } else {
                const int q = o - 6;
                const double w = (q / 3 == 1 ? GW1 : GW0) * (q % 3 == 1 ? GW1 : GW0);
                double f[4];
                flux2_dir<VarMu>(K, P[s4], sg, b == 1, f);
#pragma unroll
                for (int c = 0; c < 4; ++c) vfs[c] += w * f[c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[(bk * 16 + c) * RC_CELLS + cl] = vfs[c];
        __syncthreads();
        if (inter && k == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int f = 0; f < 4; ++f) acc += sh[((b * 4 + f) * 16 + c) * RC_CELLS + cl];
                g.vf[(b * 4 + c) * N + cell] = acc;
            }
        }
    }
    // the block reductions use moment slots of the exchange: past the
    // barriers above, no thread reads or writes them any more
    red_max<8 * RC_CELLS>(&g.red->alpha_key, amax, red);
    red_add<8 * RC_CELLS>(&g.red->pp_cells,
                          (inter && bk == 0 && (th1 < 1.0 || th2 < 1.0)) ? 1ull : 0ull,
                          reinterpret_cast<unsigned long long*>(red + 8));
}

// ---------------------------------------------------------------------------
// Weak-derivative moments (eqs. (3.6)-(3.8)) on cells of halo ring 2.
// ---------------------------------------------------------------------------
// Primitives (u, v, e) of face point p of `cell` (one reciprocal of rho).
__device__ __forceinline__ void prim3(const double* F, long long N, long long cell, int p,
                                      double* w) {
#pragma clang fp contract(off)
    const double r = F[(p * 4 + 0) * N + cell];
    const double ir = rcp(r);
    const double u = F[(p * 4 + 1) * N + cell] * ir;
    const double v = F[(p * 4 + 2) * N + cell] * ir;
    w[0] = u;
    w[1] = v;
    w[2] = F[(p * 4 + 3) * N + cell] * ir - 0.5 * (u * u + v * v);
}

// Gauss average W0 = sum_G w_G h_G and first moment W1 = sum_G w_G x_G h_G of
// the interface average h = (w- + w+)/2 of (u, v, e) over the face between
// cell `lo` (its upper points 3..5) and cell `hi` (its lower points 0..2).
// Mirror-symmetric forms: exchanging the outer points gives the same W0 and
// the negated W1.  Contraction is fixed in the source, so every kernel that
// forms the weak moments gets the same bits.
__device__ __forceinline__ void face_wavg(const double* F, long long N, long long lo, long long hi,
                                          double* W0, double* W1) {
#pragma clang fp contract(off)
    double h[3][3];   // [G][w]
#pragma unroll
    for (int G = 0; G < 3; ++G) {
        double a[3], c[3];
        prim3(F, N, lo, 3 + G, a);
        prim3(F, N, hi, G, c);
#pragma unroll
        for (int w = 0; w < 3; ++w) h[G][w] = 0.5 * (a[w] + c[w]);
    }
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        W0[w] = fma(GW0, h[0][w] + h[2][w], GW1 * h[1][w]);
        W1[w] = (GW0 * GS) * (h[2][w] - h[0][w]);
    }
}

// The three weak moments (eqs. (3.6)-(3.8)) of d w / d x_l of a cell from the
// face data of its lower and upper l-faces and its w-bar; ih = 1/dx_l.
// m[0] = moment 0, m[1] = xi moment, m[2] = eta moment.
__device__ __forceinline__ void cell_wmom(double W0lo, double W0hi, double W1lo, double W1hi,
                                          double wbl, double ih, int l, double* m) {
#pragma clang fp contract(off)
    const double d0 = (W0hi - W0lo) * ih;                    // moment 0
    const double dm = (0.5 * (W0hi + W0lo) - wbl) * ih;      // moment along l
    const double d1 = (W1hi - W1lo) * ih;                    // transverse moment
    m[0] = d0;
    m[1] = l ? d1 : dm;
    m[2] = l ? dm : d1;
}

// Block = RB_TX x RB_TY cells of the region (rows and columns 2 .. N-3).
// First every face of the tile gets its interface averages w^ = (w- + w+)/2
// at the three Gauss points, once (a face is shared by two cells): the x-faces
// of each tile row and the y-faces of each tile column, into LDS.  Then each
// cell forms the 18 weak moments of d w / d x_l from its four faces and w-bar.
constexpr int RB_TX = 32, RB_TY = 8;

__global__ __launch_bounds__(RB_TX * RB_TY) void k_rbar2(Batch bt) {
    constexpr int NXF = RB_TY * (RB_TX + 1), NYF = (RB_TY + 1) * RB_TX;
    // per face and variable w: the Gauss average W0 = sum_G w_G h_G and the
    // first moment W1 = sum_G w_G x_G h_G of the interface average h
    __shared__ double hx[6][RB_TY][RB_TX + 1];   // [3 m + w][row][face i - 1/2]
    __shared__ double hy[6][RB_TY + 1][RB_TX];   // [3 m + w][face j - 1/2][column]
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    // tiles start at multiples of RB_TX columns of the ghosted grid (whole
    // cache lines per row segment); columns 0 and 1 are outside the region
    const int tiles_x = (g.NX - 2 + RB_TX - 1) / RB_TX;
    const int i0 = (lc.b % tiles_x) * RB_TX;
    const int j0 = 2 + (lc.b / tiles_x) * RB_TY;
    const long long N = g.ncell;
    for (int t = threadIdx.x; t < NXF + NYF; t += RB_TX * RB_TY) {
        const bool xd = t < NXF;
        const int q = xd ? t : t - NXF;
        // face between cells (ilo, jlo) and (i, j): i - 1/2 (x) or j - 1/2 (y)
        int i, j, ilo, jlo;
        if (xd) {
            i = i0 + q % (RB_TX + 1);
            j = j0 + q / (RB_TX + 1);
            ilo = i - 1;
            jlo = j;
            if (j > g.NY - 3 || i > g.NX - 2 || i < 2) continue;
        } else {
            i = i0 + q % RB_TX;
            j = j0 + q / RB_TX;
            ilo = i;
            jlo = j - 1;
            if (i > g.NX - 3 || j > g.NY - 2 || i < 2) continue;
        }
        const double* F = xd ? g.xf : g.yf;
        const long long lo = (long long)jlo * g.NX + ilo, hi = (long long)j * g.NX + i;
        double W0[3], W1[3];
        face_wavg(F, N, lo, hi, W0, W1);
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            if (xd) {
                hx[w][j - j0][i - i0] = W0[w];
                hx[3 + w][j - j0][i - i0] = W1[w];
            } else {
                hy[w][j - j0][i - i0] = W0[w];
                hy[3 + w][j - j0][i - i0] = W1[w];
            }
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % RB_TX, ty = threadIdx.x / RB_TX;
    const int i = i0 + tx, j = j0 + ty;
    if (i < 2 || i > g.NX - 3 || j > g.NY - 3) return;
    const long long cell = (long long)j * g.NX + i;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        const double ih = l ? g.K.idy : g.K.idx;
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            const double W0lo = l ? hy[w][ty][tx] : hx[w][ty][tx];
            const double W0hi = l ? hy[w][ty + 1][tx] : hx[w][ty][tx + 1];
            const double W1lo = l ? hy[3 + w][ty][tx] : hx[3 + w][ty][tx];
            const double W1hi = l ? hy[3 + w][ty + 1][tx] : hx[3 + w][ty][tx + 1];
            double m[3];
            cell_wmom(W0lo, W0hi, W1lo, W1hi, g.wb[(l * 3 + w) * N + cell], ih, l, m);
            double* R = g.rb + ((l * 3 + w) * 3) * N + cell;
            R[0] = m[0];
            R[N] = m[1];       // xi moment
            R[2 * N] = m[2];   // eta moment
        }
    }
}

// ---------------------------------------------------------------------------
// Gradient reconstruction (eq. (3.9)) on halo ring 1; block 32 or 64 cells
// x 6 (thread s = 2*w + l reconstructs d w / d x_l).  Interior cells also
// form the volume-flux quadratures of eq. (3.2).
// ---------------------------------------------------------------------------
// Gradient reconstruction of component s = 2 w + l of one cell from its 17
// stencil data a (eq. (3.9)), the face gradients it stores, and on interior
// cells the volume-flux quadrature of eq. (3.2).  The block has NC cells x 6
// components (cell cl, component s); shv holds 6 x 9 x NC doubles of LDS.
// Every thread of the block calls it (it holds barriers).
template <int NC, bool VarMu, bool FULL>
__device__ __forceinline__ void grad_body(const Grid2& g, double* shv, const double* a, int cl,
                                          int s, bool valid, int j, int i) {
    const Consts& K = g.K;
    const long long N = g.ncell;
    const long long cell = (long long)j * g.NX + i;
    double C[15];
    hweno2d(a, grad_consts(K), C);
    double fo[12], vo[9];
    eval_xface(C, fo);
    eval_yface(C, fo + 6);
    eval_vol(C, vo);
    if constexpr (FULL) {
        if (valid) {
#pragma unroll
            for (int p = 0; p < 12; ++p) g.gf[(p * 6 + s) * N + cell] = fo[p];
        }
    } else {
        // the face fluxes need three combinations of the six gradients per
        // face point (stress_combos): the x-face points, then the y-face
        // points, meet in LDS, and thread s forms outputs s, s + 6, s + 12 of
        // the 18 of each half
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int q = 0; q < 6; ++q) shv[(s * 6 + q) * NC + cl] = fo[half * 6 + q];
            __syncthreads();
            if (valid) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int o = s + 6 * r, q = o / 3, z = o % 3;
                    double sq[6], dc[3];
#pragma unroll
                    for (int c = 0; c < 6; ++c) sq[c] = shv[(c * 6 + q) * NC + cl];
                    if (half == 0) stress_combos<0>(sq, dc);
                    else stress_combos<1>(sq, dc);
                    g.gf[((half * 6 + q) * 3 + z) * N + cell] = dc[z];
                }
            }
            __syncthreads();
        }
    }
    const bool inter = valid && j >= HALO && j < HALO + g.ny && i >= HALO && i < HALO + g.nx;
    // volume-flux quadratures of interior cells: the reconstruction kernel
    // left the Gauss sum of the convective flux and the velocities (and
    // viscosities) at the points; the viscous part is summed here over the
    // cell's 6 threads, 2 directions x 9 points, 3 points each (thread s:
    // direction s / 3, points 3 (s % 3) .. 3 (s % 3) + 2), and the partial
    // sums meet in LDS.  The point data are loaded before the barrier.
    const bool dy = s >= 3;
    const int q0 = 3 * (s % 3);
    const double* VC = g.vc + (long long)(dy ? VC_B : 0) * N + cell;
    double pu[3], pv[3], pm[3];
    if (inter) {
#pragma unroll
        for (int qq = 0; qq < 3; ++qq) {
            pu[qq] = VC[(4 + q0 + qq) * N];
            pv[qq] = VC[(13 + q0 + qq) * N];
            pm[qq] = VarMu ? VC[(22 + q0 + qq) * N] : K.mu_ref;
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) shv[(s * 9 + q) * NC + cl] = vo[q];
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    if (inter) {
#pragma unroll
        for (int qq = 0; qq < 3; ++qq) {
            const int q = q0 + qq;
            const double wq = (q / 3 == 1 ? GW1 : GW0) * (q % 3 == 1 ? GW1 : GW0);
            double sq[6], f[3];
#pragma unroll
            for (int z = 0; z < 6; ++z) sq[z] = shv[(z * 9 + q) * NC + cl];
            visc2_dir(K, pu[qq], pv[qq], pm[qq], sq, dy, f);
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += wq * f[c];
        }
    }
    __syncthreads();   // every read of the gradient values is done
#pragma unroll
    for (int c = 0; c < 3; ++c) shv[(s * 3 + c) * NC + cl] = acc[c];
    __syncthreads();
    if (inter && s < 2) {
        const double* VS = g.vc + (long long)s * VC_B * N + cell;
        g.vf[(s * 4) * N + cell] = VS[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double t0 = shv[((3 * s + 0) * 3 + c) * NC + cl];
            const double t1 = shv[((3 * s + 1) * 3 + c) * NC + cl];
            const double t2 = shv[((3 * s + 2) * 3 + c) * NC + cl];
            g.vf[(s * 4 + 1 + c) * N + cell] = VS[(1 + c) * N] + (t0 + t1 + t2);
        }
    }
}


template <int GR_CELLS, bool VarMu, bool FULL>
__global__ __launch_bounds__(6 * GR_CELLS) void k_grad2(Batch bt) {
    __shared__ double shv[6 * 9 * GR_CELLS];
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const Consts& K = g.K;
    const int tid = threadIdx.x;
    const int cl = tid % GR_CELLS;
    const int s = tid / GR_CELLS;
    const int w = s >> 1, l = s & 1;
    const int wc = g.NX - 6;
    const long long nreg = (long long)wc * (g.NY - 6);
    const long long cid = (long long)lc.b * GR_CELLS + cl;
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
    for (int q = 0; q < 9; ++q)
        a[q] = R0[cell + (long long)(q / 3 - 1) * g.NX + (q % 3 - 1)];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = 2 * e + 1;
        const long long nb = cell + (long long)(q / 3 - 1) * g.NX + (q % 3 - 1);
        a[9 + e] = R1[nb];
        a[13 + e] = R2[nb];
    }
    grad_body<GR_CELLS, VarMu, FULL>(g, shv, a, cl, s, valid, j, i);
}

// ---------------------------------------------------------------------------
// Weak moments and gradient reconstruction in one kernel (HWENO-GR, face
// gradients in the three combinations).  A block takes RG_TX x RG_TY cells of
// the gradient region and forms the weak moments of those cells and of the
// ring around them in LDS (the ring is formed again by the neighbouring
// tiles): first the interface data of every face of the ring's cells, then
// their 18 weak moments, then the gradient reconstruction reads its 3x3
// stencils from LDS.  Same arithmetic as k_rbar2 followed by k_grad2, without
// the weak moments' round trip through HBM.
// ---------------------------------------------------------------------------
constexpr int RG_TX = 16, RG_TY = 4, RG_CELLS = RG_TX * RG_TY;
constexpr int RG_RX = RG_TX + 2, RG_RY = RG_TY + 2;                   // tile + ring
constexpr int RG_NXF = RG_RY * (RG_RX + 1), RG_NYF = (RG_RY + 1) * RG_RX;   // faces
constexpr int RG_LDS_A = 6 * (RG_NXF + RG_NYF) + 18 * RG_RY * RG_RX;
constexpr int RG_LDS = RG_LDS_A > 54 * RG_CELLS ? RG_LDS_A : 54 * RG_CELLS;

template <bool VarMu>
__global__ __launch_bounds__(6 * RG_CELLS) void k_rgrad2(Batch bt) {
    // phase 1: hx[6][RY][RX + 1] and hy[6][RY + 1][RX] (W0 for w = 0..2, then
    // W1), rbs[18][RY][RX] (index (l * 3 + w) * 3 + moment); phase 2: the
    // gradient body's exchange over the same memory
    __shared__ double lds[RG_LDS];
    double* const hx = lds;
    double* const hy = hx + 6 * RG_NXF;
    double* const rbs = hy + 6 * RG_NYF;
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const long long N = g.ncell;
    const int tiles_x = (g.NX - 6 + RG_TX - 1) / RG_TX;
    const int i0 = 3 + (lc.b % tiles_x) * RG_TX;   // first cell of the tile
    const int j0 = 3 + (lc.b / tiles_x) * RG_TY;
    constexpr int NT = 6 * RG_CELLS;
    // interface data of the faces of the ring's cells (j0 - 1 + r, i0 - 1 + c);
    // cells of weak moments lie in rows and columns 2 .. N - 3
    for (int t = threadIdx.x; t < RG_NXF + RG_NYF; t += NT) {
        const bool xd = t < RG_NXF;
        const int q = xd ? t : t - RG_NXF;
        int r, c, i, j, ilo, jlo;
        if (xd) {   // face i - 1/2 of row j
            r = q / (RG_RX + 1);
            c = q % (RG_RX + 1);
            j = j0 - 1 + r;
            i = i0 - 1 + c;
            ilo = i - 1;
            jlo = j;
            if (j > g.NY - 3 || i > g.NX - 2) continue;
        } else {    // face j - 1/2 of column i
            r = q / RG_RX;
            c = q % RG_RX;
            j = j0 - 1 + r;
            i = i0 - 1 + c;
            ilo = i;
            jlo = j - 1;
            if (i > g.NX - 3 || j > g.NY - 2) continue;
        }
        double W0[3], W1[3];
        face_wavg(xd ? g.xf : g.yf, N, (long long)jlo * g.NX + ilo, (long long)j * g.NX + i, W0,
                  W1);
        double* H = xd ? hx : hy;
        const int plane = xd ? RG_NXF : RG_NYF;
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            H[w * plane + q] = W0[w];
            H[(3 + w) * plane + q] = W1[w];
        }
    }
    __syncthreads();
    // weak moments of the ring's cells: one task per (cell, l, w)
    for (int t = threadIdx.x; t < 6 * RG_RY * RG_RX; t += NT) {
        const int lw = t / (RG_RY * RG_RX), rc = t % (RG_RY * RG_RX);
        const int l = lw / 3, w = lw % 3;
        const int r = rc / RG_RX, c = rc % RG_RX;
        const int j = j0 - 1 + r, i = i0 - 1 + c;
        if (j > g.NY - 3 || i > g.NX - 3) continue;
        double W0lo, W0hi, W1lo, W1hi;
        if (l == 0) {
            const int f = r * (RG_RX + 1) + c;
            W0lo = hx[w * RG_NXF + f];
            W0hi = hx[w * RG_NXF + f + 1];
            W1lo = hx[(3 + w) * RG_NXF + f];
            W1hi = hx[(3 + w) * RG_NXF + f + 1];
        } else {
            const int f = r * RG_RX + c;
            W0lo = hy[w * RG_NYF + f];
            W0hi = hy[w * RG_NYF + f + RG_RX];
            W1lo = hy[(3 + w) * RG_NYF + f];
            W1hi = hy[(3 + w) * RG_NYF + f + RG_RX];
        }
        double m[3];
        cell_wmom(W0lo, W0hi, W1lo, W1hi, g.wb[(l * 3 + w) * N + (long long)j * g.NX + i],
                  l ? g.K.idy : g.K.idx, l, m);
#pragma unroll
        for (int k = 0; k < 3; ++k) rbs[(lw * 3 + k) * (RG_RY * RG_RX) + rc] = m[k];
    }
    __syncthreads();
    // gradient reconstruction: cell cl of the tile, component s = 2 w + l
    const int cl = threadIdx.x % RG_CELLS;
    const int s = threadIdx.x / RG_CELLS;
    const int w = s >> 1, l = s & 1;
    const int ty = cl / RG_TX, tx = cl % RG_TX;
    const int j = j0 + ty, i = i0 + tx;
    const bool valid = j <= g.NY - 4 && i <= g.NX - 4;
    const double* R = rbs + (long long)((l * 3 + w) * 3) * (RG_RY * RG_RX);
    double a[17];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int o = (ty + 1 + q / 3 - 1) * RG_RX + (tx + 1 + q % 3 - 1);
        a[q] = valid ? R[o] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = 2 * e + 1;
        const int o = (ty + 1 + q / 3 - 1) * RG_RX + (tx + 1 + q % 3 - 1);
        a[9 + e] = valid ? R[RG_RY * RG_RX + o] : 0.0;
        a[13 + e] = valid ? R[2 * RG_RY * RG_RX + o] : 0.0;
    }
    __syncthreads();   // the weak moments are in registers; the exchange reuses the LDS
    grad_body<RG_CELLS, VarMu, false>(g, lds, a, cl, s, valid, valid ? j : 3, valid ? i : 3);
}

// The two Gauss moments of a face flux that the assembly of eq. (3.2) takes
// from a face, per component: A = sum_G w_G F_G and B = sum_G w_G x_G F_G
// (x_G = -s, 0, s in face units).  One definition for every kernel.
// Both are written so that exchanging the outer points (a mirror image of
// the face) gives the same A and the negated B bit for bit.
__device__ __forceinline__ void face_moments(double F0, double F1, double F2, double& A,
                                             double& B) {
#pragma clang fp contract(off)
    A = fma(GW0, F0 + F2, GW1 * F1);
    B = (GW0 * GS) * (F2 - F0);
}

// The three gradient combinations of face point p (0..5 x-face, 6..11
// y-face; direction d of that face) of a cell: read as stored, or formed from
// the six gradients of the full layout.
template <int d, bool FULL>
__device__ __forceinline__ void face_grad(const Grid2& g, int p, long long cell, double* dc) {
    const long long N = g.ncell;
    if constexpr (FULL) {
        double sq[6];
#pragma unroll
        for (int z = 0; z < 6; ++z) sq[z] = g.gf[(p * 6 + z) * N + cell];
        stress_combos<d>(sq, dc);
    } else {
#pragma unroll
        for (int z = 0; z < 3; ++z) dc[z] = g.gf[(p * 3 + z) * N + cell];
    }
}

// ---------------------------------------------------------------------------
// Face fluxes (eq. (3.3)): x-faces (j, i+1/2) for interior rows, i from the
// last ghost column; y-faces (j+1/2, i) likewise.  The LF coefficient is the
// max over the face's three Gauss points and both sides.
// ---------------------------------------------------------------------------
template <int d, int FX_FACES, bool VarMu, bool FULL>   // block = 3 Gauss points x FX_FACES faces
__global__ __launch_bounds__(3 * FX_FACES) void k_flux2(Batch bt) {
    __shared__ double shb[3 * FX_FACES];
    __shared__ double shf[4][3 * FX_FACES];
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const Consts& K = g.K;
    const int nfi = d == 0 ? g.nx + 1 : g.nx;
    const int nfj = d == 0 ? g.ny : g.ny + 1;
    const int G = threadIdx.x / FX_FACES;
    const int fl = threadIdx.x % FX_FACES;
    const long long t = (long long)lc.b * FX_FACES + fl;
    const bool valid = t < (long long)nfi * nfj;
    const long long N = g.ncell;
    long long cm = 0, cp = 0;
    double fs[4] = {0.0, 0.0, 0.0, 0.0}, du[4] = {0.0, 0.0, 0.0, 0.0};
    double beta = -INFINITY;
    if (valid) {
        const int fj = (int)(t / nfi), fi = (int)(t % nfi);
        const int j = d == 0 ? HALO + fj : HALO - 1 + fj;
        const int i = d == 0 ? HALO - 1 + fi : HALO + fi;
        cm = (long long)j * g.NX + i;
        cp = d == 0 ? cm + 1 : cm + g.NX;
        const double* F = d == 0 ? g.xf : g.yf;
        const int pg = d == 0 ? 0 : 6;
        double Um[4], Up[4], sm[3], sp[3], fm[4], fp[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Um[c] = F[((3 + G) * 4 + c) * N + cm];
            Up[c] = F[(G * 4 + c) * N + cp];
        }
        face_grad<d, FULL>(g, pg + 3 + G, cm, sm);
        face_grad<d, FULL>(g, pg + G, cp, sp);
        flux2c<d, VarMu>(K, Um, sm, fm);
        flux2c<d, VarMu>(K, Up, sp, fp);
        beta = fmax(speed2c<d, VarMu>(K, Um, sm), speed2c<d, VarMu>(K, Up, sp));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            fs[c] = fm[c] + fp[c];
            du[c] = Up[c] - Um[c];
        }
    }
    shb[threadIdx.x] = beta;
    __syncthreads();
    // LF coefficient: max over the face's three Gauss points and both sides
    beta = fmax(fmax(shb[fl], shb[FX_FACES + fl]), shb[2 * FX_FACES + fl]);
    // the face's Gauss moments: the three points meet in LDS
#pragma unroll
    for (int c = 0; c < 4; ++c) shf[c][threadIdx.x] = 0.5 * fma(-beta, du[c], fs[c]);
    __syncthreads();
    if (valid && G == 0) {
        double* out = d == 0 ? g.fx : g.fy;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double A, B;
            face_moments(shf[c][fl], shf[c][FX_FACES + fl], shf[c][2 * FX_FACES + fl], A, B);
            out[c * N + cm] = A;
            out[(4 + c) * N + cm] = B;
        }
    }
    red_max<3 * FX_FACES>(&g.red->beta_key, valid && G == 0 ? beta : -INFINITY);
}

// ---------------------------------------------------------------------------
// Assembly (eq. (3.2)) and stage update (eq. (2.12) in 2D form) of interior
// cell (ii, jj), t = jj * nx + ii.  ff(c, L, R, Bo, T) gives the Gauss
// moments (A, B) of component c of the fluxes of the cell's left, right,
// bottom and top faces (L[0] = A, L[1] = B, ...).  stage 0: R and Vhat out
// (interior layout); stage 1..3: SSP-RK3 stage.  rmin, pmin and bad receive
// the cell's share of the admissibility reductions (stages 1..3; solid cells
// give none).
// ---------------------------------------------------------------------------
template <class FF>
__device__ __forceinline__ void update_cell(const Grid2& g, const Grid2& gsrc, long long t, int jj,
                                            int ii, int stage, int i0, int iin, int iout,
                                            double* __restrict__ Rout,
                                            double* __restrict__ Vout,
                                            const double* __restrict__ src, const FF& ff,
                                            double& rmin, double& pmin, unsigned int& bad) {
    // explicit fused multiply-adds, no automatic contraction: the same
    // rounding whichever kernel inlines this
#pragma clang fp contract(off)
    const double* __restrict__ S0 = gsrc.S[i0];
    const double* __restrict__ Sin = gsrc.S[iin];
    double* __restrict__ Sout = gsrc.S[iout];
    const long long nint = (long long)g.nx * g.ny;
    const long long N = g.ncell;
    const long long cell = (long long)(jj + HALO) * g.NX + ii + HALO;
    if (gsrc.solid && gsrc.solid[t]) {
        // solid cell of a masked domain: no residual, keeps the stage input,
        // not checked
        if (stage == 0) {
#pragma unroll
            for (int q = 0; q < 12; ++q) Rout[q * nint + t] = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) Vout[q * nint + t] = 0.0;
        } else {
#pragma unroll
            for (int q = 0; q < 12; ++q) Sout[q * N + cell] = Sin[q * N + cell];
        }
        return;
    }
    const double idx = g.K.idx, idy = g.K.idy;
    double Fm[3][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double L[2], R[2], Bo[2], T[2];
        ff(c, L, R, Bo, T);
        const double dfx = R[0] - L[0], sfx = L[0] + R[0], dfxe = R[1] - L[1];
        const double dgy = T[0] - Bo[0], sgy = Bo[0] + T[0], dgyx = T[1] - Bo[1];
        Fm[0][c] = fma(-dfx, idx, -dgy * idy);
        Fm[1][c] = fma(g.vf[c * N + cell], idx, fma(-sfx, 0.5 * idx, -dgyx * idy));
        Fm[2][c] = fma(g.vf[(4 + c) * N + cell], idy, fma(-dfxe, idx, -sgy * (0.5 * idy)));
    }
    if (src) {   // prescribed source moments (layout of R; single grid)
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) Fm[m][c] += src[(m * 4 + c) * nint + t];
    }
    if (stage == 0) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) Rout[(m * 4 + c) * nint + t] = Fm[m][c];
#pragma unroll
        for (int q = 0; q < 8; ++q) Vout[q * nint + t] = g.vk[q * N + cell];
        return;
    }
    const double dt = g.red->dt;
    double nw[12];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double in0 = Sin[c * N + cell];
        const double in1 = g.vk[c * N + cell];
        const double in2 = g.vk[(4 + c) * N + cell];
        if (stage == 1) {
            nw[c] = fma(dt, Fm[0][c], in0);
            nw[4 + c] = fma(dt, Fm[1][c], in1);
            nw[8 + c] = fma(dt, Fm[2][c], in2);
            g.vn[c * N + cell] = in1;
            g.vn[(4 + c) * N + cell] = in2;
        } else {
            const double a = stage == 2 ? 0.75 : 1.0 / 3.0;
            const double bb = stage == 2 ? 0.25 : 2.0 / 3.0;
            nw[c] = fma(a, S0[c * N + cell], bb * fma(dt, Fm[0][c], in0));
            nw[4 + c] = fma(a, g.vn[c * N + cell], bb * fma(dt, Fm[1][c], in1));
            nw[8 + c] = fma(a, g.vn[(4 + c) * N + cell], bb * fma(dt, Fm[2][c], in2));
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) Sout[q * N + cell] = nw[q];
    const double p = pressure2(g.K, nw[0], nw[1], nw[2], nw[3]);
    rmin = nw[0];
    pmin = p;
    bool ok = nw[0] > 0.0 && p > 0.0;
#pragma unroll
    for (int q = 0; q < 12; ++q) ok = ok && isfinite(nw[q]);
    bad = ok ? 0u : 1u;
}

// Split path: the face fluxes come from k_flux2 through HBM.
__global__ __launch_bounds__(256) void k_update2(Batch bt, int stage, int i0, int iin, int iout,
                                                 double* __restrict__ Rout,
                                                 double* __restrict__ Vout,
                                                 const double* __restrict__ src) {
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)lc.b * blockDim.x + threadIdx.x;
    double rmin = INFINITY, pmin = INFINITY;
    unsigned int bad = 0;
    if (t < nint) {
        const int jj = (int)(t / g.nx), ii = (int)(t % g.nx);
        const long long N = g.ncell;
        const long long cell = (long long)(jj + HALO) * g.NX + ii + HALO;
        auto ff = [&](int c, double* L, double* R, double* Bo, double* T) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                R[m] = g.fx[(4 * m + c) * N + cell];
                L[m] = g.fx[(4 * m + c) * N + cell - 1];
                T[m] = g.fy[(4 * m + c) * N + cell];
                Bo[m] = g.fy[(4 * m + c) * N + cell - g.NX];
            }
        };
        update_cell(g, gsrc, t, jj, ii, stage, i0, iin, iout, Rout, Vout, src, ff, rmin, pmin,
                    bad);
    }
    if (stage > 0) {
        red_min2<256>(&g.red->min_rho_key, rmin, &g.red->min_p_key, pmin);
        red_add32<256>(&g.red->bad[stage], bad);
    }
}

// ---------------------------------------------------------------------------
// Face fluxes fused with the assembly and the stage update.  A block of 256
// threads owns a tile of FU_TX x FU_TY cells (columns aligned to multiples of
// FU_TX in the ghosted grid; ghost cells in it stay idle).  First the two
// Gauss moments of the flux of every face of the tile go to LDS: thread
// (tx, ty) forms the x-face left of its cell and the y-face below it, and one
// more pass forms the x-faces right of the tile and the y-faces above it.
// Then each thread assembles and updates its cell.  A face on a tile edge is
// formed by both tiles that share it.  The arithmetic per face and per cell
// is that of k_flux2 and k_update2, so the two paths give the same bits.
// ---------------------------------------------------------------------------
constexpr int FU_TX = 32, FU_TY = 8;

// Gauss moments (A into o[c * stride], B into o[(4 + c) * stride]) of the
// flux of the face between cells cm and cp (direction d); returns the LF
// coefficient (max over the three points and both sides).
template <int d, bool VarMu, bool FULL>
__device__ __forceinline__ double face_flux3(const Grid2& g, long long cm, long long cp,
                                             double* o, int stride) {
    const Consts& K = g.K;
    const long long N = g.ncell;
    const double* F = d == 0 ? g.xf : g.yf;
    const int pg = d == 0 ? 0 : 6;
    double fs[3][4], du[3][4], bg[3];
#pragma unroll
    for (int G = 0; G < 3; ++G) {
        double Um[4], Up[4], sm[3], sp[3], fm[4], fp[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Um[c] = F[((3 + G) * 4 + c) * N + cm];
            Up[c] = F[(G * 4 + c) * N + cp];
        }
        face_grad<d, FULL>(g, pg + 3 + G, cm, sm);
        face_grad<d, FULL>(g, pg + G, cp, sp);
        flux2c<d, VarMu>(K, Um, sm, fm);
        flux2c<d, VarMu>(K, Up, sp, fp);
        bg[G] = fmax(speed2c<d, VarMu>(K, Um, sm), speed2c<d, VarMu>(K, Up, sp));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            fs[G][c] = fm[c] + fp[c];
            du[G][c] = Up[c] - Um[c];
        }
    }
    const double beta = fmax(fmax(bg[0], bg[1]), bg[2]);
    double Fg[3][4];   // the flux at each Gauss point
#pragma unroll
    for (int G = 0; G < 3; ++G)
#pragma unroll
        for (int c = 0; c < 4; ++c) Fg[G][c] = 0.5 * fma(-beta, du[G][c], fs[G][c]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        face_moments(Fg[0][c], Fg[1][c], Fg[2][c], o[c * stride], o[(4 + c) * stride]);
    return beta;
}

template <bool VarMu, bool FULL>
__global__ __launch_bounds__(FU_TX * FU_TY) void k_fluxup2(Batch bt, int stage, int i0, int iin,
                                                           int iout, double* __restrict__ Rout,
                                                           double* __restrict__ Vout,
                                                           const double* __restrict__ src) {
    constexpr int RX = FU_TX + 1;                              // x-face columns per row
    constexpr int SX = FU_TY * RX, SY = (FU_TY + 1) * FU_TX;   // plane sizes
    __shared__ double lx[8 * SX];    // [moment*4 + c][row][face column 0..FU_TX]
    __shared__ double ly[8 * SY];    // [moment*4 + c][face row 0..FU_TY][column]
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    // tiles start at multiples of FU_TX columns of the ghosted grid, so that
    // their row segments are whole cache lines; the first tile's leading
    // columns are ghost cells and stay idle
    const int tiles_x = (g.nx + HALO + FU_TX - 1) / FU_TX;
    const int ii0 = (lc.b % tiles_x) * FU_TX - HALO, jj0 = (lc.b / tiles_x) * FU_TY;
    const int tx = threadIdx.x % FU_TX, ty = threadIdx.x / FU_TX;
    double bmax = -INFINITY;
    // x-face left of interior cell (ii0 + fc, jj0 + row); fc = FU_TX and
    // ii = nx (the domain's right boundary face) included
    auto xface = [&](int fc, int row) {
        const int ii = ii0 + fc, jj = jj0 + row;
        if (ii < 0 || ii > g.nx || jj >= g.ny) return;
        const long long cp = (long long)(jj + HALO) * g.NX + ii + HALO;
        bmax = fmax(bmax, face_flux3<0, VarMu, FULL>(g, cp - 1, cp, lx + row * RX + fc, SX));
    };
    // y-face below interior cell (ii0 + col, jj0 + fr); fr = FU_TY and jj = ny
    // included
    auto yface = [&](int fr, int col) {
        const int ii = ii0 + col, jj = jj0 + fr;
        if (ii < 0 || ii >= g.nx || jj > g.ny) return;
        const long long cp = (long long)(jj + HALO) * g.NX + ii + HALO;
        bmax = fmax(bmax, face_flux3<1, VarMu, FULL>(g, cp - g.NX, cp, ly + fr * FU_TX + col, SY));
    };
    xface(tx, ty);
    yface(ty, tx);
    if (threadIdx.x < FU_TX) yface(FU_TY, threadIdx.x);                  // wavefront 0
    else if (threadIdx.x >= 64 && threadIdx.x < 64 + FU_TY) xface(FU_TX, threadIdx.x - 64);
    __syncthreads();
    const int ii = ii0 + tx, jj = jj0 + ty;
    double rmin = INFINITY, pmin = INFINITY;
    unsigned int bad = 0;
    if (ii >= 0 && ii < g.nx && jj < g.ny) {
        auto ff = [&](int c, double* L, double* R, double* Bo, double* T) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int q = 4 * m + c;
                L[m] = lx[q * SX + ty * RX + tx];
                R[m] = lx[q * SX + ty * RX + tx + 1];
                Bo[m] = ly[q * SY + ty * FU_TX + tx];
                T[m] = ly[q * SY + (ty + 1) * FU_TX + tx];
            }
        };
        update_cell(g, gsrc, (long long)jj * g.nx + ii, jj, ii, stage, i0, iin, iout, Rout, Vout,
                    src, ff, rmin, pmin, bad);
    }
    red_max<FU_TX * FU_TY>(&g.red->beta_key, bmax);
    if (stage > 0) {
        red_min2<FU_TX * FU_TY>(&g.red->min_rho_key, rmin, &g.red->min_p_key, pmin);
        red_add32<FU_TX * FU_TY>(&g.red->bad[stage], bad);
    }
}

__global__ void k_copy_in2(Grid2 g, const double* __restrict__ U, double* __restrict__ S) {
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nint * 12) return;
    const int q = (int)(t / nint);
    const long long r = t % nint;
    const int jj = (int)(r / g.nx), ii = (int)(r % g.nx);
    S[q * g.ncell + (long long)(jj + HALO) * g.NX + ii + HALO] = U[t];
}

__global__ void k_copy_out2(Grid2 g, const double* __restrict__ S, double* __restrict__ U) {
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nint * 12) return;
    const int q = (int)(t / nint);
    const long long r = t % nint;
    const int jj = (int)(r / g.nx), ii = (int)(r % g.nx);
    U[t] = S[q * g.ncell + (long long)(jj + HALO) * g.NX + ii + HALO];
}

// Input admissibility (finite values, positive density and pressure).
__global__ __launch_bounds__(256) void k_check2(Batch bt, int si) {
    const Loc lc = locate(bt);
    const Grid2& gsrc = bt.g[lc.p];   // arrays indexed at run time are read from here
    if (!gsrc.st->active) return;
    const Grid2 g = gsrc;
    const double* __restrict__ S = gsrc.S[si];
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)lc.b * blockDim.x + threadIdx.x;
    unsigned int bad = 0;
    if (t < nint && !(gsrc.solid && gsrc.solid[t])) {
        const int jj = (int)(t / g.nx), ii = (int)(t % g.nx);
        const long long cell = (long long)(jj + HALO) * g.NX + ii + HALO;
        double q[12];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            q[k] = S[k * g.ncell + cell];
            ok = ok && isfinite(q[k]);
        }
        ok = ok && q[0] > 0.0 && pressure2(g.K, q[0], q[1], q[2], q[3]) > 0.0;
        bad = ok ? 0u : 1u;
    }
    red_add32<256>(&g.red->bad[0], bad);
}

__global__ void k_reset(Reduce* r) {
    if (threadIdx.x == 0) {
        r->alpha_key = dkey(-INFINITY);
        r->beta_key = dkey(-INFINITY);
        r->pp_cells = 0;
        r->min_rho_key = dkey(INFINITY);
        r->min_p_key = dkey(INFINITY);
        r->bad[0] = r->bad[1] = r->bad[2] = r->bad[3] = 0;
    }
}

__global__ void k_dt(Reduce* r, double cfl_h, double visc_dt, double t_left) {
    if (threadIdx.x == 0) {
        r->alpha1_key = r->alpha_key;
        const double a = dkey_inv(r->alpha_key);
        double dt = cfl_h / a;
        dt = fmin(dt, visc_dt);
        dt = fmin(dt, t_left);
        r->dt = dt;
    }
}

__global__ void k_set_dt(Reduce* r, double dt) {
    if (threadIdx.x == 0) {
        r->alpha1_key = r->alpha_key;
        r->dt = dt;
    }
}

// Per-instance kernels of a batch: thread p serves the instance in slot p.
__global__ void k_reset2(const Grid2* __restrict__ gs, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    Reduce* r = gs[p].red;
    r->alpha_key = dkey(-INFINITY);
    r->beta_key = dkey(-INFINITY);
    r->pp_cells = 0;
    r->min_rho_key = dkey(INFINITY);
    r->min_p_key = dkey(INFINITY);
    r->bad[0] = r->bad[1] = r->bad[2] = r->bad[3] = 0;
}

// Trial step of the time-step rule from the stage-1 wave speed, halved once
// per rejected attempt of the current step.
__global__ void k_dt2(const Grid2* __restrict__ gs, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const InstState* st = gs[p].st;
    if (!st->active) return;
    Reduce* r = gs[p].red;
    r->alpha1_key = r->alpha_key;
    double dt = fmin(st->cfl_h / dkey_inv(r->alpha_key), st->visc_dt);
    if (st->t_final > 0.0) dt = fmin(dt, st->t_final - st->t);
    r->dt = ldexp(dt, -st->halvings);
}

__device__ __forceinline__ bool accepted(const Grid2& g) {
    const Reduce* r = g.red;
    const double dt = r->dt;
    return r->bad[1] == 0 && r->bad[2] == 0 && r->bad[3] == 0 && dt > 0.0 && isfinite(dt);
}

// Accepted instances: interior of S[1] (the stage-3 output) -> S[0].
__global__ __launch_bounds__(256) void k_commit_copy(Batch bt) {
    const Loc lc = locate(bt);
    const Grid2 g = bt.g[lc.p];
    if (!g.st->active || !accepted(g)) return;
    const long long nint = (long long)g.nx * g.ny;
    const long long t = (long long)lc.b * blockDim.x + threadIdx.x;
    if (t >= nint) return;
    const int jj = (int)(t / g.nx), ii = (int)(t % g.nx);
    const long long cell = (long long)(jj + HALO) * g.NX + ii + HALO;
#pragma unroll
    for (int q = 0; q < 12; ++q) g.S[0][q * g.ncell + cell] = g.S[1][q * g.ncell + cell];
}

__global__ void k_commit_state(const Grid2* __restrict__ gs, int n, int code_inadmissible,
                               int code_nonfinite) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const Grid2& g = gs[p];
    InstState* st = g.st;
    if (!st->active) return;
    const Reduce* r = g.red;
    st->alpha = dkey_inv(r->alpha1_key);
    st->beta_max = dkey_inv(r->beta_key);
    st->min_rho = dkey_inv(r->min_rho_key);
    st->min_p = dkey_inv(r->min_p_key);
    if (!(r->dt > 0.0) || !isfinite(r->dt)) {
        // no usable step size (a non-finite wave speed): stop the instance
        // as the single-grid driver stops, instead of halving a NaN
        st->status = code_nonfinite;
        st->active = 0;
        return;
    }
    if (accepted(g)) {
        st->t += r->dt;
        st->dt_last = r->dt;
        st->steps += 1;
        st->halvings = 0;
        st->pp_cells += r->pp_cells;
        const bool at_end = st->t_final > 0.0 && !(st->t < st->t_final);
        if (st->steps >= st->target || at_end) st->active = 0;
    } else {
        st->restarts += 1;
        if (st->halvings >= st->max_halvings) {
            st->status = code_inadmissible;
            st->active = 0;
        } else {
            st->halvings += 1;
        }
    }
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_reset(Reduce* red, hipStream_t st) {
    k_reset<<<1, 64, 0, st>>>(red);
    return hipGetLastError();
}

hipError_t launch_dt(Reduce* red, double cfl_h, double visc_dt, double t_left, hipStream_t st) {
    k_dt<<<1, 64, 0, st>>>(red, cfl_h, visc_dt, t_left);
    return hipGetLastError();
}

hipError_t launch_set_dt(Reduce* red, double dt, hipStream_t st) {
    k_set_dt<<<1, 64, 0, st>>>(red, dt);
    return hipGetLastError();
}

void batch_blocks(const Grid2* hg, int n, const Tiles& t, int* out) {
    for (int k = 0; k < KB_COUNT; ++k) {
        int* st = out + k * (n + 1);
        st[0] = 0;
        for (int p = 0; p < n; ++p) {
            const Grid2& g = hg[p];
            long long work = 0;
            int per = 256;
            switch (k) {
                case KB_GHOST: work = (long long)(g.ny + g.NX) * 2 * HALO; break;
                case KB_RECON:   // row segments of t.recon cells
                    work = (long long)(g.NY - 2) * ((g.NX - 2 + t.recon - 1) / t.recon);
                    per = 1;
                    break;
                case KB_RBAR:    // tiles of RB_TX x RB_TY cells, aligned to ghosted columns
                    work = (long long)((g.NX - 2 + RB_TX - 1) / RB_TX) *
                           ((g.NY - 4 + RB_TY - 1) / RB_TY);
                    per = 1;
                    break;
                case KB_GRAD:    // the split kernel (32 cells per block with the fused one chosen)
                    work = (long long)(g.NX - 6) * (g.NY - 6);
                    per = t.grad ? t.grad : 32;
                    break;
                case KB_RGRAD:   // tiles of RG_TX x RG_TY cells of the gradient region
                    work = (long long)((g.NX - 6 + RG_TX - 1) / RG_TX) *
                           ((g.NY - 6 + RG_TY - 1) / RG_TY);
                    per = 1;
                    break;
                case KB_FLUX0:   // none when the update kernel forms the fluxes
                    work = t.flux ? (long long)(g.nx + 1) * g.ny : 0;
                    per = t.flux ? t.flux : 1;
                    break;
                case KB_FLUX1:
                    work = t.flux ? (long long)g.nx * (g.ny + 1) : 0;
                    per = t.flux ? t.flux : 1;
                    break;
                case KB_FLUXUP:  // tiles of FU_TX x FU_TY cells, aligned to ghosted columns
                    work = (long long)((g.nx + HALO + FU_TX - 1) / FU_TX) *
                           ((g.ny + FU_TY - 1) / FU_TY);
                    per = 1;
                    break;
                default: work = (long long)g.nx * g.ny; break;
            }
            st[p + 1] = st[p] + (int)nblk(work, per);
        }
    }
}

hipError_t launch_check2(const BatchL& b, int si, hipStream_t st) {
    k_check2<<<b.blocks(KB_CELLS), 256, 0, st>>>(b.arg(KB_CELLS), si);
    return hipGetLastError();
}

hipError_t launch_solid2(const Grid2* g, int n, int si, hipStream_t st) {
    if (n > 0) k_solid2<<<nblk(n, 256), 256, 0, st>>>(g, si);
    return hipGetLastError();
}

hipError_t launch_copy_in2(const Grid2& g, const double* U, double* S, hipStream_t st) {
    const long long n = (long long)g.nx * g.ny * 12;
    k_copy_in2<<<nblk(n, 256), 256, 0, st>>>(g, U, S);
    return hipGetLastError();
}

hipError_t launch_copy_out2(const Grid2& g, const double* S, double* U, hipStream_t st) {
    const long long n = (long long)g.nx * g.ny * 12;
    k_copy_out2<<<nblk(n, 256), 256, 0, st>>>(g, S, U);
    return hipGetLastError();
}

// Launch of a kernel that is a timing class of its own: when the class is
// timed, the kernel records the two events itself at the start and end of
// its execution; otherwise a plain launch (the one graphs record).
template <typename F, typename... Args>
void tlaunch(Timer* tm, int k, F kern, unsigned grid, unsigned block, hipStream_t st,
             Args... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) tm->ext(k, &e0, &e1);
    if (e0) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, e0, e1, 0, args...);
    else hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, args...);
}

hipError_t launch_ghost2(const BatchL& b, int si, hipStream_t st, Timer* tm, int stage) {
    tlaunch(tm, KC_GHOST, k_ghost2, b.blocks(KB_GHOST), 256, st, b.arg(KB_GHOST), si, stage);
    return hipGetLastError();
}

// The split face-flux kernels of both directions for the launch's tiles.
template <bool FULL>
void launch_flux2(const BatchL& b, hipStream_t st) {
    const Batch a0 = b.arg(KB_FLUX0), a1 = b.arg(KB_FLUX1);
    const unsigned n0 = b.blocks(KB_FLUX0), n1 = b.blocks(KB_FLUX1);
    if (b.tiles.flux == 128) {
        if (b.var_mu) {
            k_flux2<0, 128, true, FULL><<<n0, 384, 0, st>>>(a0);
            k_flux2<1, 128, true, FULL><<<n1, 384, 0, st>>>(a1);
        } else {
            k_flux2<0, 128, false, FULL><<<n0, 384, 0, st>>>(a0);
            k_flux2<1, 128, false, FULL><<<n1, 384, 0, st>>>(a1);
        }
    } else {
        if (b.var_mu) {
            k_flux2<0, 64, true, FULL><<<n0, 192, 0, st>>>(a0);
            k_flux2<1, 64, true, FULL><<<n1, 192, 0, st>>>(a1);
        } else {
            k_flux2<0, 64, false, FULL><<<n0, 192, 0, st>>>(a0);
            k_flux2<1, 64, false, FULL><<<n1, 192, 0, st>>>(a1);
        }
    }
}

hipError_t launch_residual2(const BatchL& b, int si, hipStream_t st, Timer* tm) {
    const unsigned nr = b.blocks(KB_RECON), ng = b.blocks(KB_GRAD);
    const Batch ar = b.arg(KB_RECON);
    if (b.dr) {   // HWENO-DR: gradients and volume fluxes come with the reconstruction
        if (b.tiles.recon == 16) {
            if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<16, true, true>, nr, 128, st, ar, si);
            else tlaunch(tm, KC_RECON, k_recon2<16, true, false>, nr, 128, st, ar, si);
        } else {
            if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<32, true, true>, nr, 256, st, ar, si);
            else tlaunch(tm, KC_RECON, k_recon2<32, true, false>, nr, 256, st, ar, si);
        }
    } else if (b.full_grad) {   // the reverse mode also stores the full volume values
        if (b.tiles.recon == 16) {
            if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<16, false, true, true>, nr, 128, st, ar, si);
            else tlaunch(tm, KC_RECON, k_recon2<16, false, false, true>, nr, 128, st, ar, si);
        } else {
            if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<32, false, true, true>, nr, 256, st, ar, si);
            else tlaunch(tm, KC_RECON, k_recon2<32, false, false, true>, nr, 256, st, ar, si);
        }
    } else if (b.tiles.recon == 16) {
        if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<16, false, true>, nr, 128, st, ar, si);
        else tlaunch(tm, KC_RECON, k_recon2<16>, nr, 128, st, ar, si);
    } else {
        if (b.var_mu) tlaunch(tm, KC_RECON, k_recon2<32, false, true>, nr, 256, st, ar, si);
        else tlaunch(tm, KC_RECON, k_recon2<32>, nr, 256, st, ar, si);
    }
    if (!b.dr && !b.full_grad && b.tiles.grad == 0) {
        // HWENO-GR, weak moments formed inside the gradient kernel
        const Batch ag = b.arg(KB_RGRAD);
        if (b.var_mu) tlaunch(tm, KC_GRAD, k_rgrad2<true>, b.blocks(KB_RGRAD), 6 * RG_CELLS, st, ag);
        else tlaunch(tm, KC_GRAD, k_rgrad2<false>, b.blocks(KB_RGRAD), 6 * RG_CELLS, st, ag);
    } else if (!b.dr) {   // HWENO-GR: weak-derivative moments, then their reconstruction
        tlaunch(tm, KC_RBAR, k_rbar2, b.blocks(KB_RBAR), RB_TX * RB_TY, st, b.arg(KB_RBAR));
        const Batch ag = b.arg(KB_GRAD);
        if (b.full_grad) {   // the reverse mode reads all six gradients (and the adjoint
                             // the weak moments)
            if (b.tiles.grad == 64) {
                if (b.var_mu) tlaunch(tm, KC_GRAD, k_grad2<64, true, true>, ng, 384, st, ag);
                else tlaunch(tm, KC_GRAD, k_grad2<64, false, true>, ng, 384, st, ag);
            } else {
                if (b.var_mu) tlaunch(tm, KC_GRAD, k_grad2<32, true, true>, ng, 192, st, ag);
                else tlaunch(tm, KC_GRAD, k_grad2<32, false, true>, ng, 192, st, ag);
            }
        } else if (b.tiles.grad == 64) {
            if (b.var_mu) tlaunch(tm, KC_GRAD, k_grad2<64, true, false>, ng, 384, st, ag);
            else tlaunch(tm, KC_GRAD, k_grad2<64, false, false>, ng, 384, st, ag);
        } else {
            if (b.var_mu) tlaunch(tm, KC_GRAD, k_grad2<32, true, false>, ng, 192, st, ag);
            else tlaunch(tm, KC_GRAD, k_grad2<32, false, false>, ng, 192, st, ag);
        }
    }
    if (b.tiles.flux == 0) return hipGetLastError();   // fluxes formed by the update kernel
    tbeg(tm, KC_FLUX, st);
    if (b.full_grad) launch_flux2<true>(b, st);
    else launch_flux2<false>(b, st);
    tend(tm, st);
    return hipGetLastError();
}

hipError_t launch_update2(const BatchL& b, int stage, int i0, int iin, int iout, double* R,
                          double* Vhat, hipStream_t st, Timer* tm, const double* src) {
    if (b.tiles.flux == 0) {
        const unsigned nb = b.blocks(KB_FLUXUP);
        const Batch a = b.arg(KB_FLUXUP);
        constexpr unsigned NT = FU_TX * FU_TY;
        if (b.full_grad) {
            if (b.var_mu)
                tlaunch(tm, KC_FLUXUP, k_fluxup2<true, true>, nb, NT, st, a, stage, i0, iin, iout,
                        R, Vhat, src);
            else
                tlaunch(tm, KC_FLUXUP, k_fluxup2<false, true>, nb, NT, st, a, stage, i0, iin,
                        iout, R, Vhat, src);
        } else if (b.var_mu) {
            tlaunch(tm, KC_FLUXUP, k_fluxup2<true, false>, nb, NT, st, a, stage, i0, iin, iout, R,
                    Vhat, src);
        } else {
            tlaunch(tm, KC_FLUXUP, k_fluxup2<false, false>, nb, NT, st, a, stage, i0, iin, iout,
                    R, Vhat, src);
        }
    } else {
        tlaunch(tm, KC_UPDATE, k_update2, b.blocks(KB_CELLS), 256, st, b.arg(KB_CELLS), stage, i0,
                iin, iout, R, Vhat, src);
    }
    return hipGetLastError();
}

hipError_t launch_reset2(const BatchL& b, hipStream_t st) {
    k_reset2<<<nblk(b.n, 64), 64, 0, st>>>(b.dg, b.n);
    return hipGetLastError();
}

hipError_t launch_dt2(const BatchL& b, hipStream_t st) {
    k_dt2<<<nblk(b.n, 64), 64, 0, st>>>(b.dg, b.n);
    return hipGetLastError();
}

hipError_t launch_commit2(const BatchL& b, hipStream_t st) {
    k_commit_copy<<<b.blocks(KB_CELLS), 256, 0, st>>>(b.arg(KB_CELLS));
    k_commit_state<<<nblk(b.n, 64), 64, 0, st>>>(b.dg, b.n, 4, 5);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free residual: a file-scope array in device
// memory, one per device the library runs on.  Host code never passes the
// array's name to a kernel (on the host it only names a stand-in); it takes
// the device address from hipGetSymbolAddress, once per device with that
// device current, and hands that pointer on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    *out = nullptr;
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[d]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[d] = p;
    }
    *out = addr[d];
    return hipSuccess;
}

}  // namespace hw
