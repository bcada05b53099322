"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

Only initial data lives here (the workloads' definitions): pointwise
primitive fields are converted to conserved variables and projected onto the
cell average and scaled first-order moments with a 6-point Gauss-Legendre
rule per direction.  None of the scheme's arithmetic is in this module.

Every generator returns numpy float64 arrays in the D1 layout of
include/hweno.h: 1D U[m, c, i] (2, 3, nx); 2D U[m, c, j, i] (3, 4, ny, nx).
Random draws use numpy's PCG64 with the base seed 2608.
"""

import math

import numpy as np

SEED = 2608


def _gauss6():
    x, w = np.polynomial.legendre.leggauss(6)
    return 0.5 * x, 0.5 * w


def _cons1(rho, u, p, gamma):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _cons2(rho, u, v, p, gamma):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def project1d(prim, nx, x0, x1, gamma):
    """prim(x) -> (rho, u, p); returns U (2, 3, nx)."""
    gx, gw = _gauss6()
    dx = (x1 - x0) / nx
    xc = x0 + (np.arange(nx) + 0.5) * dx
    X = xc[None, :] + gx[:, None] * dx                       # (6, nx)
    Q = _cons1(*[np.broadcast_to(a, X.shape) for a in prim(X)], gamma)   # (3, 6, nx)
    avg = np.einsum('g,cgi->ci', gw, Q)
    mom = np.einsum('g,cgi->ci', gw * gx, Q)
    return np.ascontiguousarray(np.stack([avg, mom]))


def project2d(prim, nx, ny, extent, gamma):
    """prim(X, Y) -> (rho, u, v, p); returns U (3, 4, ny, nx)."""
    x0, x1, y0, y1 = extent
    gx, gw = _gauss6()
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    out = np.zeros((3, 4, ny, nx))
    for b in range(6):            # eta points
        Y = (yc + gx[b] * dy)[:, None] + np.zeros((1, nx))
        for a in range(6):        # xi points
            X = (xc + gx[a] * dx)[None, :] + np.zeros((ny, 1))
            Q = _cons2(*[np.broadcast_to(f, X.shape) for f in prim(X, Y)], gamma)
            w = gw[a] * gw[b]
            out[0] += w * Q
            out[1] += w * gx[a] * Q
            out[2] += w * gx[b] * Q
    return out


# ---------------------------------------------------------------------------
# 1D workloads
# ---------------------------------------------------------------------------

def smooth_wave_1d(nx=200, gamma=1.4, seed=None, amp=1e-3):
    """Smooth density wave on [0, 2 pi) periodic: rho = 1 + 0.2 sin x, u = 1,
    p = 1.  With ``seed``, a random Fourier perturbation of relative size
    ``amp`` (modes 1..8) is added to rho, u and p."""
    if seed is None:
        def prim(x):
            return 1.0 + 0.2 * np.sin(x), np.ones_like(x), np.ones_like(x)
    else:
        rng = np.random.default_rng([SEED, 1, seed])
        k = np.arange(1, 9)
        ph = rng.uniform(0, 2 * np.pi, (3, 8))
        a = rng.standard_normal((3, 8)) * amp

        def prim(x):
            pert = [np.sum(a[q][:, None, None] * np.sin(k[:, None, None] * x[None] + ph[q][:, None, None]),
                           axis=0) for q in range(3)]
            return (1.0 + 0.2 * np.sin(x) + pert[0], 1.0 + pert[1], 1.0 + pert[2])
    return project1d(prim, nx, 0.0, 2 * np.pi, gamma)


def riemann_1d(left, right, nx=2000, x0=0.0, x1=1.0, xd=0.5, gamma=1.4):
    """Piecewise-constant (rho, u, p) states with the diaphragm at xd."""
    def prim(x):
        L = x < xd
        return tuple(np.where(L, left[q], right[q]) for q in range(3))
    return project1d(prim, nx, x0, x1, gamma)


def sod_1d(nx=2000, gamma=1.4):
    return riemann_1d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), nx, gamma=gamma)


def double_rarefaction_1d(nx=2000, gamma=1.4):
    """Low-density double rarefaction (1,-2,0.4) | (1,2,0.4)."""
    return riemann_1d((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), nx, gamma=gamma)


def sedov_1d(nx=400, gamma=1.4, e_blast=3200000.0):
    """Example 5.5: (rho, u, E) = (1, 0, 1e-12) on [-2, 2], the cell right of
    x = 0 (the centre cell for even nx) holding E = e_blast / dx.  Returns U
    (2, 3, nx); zero moments."""
    dx = 4.0 / nx
    U = np.zeros((2, 3, nx))
    U[0, 0] = 1.0
    U[0, 2] = 1e-12
    U[0, 2, nx // 2] = e_blast / dx
    return U


def leblanc_1d(nx=3200, gamma=1.4):
    """Example 5.6: (rho, u, p) = (2, 0, 1e9) on [-10, 0), (0.001, 0, 1) on [0, 10]."""
    return riemann_1d((2.0, 0.0, 1e9), (0.001, 0.0, 1.0), nx, -10.0, 10.0, 0.0, gamma)


def random_smooth_1d(nx, seed, gamma=1.4):
    """Smooth random periodic state on [0, 1] (modes 1..4) plus small
    cell-level noise on the moments, for parity tests."""
    rng = np.random.default_rng([SEED, 11, seed])
    k = np.arange(1, 5)
    a = rng.uniform(-1, 1, (3, 4)) * np.array([0.15, 0.3, 0.15])[:, None] / k
    ph = rng.uniform(0, 2 * np.pi, (3, 4))

    def prim(x):
        f = [np.sum(a[q][:, None, None] * np.sin(2 * np.pi * k[:, None, None] * x[None]
                                                + ph[q][:, None, None]), axis=0) for q in range(3)]
        return 1.0 + f[0], 0.5 + f[1], 1.0 + f[2]
    U = project1d(prim, nx, 0.0, 1.0, gamma)
    U[1] += 1e-4 * rng.standard_normal(U[1].shape)
    return U


# ---------------------------------------------------------------------------
# 2D workloads
# ---------------------------------------------------------------------------

def viscous_shock_tube_2d(nx=1000, ny=500, gamma=1.4, seed=None, amp=0.0):
    """Viscous shock tube on [0,1] x [0,0.5]: (rho, p) = (120, 120/gamma) for
    x < 0.5 and (1.2, 1.2/gamma) for x >= 0.5, at rest.  With ``seed``, smooth
    random modes of relative amplitude ``amp`` perturb rho, u, v and p (for
    parity tests that need flow next to the walls)."""
    modes = None
    if seed is not None:
        rng = np.random.default_rng([SEED, 13, seed])
        modes = (rng.integers(1, 6, (4, 3)), rng.integers(1, 6, (4, 3)),
                 rng.uniform(0, 2 * np.pi, (4, 3)), rng.uniform(-1, 1, (4, 3)) * amp)

    def prim(X, Y):
        L = X < 0.5
        rho = np.where(L, 120.0, 1.2)
        f = [np.zeros_like(X) for _ in range(4)]
        if modes is not None:
            kx, ky, ph, a = modes
            f = [sum(a[q, m] * np.sin(np.pi * kx[q, m] * X + 2 * np.pi * ky[q, m] * Y + ph[q, m])
                     for m in range(3)) for q in range(4)]
        return rho * (1.0 + f[0]), f[1], f[2], rho / gamma * (1.0 + f[3])
    return project2d(prim, nx, ny, (0.0, 1.0, 0.0, 0.5), gamma)


def sedov_2d(n=160, gamma=1.4, e_blast=0.244816, extent=1.1):
    """Example 5.7: on [0, 1.1]^2, (rho, u, v, E) = (1, 0, 0, 1e-12), the
    corner cell [0, dx] x [0, dy] holding E = e_blast / (dx dy).  Returns U
    (3, 4, n, n); zero moments."""
    h = extent / n
    U = np.zeros((3, 4, n, n))
    U[0, 0] = 1.0
    U[0, 3] = 1e-12
    U[0, 3, 0, 0] = e_blast / (h * h)
    return U


def mach2000_jet(nx=640, ny=320, gamma=5.0 / 3.0):
    """Example 5.9 on [0, 1] x [-0.25, 0.25]: ambient (rho, u, v, p) =
    (0.5, 0, 0, 0.4127) everywhere; the left side takes (5, 800, 0, 0.4127)
    where the boundary cell's centre has |y| < 0.05 and (5, 0, 0, 0.4127)
    elsewhere.  Returns U (3, 4, ny, nx) (zero moments) and the inflow profile
    (ny, 4) of primitive states."""
    U = np.zeros((3, 4, ny, nx))
    U[0, 0] = 0.5
    U[0, 3] = 0.4127 / (gamma - 1.0)
    yc = -0.25 + (np.arange(ny) + 0.5) * (0.5 / ny)
    prof = np.tile(np.array([5.0, 0.0, 0.0, 0.4127]), (ny, 1))
    prof[np.abs(yc) < 0.05, 1] = 800.0
    return U, prof


def shock_diffraction(h=0.125, mach=5.09, gamma=1.4):
    """Example 5.8: the domain [0,1]x[6,11] U [1,13]x[0,11] inside the grid of
    [0,13]x[0,11] with square cells of size h (1/h integer, so the step's
    faces are cell faces); a Mach-`mach` shock at x = 0.5 above the step
    moving right into (rho, u, v, p) = (1.4, 0, 0, 1); the post-shock state
    from the Rankine-Hugoniot relations.  Returns (U, solid mask (ny, nx),
    post-shock primitive state)."""
    nx, ny = int(round(13.0 / h)), int(round(11.0 / h))
    m2 = mach * mach
    r1, p1 = 1.4, 1.0
    c1 = np.sqrt(gamma * p1 / r1)
    r2 = r1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u2 = mach * c1 * (1.0 - r1 / r2)
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(xc, yc)
    solid = (X < 1.0) & (Y < 6.0)
    post = (X < 0.5) & ~solid
    U = np.zeros((3, 4, ny, nx))
    U[0] = np.where(post, _cons2(r2, u2, 0.0, p2, gamma)[:, None, None] * np.ones((4, ny, nx)),
                    _cons2(r1, 0.0, 0.0, p1, gamma)[:, None, None] * np.ones((4, ny, nx)))
    return U, solid, (r2, u2, 0.0, p2)


class ShockMixingLayer:
    """Example 5.11 on [0, 200] x [-20, 20]: a mixing layer u = 2.5 +
    0.5 tanh(2y), rho = 1.6374 above y = 0 and 0.3626 below, p = 0.3327,
    forced at the inflow by v'(y, t) = sum_k a_k cos(2 pi k t / T0 + phi_k)
    exp(-y^2 / b) (a_1 = a_2 = 0.05, phi = (0, pi/2), b = 10, T0 = 30 / 2.68);
    the post-shock state (2.1101, 2.9709, -0.1367, 0.4754) enters through the
    top, slip wall at the bottom, outflow on the right.  Initial state: the
    inflow state at t = 0 in every column."""

    extent = (0.0, 200.0, -20.0, 20.0)
    bc = ('inflow', 'outflow', 'slip', 'inflow')
    top = (2.1101, 2.9709, -0.1367, 0.4754)

    def __init__(self, nx=500, ny=100, gamma=1.4):
        self.nx, self.ny, self.gamma = nx, ny, gamma
        self.yc = -20.0 + (np.arange(ny) + 0.5) * (40.0 / ny)

    @staticmethod
    def prim(y, t):
        """(rho, u, v, p) of the inflow at heights y and time t."""
        T0 = 30.0 / 2.68
        v = sum(0.05 * np.cos(2.0 * np.pi * k * t / T0 + ph) * np.exp(-y * y / 10.0)
                for k, ph in ((1, 0.0), (2, 0.5 * np.pi)))
        rho = np.where(y > 0.0, 1.6374, 0.3626)
        return rho, 2.5 + 0.5 * np.tanh(2.0 * y), v, np.full_like(y, 0.3327)

    def inflow(self, t):
        """Left-side profile (ny, 4) of primitive states at time t."""
        return np.column_stack([np.broadcast_to(q, self.yc.shape) for q in self.prim(self.yc, t)])

    def initial(self):
        return project2d(lambda X, Y: self.prim(Y, 0.0), self.nx, self.ny, self.extent, self.gamma)


class Mach10Reflection:
    """Example 5.10 (gamma = 1.4): a Mach-10 shock at 60 degrees to a wall
    reflects along it and diffracts round a step.  The domain is read as
    [0,1]x[0,1] U [1,3]x[-1,1] (the text lists the second rectangle's
    intervals in the order y, x), inside the grid of [0,3]x[-1,1], whose
    cells with centres at x < 1, y < 0 are solid.  Post-shock state (8,
    33/4 sin(pi/3), -33/4 cos(pi/3), 116.5) left of x = 1/6 + y/sqrt(3),
    (1.4, 0, 0, 1) right of it.  Left side: inflow of the post-shock state;
    right side and bottom: outflow; along y = 0 the solid cells with centres
    at x < 1/6 hold the post-shock state, and the wall from x = 1/6 to 1 and
    the step face {1} x [-1, 0] are reflective; the top follows the exact
    shock, one state per boundary cell from its centre: post-shock for
    x <= 1/6 + (1 + 20 t)/sqrt(3)."""

    extent = (0.0, 3.0, -1.0, 1.0)
    bc = ('inflow', 'outflow', 'outflow', 'inflow')
    post = (8.0, 8.25 * np.sin(np.pi / 3.0), -8.25 * np.cos(np.pi / 3.0), 116.5)
    pre = (1.4, 0.0, 0.0, 1.0)

    def __init__(self, nx=480, ny=480, gamma=1.4):
        self.nx, self.ny, self.gamma = nx, ny, gamma
        self.xc = (np.arange(nx) + 0.5) * (3.0 / nx)
        self.yc = -1.0 + (np.arange(ny) + 0.5) * (2.0 / ny)
        X, Y = np.meshgrid(self.xc, self.yc)
        self.solid = (X < 1.0) & (Y < 0.0)
        self.fixed = self.solid & (X < 1.0 / 6.0)

    def prim(self, X, Y):
        left = X < 1.0 / 6.0 + Y / np.sqrt(3.0)
        return tuple(np.where(left, a, b) for a, b in zip(self.post, self.pre))

    def top(self, t):
        """Top-side profile (nx, 4) of primitive states at time t."""
        left = self.xc <= 1.0 / 6.0 + (1.0 + 20.0 * t) / np.sqrt(3.0)
        return np.where(left[:, None], np.array(self.post)[None, :], np.array(self.pre)[None, :])

    def initial(self):
        return project2d(self.prim, self.nx, self.ny, self.extent, self.gamma)


def random_smooth_2d(nx, ny, seed, gamma=1.4, extent=(0.0, 1.0, 0.0, 1.0), noise=1e-4):
    """Smooth random periodic state (4 Fourier modes per field, Mach < 0.5)
    with small cell-level noise on the moments, for parity tests."""
    rng = np.random.default_rng([SEED, 12, seed])
    x0, x1, y0, y1 = extent
    kx = rng.integers(-3, 4, (4, 4))
    ky = rng.integers(-3, 4, (4, 4))
    a = rng.uniform(-1, 1, (4, 4)) * np.array([0.1, 0.15, 0.15, 0.1])[:, None]
    ph = rng.uniform(0, 2 * np.pi, (4, 4))

    def prim(X, Y):
        xs = 2 * np.pi * (X - x0) / (x1 - x0)
        ys = 2 * np.pi * (Y - y0) / (y1 - y0)
        f = [sum(a[q, m] * np.sin(kx[q, m] * xs + ky[q, m] * ys + ph[q, m]) for m in range(4))
             for q in range(4)]
        return 1.0 + f[0], 0.3 + f[1], -0.2 + f[2], 1.0 / gamma + f[3]
    U = project2d(prim, nx, ny, extent, gamma)
    U[1:] += noise * rng.standard_normal(U[1:].shape)
    return U


def shear_layer_2d(n=256, gamma=1.4):
    """Double shear layer on [0,1]^2 periodic: rho = 1, p = 1/gamma,
    u = tanh(80(y-1/4)) for y <= 1/2 else tanh(80(3/4-y)), v = 0.05 sin(2 pi x)."""
    def prim(X, Y):
        u = np.where(Y <= 0.5, np.tanh(80.0 * (Y - 0.25)), np.tanh(80.0 * (0.75 - Y)))
        return np.ones_like(X), u, 0.05 * np.sin(2 * np.pi * X), np.full_like(X, 1.0 / gamma)
    return project2d(prim, n, n, (0.0, 1.0, 0.0, 1.0), gamma)


def batched_periodic_2d(n_instances=64, gamma=1.4, sizes=(64, 128, 256, 512), modes=8,
                        amp=0.3):
    """Instance k (rng([2608, k])): n from ``sizes``, log10 Re ~ U(2, 4),
    rho = 1, p = 1/gamma, u and v sums of ``modes`` random-phase Fourier modes
    (wave numbers in {-4..4}^2 without 0) normalised to max |.| = amp (the max
    taken on a 4n x 4n point grid).  Returns a list of (n, Re, U).

    A mode cos(2 pi (kx x + ky y) + phi) is separable,
    cos(2 pi kx x) cos(2 pi ky y + phi) - sin(2 pi kx x) sin(2 pi ky y + phi),
    so every field on a tensor grid is a (modes x ny)^T (modes x nx) product."""
    gx, gw = _gauss6()
    out = []
    for k in range(n_instances):
        rng = np.random.default_rng([SEED, k])
        n = int(rng.choice(sizes))
        Re = 10.0 ** rng.uniform(2.0, 4.0)
        kv = []
        while len(kv) < 2 * modes:
            w = rng.integers(-4, 5, 2)
            if w[0] or w[1]:
                kv.append(w)
        kv = np.array(kv).reshape(2, modes, 2)
        ph = rng.uniform(0, 2 * np.pi, (2, modes))

        def field(q, xs, ys):
            ax = 2 * np.pi * np.outer(kv[q, :, 0], xs)                   # (modes, nx)
            by = 2 * np.pi * np.outer(kv[q, :, 1], ys) + ph[q][:, None]  # (modes, ny)
            return np.cos(by).T @ np.cos(ax) - np.sin(by).T @ np.sin(ax)
        xs4 = (np.arange(4 * n) + 0.5) / (4 * n)
        scale = [amp / np.max(np.abs(field(q, xs4, xs4))) for q in range(2)]
        h = 1.0 / n
        xc = (np.arange(n) + 0.5) * h
        U = np.zeros((3, 4, n, n))
        for b in range(6):            # eta points
            yb = xc + gx[b] * h
            for a in range(6):        # xi points
                xa = xc + gx[a] * h
                u = scale[0] * field(0, xa, yb)
                v = scale[1] * field(1, xa, yb)
                Q = _cons2(np.ones_like(u), u, v, np.full_like(u, 1.0 / gamma), gamma)
                w = gw[a] * gw[b]
                U[0] += w * Q
                U[1] += w * gx[a] * Q
                U[2] += w * gx[b] * Q
        out.append((n, Re, U))
    return out


def c1_config():
    """Smooth 1D wave: gamma 1.4, Pr 0.72, mu 0.01, CFL 0.3, to t = 1."""
    return dict(nx=200, extent=(0.0, 2 * math.pi), gamma=1.4, Pr=0.72, mu_ref=0.01, cfl=0.3,
                t_final=1.0, bc=('periodic', 'periodic'))
