"""Pins of the oracle's characteristic bases, positivity wave-speed bound,
smoothness-indicator quadratic form, limiter output and stencil tables.

Each test checks the oracle against a property the paper or the mathematics
fixes, computed here by a different route than the oracle's own:

* characteristic bases (Sec. 2.1 and 3.1): the right eigenvectors must
  diagonalise the convective-flux Jacobian, obtained here by a complex-step
  derivative of the Euler flux of eqs. (2.1)/(3.1);
* the positivity bound of the Lax-Friedrichs coefficient (eqs. (2.3), (3.3)):
  for any coefficient above it, the states u -+ f(u, s)/beta must have
  positive density and internal energy (the property the bound is derived
  for), with equality reached in the cases where it is sharp;
* the Sobolev smoothness indicator (reading of the indicators of
  Appendix A): exact symbolic integrals of the squared derivatives of
  rational quartics, and a closed form worked by hand;
* the positivity limiter (Sec. 2.1 and 3.1, limiter paragraphs): every
  limited point has density and pressure at least the floor, and in 2D the
  same scaling also keeps the checked-but-unmodified volume points admissible;
* P18: the oracle's floating-point stencil maps agree with the exact
  rational maps from which the device code is generated.
"""

import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import rk
from oracle.common import (Options, Physics, beta_pp1d, beta_pp2d, invert_cells, pressure,
                           right_eigvecs1d, right_eigvecs2d)
from oracle.recon import Hweno1D, Hweno2D
from oracle.scheme1d import Scheme1D
from oracle.scheme2d import Scheme2D
from paper_2608_10569_amd import workloads

GAMMA = 1.4


# ---------------------------------------------------------------------------
# Characteristic bases: L A(u) R = diag(eigenvalues), A by complex step
# ---------------------------------------------------------------------------

def euler_flux(U, gamma, direction):
    """Convective flux of eqs. (2.1)/(3.1) (viscosity zero), written from the
    conservation laws: mass flux, momentum flux plus pressure, enthalpy flux."""
    rho, E = U[0], U[-1]
    mom = U[1:-1]
    p = (gamma - 1.0) * (E - 0.5 * sum(m * m for m in mom) / rho)
    un = mom[direction] / rho
    out = [mom[direction]]
    for k, m in enumerate(mom):
        out.append(m * un + (p if k == direction else 0.0))
    out.append((E + p) * un)
    return np.array(out)


def jacobian_cs(U, gamma, direction):
    """Complex-step Jacobian dF/dU (exact to rounding; step 1e-30)."""
    n = len(U)
    A = np.zeros((n, n))
    for k in range(n):
        Uc = U.astype(complex)
        Uc[k] += 1e-30j
        A[:, k] = np.imag(euler_flux(Uc, gamma, direction)) / 1e-30
    return A


def random_states(rng, dim, n):
    """Primitive states over a wide range, including strong flows and near-vacuum."""
    rho = 10.0 ** rng.uniform(-3, 2, n)
    p = 10.0 ** rng.uniform(-4, 3, n)
    vel = rng.uniform(-1, 1, (dim, n)) * 10.0 ** rng.uniform(-2, 2, (dim, n))
    return rho, vel, p


def cons(rho, vel, p, gamma):
    kin = 0.5 * rho * sum(v * v for v in vel)
    return np.array([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + kin])


@pytest.mark.parametrize('dim,direction', [(1, 0), (2, 0), (2, 1)])
def test_eigenbasis_diagonalises_flux_jacobian(dim, direction):
    rng = np.random.default_rng([2608, 101, dim, direction])
    rho, vel, p = random_states(rng, dim, 200)
    U = cons(rho, vel, p, GAMMA)
    if dim == 1:
        R = right_eigvecs1d(U, GAMMA)
    else:
        R = right_eigvecs2d(U, GAMMA, direction)
    L = invert_cells(R)
    worst = 0.0
    for n in range(U.shape[1]):
        A = jacobian_cs(U[:, n], GAMMA, direction)
        Rn, Ln = R[:, :, n], L[:, :, n]
        c = math.sqrt(GAMMA * p[n] / rho[n])
        un = vel[direction][n]
        lam = [un - c] + [un] * dim + [un + c]
        D = Ln @ A @ Rn
        # rounding of the inverse grows with the conditioning of R (strong
        # flows make the acoustic columns nearly parallel)
        kappa = np.linalg.cond(Rn)
        scale = (abs(un) + c) * kappa
        worst = max(worst, np.max(np.abs(D - np.diag(lam))) / scale)
        assert np.max(np.abs(Ln @ Rn - np.eye(dim + 2))) < 1e-13 * kappa
        # textbook normalisation (the nonlinear weights are not invariant to
        # rescaling a field): unit density entry of the acoustic and entropy
        # columns; the shear column carries a unit tangential momentum
        assert Rn[0, 0] == 1.0 and Rn[0, 1] == 1.0 and Rn[0, dim + 1] == 1.0
        if dim == 2:
            tang = 2 - direction
            assert Rn[0, 2] == 0.0 and Rn[tang, 2] == 1.0 and Rn[1 + direction, 2] == 0.0
    assert worst < 1e-13, worst


# ---------------------------------------------------------------------------
# Positivity bound of the Lax-Friedrichs coefficient
# ---------------------------------------------------------------------------

def total_flux_1d(U, tau, q, gamma):
    """f = (m, m u + p - tau, (E + p) u - tau u + q): eq. (2.1) with the
    viscous stress tau and the heat flux q as given numbers."""
    rho, m, E = U
    u = m / rho
    p = (gamma - 1) * (E - m * u / 2)
    return np.array([m, m * u + p - tau, (E + p) * u - tau * u + q], dtype=object)


def total_flux_2d(U, txx, txy, q, gamma):
    """x-flux of eq. (3.1) with stresses and heat flux as given numbers."""
    rho, m, n, E = U
    u, v = m / rho, n / rho
    p = (gamma - 1) * (E - (m * u + n * v) / 2)
    return np.array([m, m * u + p - txx, n * u - txy, (E + p) * u - txx * u - txy * v + q],
                    dtype=object)


def admissible(W):
    """Positive density and internal energy, decided in exact arithmetic."""
    rho, E = W[0], W[-1]
    if rho <= 0:
        return False
    kin = sum(m * m for m in W[1:-1]) / (2 * rho)
    return E - kin > 0


def exact(x):
    return np.array([Fraction(float(v)) for v in np.ravel(x)], dtype=object)


def smallest_admissible_beta(U, f, hi):
    """Smallest b (to 1e-13 relative) with U - f/b' and U + f/b' admissible for
    every b' >= b.  For fixed U and f the admissible set of s = 1/b is an
    interval [0, s*) (density is linear in s, density times internal energy
    a quadratic positive at s = 0), so bisection applies.  U and f hold exact
    rationals: near a strong flow the internal energy of the split states is
    far below the rounding of a floating-point E - |m|^2/(2 rho)."""
    def ok(b):
        fb = Fraction(b)
        return admissible(U - f / fb) and admissible(U + f / fb)
    assert ok(hi)
    lo = 0.0
    while hi - lo > 1e-13 * hi:
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


def _check_bound(U, f, beta):
    # just above the bound the split states are admissible ...
    b = beta * (1.0 + 1e-9)
    fb = Fraction(b)
    assert admissible(U - f / fb) and admissible(U + f / fb)
    # ... and the bound is never below the smallest admissible coefficient
    bstar = smallest_admissible_beta(U, f, b)
    assert bstar <= b
    return bstar / beta


def test_beta_pp_bound_admissibility_1d():
    """Eq. (2.3): beta above the bracket keeps u -+ f/beta admissible, for
    stresses and heat fluxes of any size; sharp where the convective speed
    vanishes and only one of the viscous terms is present."""
    rng = np.random.default_rng([2608, 102])
    ph = Physics(gamma=GAMMA, Pr=0.72, mu_ref=1.0)
    tight = []
    cases = []
    for _ in range(300):
        rho, vel, p = random_states(rng, 1, 1)
        rho, u, p = rho[0], vel[0, 0], p[0]
        tau = p * rng.uniform(-30, 30)
        e = p / ((GAMMA - 1) * rho)
        q = rho * e ** 1.5 * rng.uniform(-30, 30)
        cases.append((rho, u, p, tau, q))
    # the sharp cases: u = 0 with tau = p (heat flux only), or q = 0
    cases += [(1.3, 0.0, 0.7, 0.7, 5.0), (0.2, 0.0, 2.0, 2.0, -40.0),
              (1.3, 0.0, 0.7, -3.0, 0.0), (0.05, 0.0, 1e-3, 0.5, 0.0)]
    for rho, u, p, tau, q in cases:
        U = cons(rho, [u], p, GAMMA)
        # the oracle takes gradients: tau = (4/3) mu u_x, q = -gamma mu e_x / Pr
        ux = tau / (4.0 / 3.0)
        ex = -q * ph.Pr / GAMMA
        beta = float(beta_pp1d(U, ux, ex, ph))
        Ue = exact(U)
        f = total_flux_1d(Ue, Fraction(tau), Fraction(q), Fraction(GAMMA))
        tight.append(_check_bound(Ue, f, beta))
    assert max(tight[-4:]) > 1.0 - 1e-6          # sharp: equality reached
    assert max(tight) <= 1.0 + 1e-9


def test_beta_pp_bound_admissibility_2d():
    """Eq. (3.3), x- and y-directions: the same property with the normal
    stress, the shear stress and the heat flux of that direction."""
    rng = np.random.default_rng([2608, 103])
    ph = Physics(gamma=GAMMA, Pr=0.73, mu_ref=1.0)
    tight = []
    cases = []
    for _ in range(300):
        rho, vel, p = random_states(rng, 2, 1)
        rho, p, u, v = rho[0], p[0], vel[0, 0], vel[1, 0]
        e = p / ((GAMMA - 1) * rho)
        s = rng.uniform(-30, 30, 6) * np.array([p, p, p, p, rho * e ** 1.5, rho * e ** 1.5])
        cases.append((rho, u, v, p, s))
    # sharp cases: no convective speed, only the shear stress (normal stress
    # equal to the pressure), or only the heat flux
    sharp = [(1.1, 0.0, 0.3, 0.9, 'shear'), (0.4, 0.0, -2.0, 3.0, 'heat')]
    for d in (0, 1):
        for rho, u, v, p, s in cases:
            U = cons(rho, [u, v], p, GAMMA)
            grads = stresses_to_gradients(s, 1.0, ph)
            beta = float(beta_pp2d(U, grads, ph, d))
            tight.append(_check_bound(*_flux_2d_exact(U, s, d), beta))
        for rho, u, v, p, kind in sharp:
            vel = [u, v] if d == 0 else [v, u]
            U = cons(rho, vel, p, GAMMA)
            s = np.zeros(6)
            if kind == 'shear':
                s[0] = s[2] = p          # normal stress equal to the pressure
                s[1] = 7.0 * p
            else:
                s[0] = s[2] = p
                s[4] = s[5] = 9.0 * rho * (p / ((GAMMA - 1) * rho)) ** 1.5
            grads = stresses_to_gradients(s, 1.0, ph)
            beta = float(beta_pp2d(U, grads, ph, d))
            r = _check_bound(*_flux_2d_exact(U, s, d), beta)
            assert r > 1.0 - 1e-6, (kind, d, r)
    assert max(tight) <= 1.0 + 1e-9


def _flux_2d_exact(U, s, d):
    """Exact-rational state and flux of direction d with stresses s[0:3] and
    heat fluxes s[4:6] (the y-flux by exchanging the roles of x and y)."""
    Ue = exact(U)
    txx, txy, tyy, qx, qy = (Fraction(float(s[k])) for k in (0, 1, 2, 4, 5))
    g = Fraction(GAMMA)
    if d == 0:
        return Ue, total_flux_2d(Ue, txx, txy, qx, g)
    Us = np.array([Ue[0], Ue[2], Ue[1], Ue[3]], dtype=object)
    f = total_flux_2d(Us, tyy, txy, qy, g)
    return Ue, np.array([f[0], f[2], f[1], f[3]], dtype=object)


def stresses_to_gradients(s, mu, ph):
    """Velocity and energy gradients (u_x, u_y, v_x, v_y, e_x, e_y) whose
    stresses (tau_xx, tau_xy, tau_yy) and heat fluxes (q_x, q_y) are s[0:3],
    s[4:6] (s[3] unused): tau_xx = mu (4/3 u_x - 2/3 v_y), tau_yy =
    mu (4/3 v_y - 2/3 u_x), tau_xy = mu (u_y + v_x), q = -gamma mu e_l / Pr."""
    txx, txy, tyy = s[0] / mu, s[1] / mu, s[2] / mu
    # solve [[4/3, -2/3], [-2/3, 4/3]] (u_x, v_y) = (txx, tyy)
    det = 16.0 / 9.0 - 4.0 / 9.0
    ux = (4.0 / 3.0 * txx + 2.0 / 3.0 * tyy) / det
    vy = (2.0 / 3.0 * txx + 4.0 / 3.0 * tyy) / det
    uy = vx = 0.5 * txy
    ex = -s[4] * ph.Pr / (ph.gamma * mu)
    ey = -s[5] * ph.Pr / (ph.gamma * mu)
    return np.array([ux, uy, vx, vy, ex, ey])


# ---------------------------------------------------------------------------
# Sobolev smoothness indicator: exact integrals
# ---------------------------------------------------------------------------

XI, ETA = sp.symbols('xi eta')
HALF = sp.Rational(1, 2)


def exact_sobolev(poly, ndim):
    total = sp.Integer(0)
    if ndim == 1:
        for k in range(1, 5):
            total += sp.integrate(sp.diff(poly, XI, k) ** 2, (XI, -HALF, HALF))
        return total
    for a in range(5):
        for b in range(5 - a):
            if a + b == 0:
                continue
            d = poly
            if a:
                d = sp.diff(d, XI, a)
            if b:
                d = sp.diff(d, ETA, b)
            total += sp.integrate(sp.integrate(d ** 2, (XI, -HALF, HALF)), (ETA, -HALF, HALF))
    return total


def test_sobolev_indicator_exact_integrals_1d():
    rng = np.random.default_rng([2608, 104])
    G = Hweno1D().G
    for _ in range(5):
        num = rng.integers(-9, 10, 5)
        den = rng.integers(1, 8, 5)
        coef = [sp.Rational(int(a), int(b)) for a, b in zip(num, den)]
        poly = sum(c * XI ** k for k, c in enumerate(coef))
        want = float(exact_sobolev(poly, 1))
        cv = np.array([float(c) for c in coef])
        got = cv @ G @ cv
        assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (got, want)
    # hand value: p = xi^2 gives int (2 xi)^2 + int 2^2 = 1/3 + 4
    c = np.zeros(5)
    c[2] = 1.0
    assert abs(c @ G @ c - 13.0 / 3.0) < 1e-14


def test_sobolev_indicator_exact_integrals_2d():
    rng = np.random.default_rng([2608, 105])
    rec = Hweno2D()
    G = rec.G
    for _ in range(4):
        num = rng.integers(-9, 10, 15)
        den = rng.integers(1, 8, 15)
        coef = [sp.Rational(int(a), int(b)) for a, b in zip(num, den)]
        poly = sum(c * XI ** px * ETA ** py for c, (px, py) in zip(coef, rec.MONOS))
        want = float(exact_sobolev(poly, 2))
        cv = np.array([float(c) for c in coef])
        got = cv @ G @ cv
        assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (got, want)
    # hand value for p = xi^2 eta^2: the derivatives of orders 1..4 with each
    # multi-index once, d_x: 1/240, d_y: 1/240, d_xx: 1/20, d_yy: 1/20,
    # d_xy: 1/9, d_xxy: 4/3, d_xyy: 4/3, d_xxyy: 16 (the others vanish)
    c = np.zeros(15)
    c[rec.MONOS.index((2, 2))] = 1.0
    want = (Fraction(1, 240) * 2 + Fraction(1, 20) * 2 + Fraction(1, 9) + Fraction(4, 3) * 2
            + 16)
    assert abs(c @ G @ c - float(want)) < 1e-13
    # a linear candidate a + b xi + c eta has beta = b^2 + c^2
    c = np.zeros(15)
    c[0], c[1], c[2] = 5.0, -3.0, 2.0
    assert abs(c @ G @ c - 13.0) < 1e-13


# ---------------------------------------------------------------------------
# Positivity limiter output
# ---------------------------------------------------------------------------

def _pressure_rounding(W, Wbar, gamma):
    """Size of the rounding of the pressure of a limited point: the point is
    formed as ubar + theta (u - ubar), so its energy carries rounding of the
    size of the larger of the two energies."""
    def scale(X):
        return np.abs(X[-1]) + 0.5 * sum(m * m for m in X[1:-1]) / X[0]
    return 16.0 * np.finfo(float).eps * (gamma - 1.0) * np.maximum(scale(W), scale(Wbar))


def _assert_points_admissible(P, ubar, gamma, eps_pp):
    """P[p, c, ...] limited points of cells with averages ubar[c, ...]."""
    rbar = ubar[0]
    pbar = pressure(ubar, gamma)
    eps = np.minimum(np.minimum(eps_pp, rbar), pbar)
    rho = P[:, 0]
    assert np.all(rho >= eps * (1.0 - 1e-12)), float(np.min(rho - eps))
    for q in range(P.shape[0]):
        pq = pressure(P[q], gamma)
        tol = _pressure_rounding(P[q], ubar, gamma)
        assert np.all(pq >= eps - tol), float(np.min(pq - eps + tol))


class _Checked1D(Scheme1D):
    """Scheme1D that checks the limited points after every residual."""

    def residual(self, U, source=None):
        out = super().residual(U, source)
        pts = self.last['points']                       # (4, c, nx), limited
        _assert_points_admissible(pts, U[0], self.phys.gamma, self.opts.eps_pp)
        self.acts = getattr(self, 'acts', 0) + out[2]['pp_cells']
        return out


def test_limited_points_admissible_1d_double_rarefaction():
    """Example 5.4 data: the limiter acts during the run; every limited LGL
    value has density and pressure at least the floor."""
    ph = Physics(gamma=GAMMA, Pr=0.72, mu_ref=1e-3)
    n = 100
    s = _Checked1D(n, 0.0, 1.0, ph, Options(cfl=0.3, b_visc=0.001, t_final=0.1),
                   bc=('outflow', 'outflow'))
    U = workloads.riemann_1d((7.0, -1.0, 0.2), (7.0, 1.0, 0.2), n)
    t = 0.0
    while t < 0.1 - 1e-12:
        U, dt, info = rk.rk3_step(s, U, t)
        t += dt
    assert s.acts > 0


def test_limited_points_admissible_1d_sedov():
    """Example 5.5 start (blast cell, ambient pressure below the floor): the
    limiter acts in the first steps; its output is admissible."""
    ph = Physics(gamma=GAMMA, Pr=0.72, mu_ref=1e-3)
    n = 80
    s = _Checked1D(n, -2.0, 2.0, ph, Options(cfl=0.6, b_visc=0.001),
                   bc=('inflow', 'outflow'), inflow={0: np.array([1.0, 0.0, 1e-12])})
    U = workloads.sedov_1d(n, e_blast=3200000.0)
    t = 0.0
    for _ in range(4):
        U, dt, info = rk.rk3_step(s, U, t)
        t += dt
    assert s.acts > 0


def _check_2d_limiter(sc, U):
    Ug = sc.ghost(U)
    r = sc.reconstruct(Ug)
    g, eps_pp = sc.phys.gamma, sc.opts.eps_pp
    ubar = r['ubar']
    active = (np.real(r['theta1']) < 1.0) | (np.real(r['theta2']) < 1.0)
    _assert_points_admissible(np.concatenate([r['xface'], r['yface']]), ubar, g, eps_pp)
    # the volume points are checked but not modified: the same two scalings
    # applied to them must keep them admissible too (they take part in theta)
    for vol in (r['xvol'], r['yvol']):
        V = vol.copy()
        V[:, 0] = ubar[0] + r['theta1'] * (vol[:, 0] - ubar[0])
        V = ubar + r['theta2'] * (V - ubar)
        _assert_points_admissible(V, ubar, g, eps_pp)
    return int(np.count_nonzero(active))


def test_limited_points_admissible_2d():
    """2D: the Sedov corner blast (Example 5.7) and near-vacuum troughs in a
    smooth flow; the limiter acts and every face point it returns, and every
    volume point under the same scaling, has density and pressure at least
    the floor."""
    ph = Physics(gamma=GAMMA, Pr=0.72, mu_ref=1e-3)
    n = 24
    sc = Scheme2D(n, n, 0.0, 1.1, 0.0, 1.1, ph, Options(),
                  bc=('slip', 'outflow', 'slip', 'outflow'))
    assert _check_2d_limiter(sc, workloads.sedov_2d(n)) > 0
    U = workloads.random_smooth_2d(16, 16, seed=3)
    U[0, 0, 6:9, 5:10] = 2e-3
    U[0, 3, 6:9, 5:10] = 0.5 * (U[0, 1, 6:9, 5:10] ** 2 + U[0, 2, 6:9, 5:10] ** 2) / 2e-3 + 2e-3
    sc = Scheme2D(16, 16, 0.0, 1.0, 0.0, 1.0, ph, Options())
    assert _check_2d_limiter(sc, U) > 0
    # an isolated near-vacuum cell: its reconstruction dips below the floor
    # inside the cell while the face values stay positive, so the volume
    # points decide theta there
    U = workloads.random_smooth_2d(16, 16, seed=3)
    U[0, 0, 7, 7] = 1e-2
    U[0, 3, 7, 7] = 0.5 * (U[0, 1, 7, 7] ** 2 + U[0, 2, 7, 7] ** 2) / 1e-2 + 1e-2
    assert _check_2d_limiter(sc, U) > 0


# ---------------------------------------------------------------------------
# P18: oracle stencil maps against the exact rational maps of the generator
# ---------------------------------------------------------------------------

def _gen_tables():
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        'paper_2608_10569_amd', 'csrc')
    sys.path.insert(0, here)
    try:
        import gen_tables
    finally:
        sys.path.remove(here)
    return gen_tables


def test_p18_oracle_maps_match_exact_rationals():
    """The oracle solves its moment systems in FP64; the generator derives the
    same maps in exact rationals.  They agree to a few units in the last place
    of the largest map entry (16 ulps allowed)."""
    gt = _gen_tables()
    ulp16 = 16.0 * np.finfo(float).eps
    # 1D p0: inputs (um, uc, up, vm, vp), the oracle's input order
    ins1, co1 = gt.derive_1d()
    W1 = np.array([[float(co1[k].coeff(s)) for s in ins1] for k in range(5)])
    Q1 = Hweno1D().Q[0]
    assert np.max(np.abs(Q1 - W1)) <= ulp16 * np.max(np.abs(W1))
    # 2D p0: inputs a1..a9, x2 x4 x6 x8, y2 y4 y6 y8, the oracle's input order
    ins2, co2 = gt.derive_2d()
    rec = Hweno2D()
    assert [tuple(m) for m in gt.MONOS2] == [tuple(m) for m in rec.MONOS]
    W2 = np.array([[float(co2[m].coeff(s)) for s in ins2] for m in gt.MONOS2])
    assert np.max(np.abs(rec.Q[0] - W2)) <= ulp16 * np.max(np.abs(W2))
    # Sobolev quadratic forms
    for ndim, monos, G in ((1, list(range(5)), Hweno1D().G), (2, gt.MONOS2, rec.G)):
        beta, syms = gt.sobolev_form(monos, ndim)
        poly = sp.Poly(beta, *syms)
        for i in range(len(syms)):
            for j in range(len(syms)):
                mono = [0] * len(syms)
                mono[i] += 1
                mono[j] += 1
                q = poly.coeff_monomial(tuple(mono))
                want = float(q) if i == j else float(q) / 2.0
                assert abs(G[i, j] - want) <= 1e-13 * max(1.0, abs(want)), (ndim, i, j)
