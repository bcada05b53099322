"""Quadrature, complex-step-safe helpers and gas physics for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Citations refer to the paper (arXiv 2608.10569): sections, equations and
examples as numbered there.
"""

from dataclasses import dataclass, field
import math

import numpy as np

# ----------------------------------------------------------------------------
# Quadrature rules on the scaled cell [-1/2, 1/2].
# ----------------------------------------------------------------------------

#: Four-point Legendre-Gauss-Lobatto rule of the 1D scheme (Sec. 2.1, the
#: quadrature points listed after eq. (2.3)): end points are the interface
#: traces, the two interior points serve the volume-flux term of the moment
#: equation.  Exact for polynomials of degree <= 5.
LGL_NODES = np.array([-0.5, -math.sqrt(5.0) / 10.0, math.sqrt(5.0) / 10.0, 0.5])
LGL_WEIGHTS = np.array([1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0])

#: Three-point Gauss rule per direction of the 2D scheme (Sec. 3.1, after
#: eq. (3.3)).  Exact for polynomials of degree <= 5 per direction.
GAUSS3_NODES = np.array([-math.sqrt(15.0) / 10.0, 0.0, math.sqrt(15.0) / 10.0])
GAUSS3_WEIGHTS = np.array([5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0])


def gauss_legendre(n):
    """n-point Gauss-Legendre rule mapped to [-1/2, 1/2] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * x, 0.5 * w


# ----------------------------------------------------------------------------
# Helpers that treat complex arrays by their real part (complex-step safe).
# ----------------------------------------------------------------------------

def cabs(x):
    """|x| with the derivative of |x| at 0 taken as 0."""
    return x * np.sign(np.real(x))


def cmax(a, b):
    """Elementwise max by real part; ties go to the first argument."""
    return np.where(np.real(a) >= np.real(b), a, b)


def cmin(a, b):
    """Elementwise min by real part; ties go to the first argument."""
    return np.where(np.real(a) <= np.real(b), a, b)


def cmax_axis(x, axis):
    """Max along ``axis`` by real part; ties go to the lowest index."""
    idx = np.argmax(np.real(x), axis=axis)
    return np.take_along_axis(x, np.expand_dims(idx, axis), axis).squeeze(axis)


def cmin_axis(x, axis):
    """Min along ``axis`` by real part; ties go to the lowest index."""
    idx = np.argmin(np.real(x), axis=axis)
    return np.take_along_axis(x, np.expand_dims(idx, axis), axis).squeeze(axis)


# ----------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------

@dataclass
class Physics:
    """Ideal-gas Navier-Stokes parameters (eqs. (2.1) and (3.1)).

    The paper writes every viscous term with a factor 1/Re and a constant
    dynamic viscosity.  Here that factor is the viscosity law
    ``mu(T) = mu_ref * (T / T_ref) ** mu_exp`` with the temperature
    ``T = p / rho``; ``mu_exp = 0`` (the default) is the paper's constant
    viscosity, ``mu_ref = 1/Re``.
    """

    gamma: float = 1.4
    Pr: float = 0.72
    mu_ref: float = 0.01
    mu_exp: float = 0.0
    T_ref: float = 1.0

    def mu(self, rho, p):
        if self.mu_exp == 0.0:
            return self.mu_ref
        T = p / rho
        return self.mu_ref * (T / self.T_ref) ** self.mu_exp


@dataclass
class Options:
    """Scheme constants (Sec. 5 preamble and Appendix A)."""

    cfl: float = 0.6            #: CFL number (0.3 for Example 5.12)
    b_visc: float = 0.001       #: viscous time-step constant b (<= 0 or inf: no bound)
    eps_pp: float = 1e-12       #: positivity-limiter floor
    eps_weno: float = 1e-8      #: epsilon of the nonlinear weights
    t_final: float = math.inf   #: last step is clipped to reach t_final
    linear_weights: bool = False  #: test mode: omega = gamma (no nonlinearity)
    #: Remark 3.1 ablation: omega = gamma in the gradient reconstruction only
    linear_gradients: bool = False
    #: viscous gradients: 'GR' (weak-derivative moments reconstructed, Sec. 2.2
    #: and 3.2) or 'DR' (the comparison scheme: derivatives of the convective
    #: reconstruction with its weights reused, eqs. (2.5) and (3.5))
    gradients: str = 'GR'
    max_halvings: int = 64      #: restarts allowed per step before giving up
    #: linear weights gamma_m (1D: eq. (A.3); 2D: eq. (A.6))
    gamma1d: tuple = field(default=(199.0 / 200.0, 1.0 / 400.0, 1.0 / 400.0))
    gamma2d: tuple = field(default=(99.0 / 100.0, 1.0 / 400.0, 1.0 / 400.0,
                                    1.0 / 400.0, 1.0 / 400.0))


# ----------------------------------------------------------------------------
# Gas physics
# ----------------------------------------------------------------------------

def pressure(U, gamma):
    """p = (gamma-1) * rho * e with e = E/rho - |u|^2/2, for U[c, ...]."""
    rho = U[0]
    E = U[-1]
    kin = 0.0
    for c in range(1, U.shape[0] - 1):
        kin = kin + U[c] * U[c]
    return (gamma - 1.0) * (E - 0.5 * kin / rho)


def sound_speed(rho, p, gamma):
    return np.sqrt(gamma * p / rho)


def primitives(U):
    """Velocity components and specific internal energy e (Sec. 2.1, 3.1).

    Returns a list ``[u, (v,) e]`` -- the dissipative variables w whose
    derivatives feed the viscous fluxes.
    """
    rho = U[0]
    vel = [U[c] / rho for c in range(1, U.shape[0] - 1)]
    kin = 0.0
    for v in vel:
        kin = kin + v * v
    e = U[-1] / rho - 0.5 * kin
    return vel + [e]


def flux1d(U, ux, ex, phys):
    """Total flux f = f^a - f^d of eq. (2.1) at points, U[c, ...].

    tau = (4/3) mu u_x,  q = -gamma mu e_x / Pr  (mu = 1/Re for mu_exp = 0).
    """
    rho, m, E = U[0], U[1], U[2]
    u = m / rho
    p = pressure(U, phys.gamma)
    mu = phys.mu(rho, p)
    tau = (4.0 / 3.0) * mu * ux
    q = -phys.gamma * mu * ex / phys.Pr
    return np.stack([m, m * u + p - tau, (E + p) * u - (tau * u - q)])


def beta_pp1d(U, ux, ex, phys):
    """Positivity wave-speed bound of eq. (2.3) (the bracket under the max)."""
    rho, m = U[0], U[1]
    u = m / rho
    p = pressure(U, phys.gamma)
    e = p / ((phys.gamma - 1.0) * rho)
    mu = phys.mu(rho, p)
    tau = (4.0 / 3.0) * mu * ux
    q = -phys.gamma * mu * ex / phys.Pr
    r2e = rho * rho * e
    root = np.sqrt(rho * rho * q * q + 2.0 * r2e * (tau - p) ** 2)
    return cabs(u) + (root + rho * cabs(q)) / (2.0 * r2e)


def stresses2d(s, mu):
    """(tau_xx, tau_xy, tau_yy) / Re of Sec. 3.1, s = (u_x,u_y,v_x,v_y,e_x,e_y)."""
    ux, uy, vx, vy = s[0], s[1], s[2], s[3]
    txx = mu * (4.0 / 3.0 * ux - 2.0 / 3.0 * vy)
    txy = mu * (uy + vx)
    tyy = mu * (4.0 / 3.0 * vy - 2.0 / 3.0 * ux)
    return txx, txy, tyy


def flux2d(U, s, phys, direction):
    """Total flux f (direction 0) or g (direction 1) of eq. (3.1) at points."""
    rho, m, n, E = U[0], U[1], U[2], U[3]
    u = m / rho
    v = n / rho
    p = pressure(U, phys.gamma)
    mu = phys.mu(rho, p)
    txx, txy, tyy = stresses2d(s, mu)
    kq = phys.gamma * mu / phys.Pr
    if direction == 0:
        return np.stack([m, m * u + p - txx, n * u - txy,
                         (E + p) * u - (txx * u + txy * v + kq * s[4])])
    return np.stack([n, m * v - txy, n * v + p - tyy,
                     (E + p) * v - (txy * u + tyy * v + kq * s[5])])


def beta_pp2d(U, s, phys, direction):
    """Positivity wave-speed bounds of eq. (3.3) (the brackets under the max)."""
    rho, m, n = U[0], U[1], U[2]
    p = pressure(U, phys.gamma)
    e = p / ((phys.gamma - 1.0) * rho)
    mu = phys.mu(rho, p)
    txx, txy, tyy = stresses2d(s, mu)
    kq = phys.gamma * mu / phys.Pr
    if direction == 0:
        un = m / rho
        q = kq * s[4]
        t2 = (txx - p) ** 2 + txy ** 2
    else:
        un = n / rho
        q = kq * s[5]
        t2 = txy ** 2 + (tyy - p) ** 2
    r2e = rho * rho * e
    root = np.sqrt(rho * rho * q * q + 2.0 * r2e * t2)
    return cabs(un) + (root + rho * cabs(q)) / (2.0 * r2e)


# ----------------------------------------------------------------------------
# Characteristic bases (Sec. 2.1 and 3.1): right eigenvectors of the
# convective-flux Jacobian at a state; the left ones are the matrix inverse.
# ----------------------------------------------------------------------------

def right_eigvecs1d(Ubar, gamma):
    """R(ubar)[c, k, ...] with columns (1,u-c,H-uc), (1,u,u^2/2), (1,u+c,H+uc)."""
    rho, m, E = Ubar[0], Ubar[1], Ubar[2]
    u = m / rho
    p = pressure(Ubar, gamma)
    c = sound_speed(rho, p, gamma)
    H = (E + p) / rho
    one = np.ones_like(u)
    R = np.stack([
        np.stack([one, one, one]),
        np.stack([u - c, u, u + c]),
        np.stack([H - u * c, 0.5 * u * u, H + u * c]),
    ])
    return R


def right_eigvecs2d(Ubar, gamma, direction):
    """R(ubar)[c, k, ...] of the x- (direction 0) or y-Jacobian (direction 1).

    x: columns (1,u-c,v,H-uc), (1,u,v,q2/2), (0,0,1,v), (1,u+c,v,H+uc);
    y: the same with the roles of u and v exchanged.
    """
    rho, m, n, E = Ubar[0], Ubar[1], Ubar[2], Ubar[3]
    u = m / rho
    v = n / rho
    p = pressure(Ubar, gamma)
    c = sound_speed(rho, p, gamma)
    H = (E + p) / rho
    q2 = u * u + v * v
    one = np.ones_like(u)
    zero = np.zeros_like(u)
    if direction == 0:
        R = np.stack([
            np.stack([one, one, zero, one]),
            np.stack([u - c, u, zero, u + c]),
            np.stack([v, v, one, v]),
            np.stack([H - u * c, 0.5 * q2, v, H + u * c]),
        ])
    else:
        R = np.stack([
            np.stack([one, one, zero, one]),
            np.stack([u, u, one, u]),
            np.stack([v - c, v, zero, v + c]),
            np.stack([H - v * c, 0.5 * q2, u, H + v * c]),
        ])
    return R


def invert_cells(R):
    """Left eigenvectors L = R^{-1} per cell, for R[c, k, ...]."""
    nc = R.shape[0]
    Rm = np.moveaxis(R.reshape(nc, nc, -1), -1, 0)   # (ncell, c, k)
    Lm = np.linalg.inv(Rm)                           # (ncell, k, c)
    return np.moveaxis(Lm, 0, -1).reshape(R.shape)
