"""Manufactured solutions of Examples 5.1 (1D) and 5.2 (2D) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The source S is obtained by substituting the exact fields into the
equations (sympy differentiates them); its cell moments, and those of the
exact solution, are computed with a 6-point Gauss-Legendre rule per
direction.  The stage times of SSP-RK3 are t, t + dt, t + dt/2.
"""

import numpy as np
import sympy as sp

from .common import gauss_legendre


def _fields1d(x, t):
    """Example 5.1: rho, velocity, internal energy."""
    rho = 2 + sp.Rational(1, 5) * sp.exp(-t) * sp.sin(2 * sp.pi * x)
    u = 1 + sp.Rational(1, 5) * sp.exp(-t) * sp.cos(2 * sp.pi * x)
    e = 1 + sp.Rational(1, 5) * sp.exp(-t) * sp.sin(2 * sp.pi * x)
    return rho, u, e


def _fields2d(x, y, t):
    """Example 5.2: rho, velocities, internal energy (mixed-direction modes)."""
    a = sp.Rational(1, 10) * sp.exp(-t)
    tp = 2 * sp.pi
    rho = 2 + a * (sp.sin(tp * (2 * x - y)) + sp.cos(tp * (-x + 2 * y)))
    u = 1 + a * (sp.sin(tp * (-x + y)) + sp.cos(tp * (x + y)))
    v = 2 + a * (sp.sin(tp * (x + y)) + sp.cos(tp * (x - y)))
    e = 2 + a * (sp.sin(tp * (x - y)) + sp.cos(tp * (x + y)))
    return rho, u, v, e


class MMS1D:
    """Source and exact moments of Example 5.1 on a Scheme1D grid."""

    def __init__(self, scheme):
        ph = scheme.phys
        assert ph.mu_exp == 0.0
        x, t = sp.symbols('x t', real=True)
        rho, u, e = _fields1d(x, t)
        g = sp.nsimplify(ph.gamma)
        p = (g - 1) * rho * e
        E = rho * (e + u * u / 2)
        mu = sp.nsimplify(ph.mu_ref)
        tau = sp.Rational(4, 3) * mu * sp.diff(u, x)
        q = -g * mu * sp.diff(e, x) / sp.nsimplify(ph.Pr)
        Uc = [rho, rho * u, E]
        f = [rho * u, rho * u * u + p - tau, (E + p) * u - (tau * u - q)]
        S = [sp.diff(Uc[c], t) + sp.diff(f[c], x) for c in range(3)]
        self.symbols, self.source_expr, self.state_expr = (x, t), S, Uc
        self._S = sp.lambdify((x, t), S, 'numpy')
        self._U = sp.lambdify((x, t), Uc, 'numpy')
        self._Ut = sp.lambdify((x, t), [sp.diff(q, t) for q in Uc], 'numpy')
        gx, gw = gauss_legendre(6)
        xc = scheme.x0 + (np.arange(scheme.nx) + 0.5) * scheme.dx
        self.X = xc[None, :] + gx[:, None] * scheme.dx           # (6, nx)
        self.gw, self.gx = gw, gx

    def _moments(self, fn, t):
        vals = np.array([np.broadcast_to(v, self.X.shape) for v in fn(self.X, t)])
        avg = np.tensordot(self.gw, vals, axes=([0], [1]))
        mom = np.tensordot(self.gw * self.gx, vals, axes=([0], [1]))
        return avg, mom

    def exact(self, t):
        a, m = self._moments(self._U, t)
        return np.stack([a, m])

    def exact_dt(self, t):
        """Time derivative of the exact cell moments."""
        return np.stack(self._moments(self._Ut, t))

    def source(self, t):
        return self._moments(self._S, t)


class MMS2D:
    """Source and exact moments of Example 5.2 on a Scheme2D grid."""

    def __init__(self, scheme, x0=0.0, y0=0.0):
        ph = scheme.phys
        assert ph.mu_exp == 0.0
        x, y, t = sp.symbols('x y t', real=True)
        rho, u, v, e = _fields2d(x, y, t)
        g = sp.nsimplify(ph.gamma)
        Pr = sp.nsimplify(ph.Pr)
        mu = sp.nsimplify(ph.mu_ref)
        p = (g - 1) * rho * e
        E = rho * (e + (u * u + v * v) / 2)
        ux, uy, vx, vy = sp.diff(u, x), sp.diff(u, y), sp.diff(v, x), sp.diff(v, y)
        txx = mu * (sp.Rational(4, 3) * ux - sp.Rational(2, 3) * vy)
        txy = mu * (uy + vx)
        tyy = mu * (sp.Rational(4, 3) * vy - sp.Rational(2, 3) * ux)
        Uc = [rho, rho * u, rho * v, E]
        f = [rho * u, rho * u * u + p - txx, rho * u * v - txy,
             (E + p) * u - (txx * u + txy * v + g * mu * sp.diff(e, x) / Pr)]
        gg = [rho * v, rho * u * v - txy, rho * v * v + p - tyy,
              (E + p) * v - (txy * u + tyy * v + g * mu * sp.diff(e, y) / Pr)]
        S = [sp.diff(Uc[c], t) + sp.diff(f[c], x) + sp.diff(gg[c], y) for c in range(4)]
        self.symbols, self.source_expr, self.state_expr = (x, y, t), S, Uc
        self._S = sp.lambdify((x, y, t), S, 'numpy')
        self._U = sp.lambdify((x, y, t), Uc, 'numpy')
        self._Ut = sp.lambdify((x, y, t), [sp.diff(q, t) for q in Uc], 'numpy')
        gx, gw = gauss_legendre(6)
        xc = x0 + (np.arange(scheme.nx) + 0.5) * scheme.dx
        yc = y0 + (np.arange(scheme.ny) + 0.5) * scheme.dy
        # points (6 eta, 6 xi, ny, nx)
        X = xc[None, None, None, :] + gx[None, :, None, None] * scheme.dx
        Y = yc[None, None, :, None] + gx[:, None, None, None] * scheme.dy
        self.X, self.Y = (np.ascontiguousarray(A) for A in np.broadcast_arrays(X, Y))
        self.gx, self.gw = gx, gw

    def _moments(self, fn, t):
        vals = np.array([np.broadcast_to(v, self.X.shape) for v in fn(self.X, self.Y, t)])
        w2 = np.outer(self.gw, self.gw)                              # (eta, xi)
        avg = np.einsum('ab,cabji->cji', w2, vals)
        mxi = np.einsum('ab,cabji->cji', w2 * self.gx[None, :], vals)
        meta = np.einsum('ab,cabji->cji', w2 * self.gx[:, None], vals)
        return avg, mxi, meta

    def exact(self, t):
        return np.stack(self._moments(self._U, t))

    def exact_dt(self, t):
        """Time derivative of the exact cell moments."""
        return np.stack(self._moments(self._Ut, t))

    def source(self, t):
        return self._moments(self._S, t)
