"""Scalar HWENO reconstruction with unified stencils (Appendix A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same routine serves the conservative reconstruction (inputs: projected
cell averages and first-order moments) and the gradient reconstruction
(inputs: weak-derivative moments); only the input array differs (Appendix A
preamble, Sec. 2.2, Sec. 3.3).

Every candidate polynomial is built here from its moment conditions by a
dense linear solve in FP64 on a monomial basis of the scaled coordinates
(xi, eta) of the target cell, with the moment integrals computed by a
Gauss-Legendre rule that is exact for them.  Nothing is tabulated by hand.

Readings where the paper is silent:

* Smoothness indicators (the paper defers them to its reference on unified
  stencils): the Sobolev form in scaled coordinates,
  ``beta = sum_{1 <= |alpha| <= deg p} int_{[-1/2,1/2]^d} (d^alpha p)^2``,
  each multi-index once.  A linear candidate a + b*xi + c*eta gets
  ``beta = b^2 + c^2``.
* The least-squares part of the 2D quartic (Appendix A.2): unweighted least
  squares on the four scaled-moment residuals, subject to the thirteen exact
  conditions, solved through the KKT system.
* Stencil labels in 2D: row-major from (i-1, j-1), so 2 = below, 4 = left,
  6 = right, 8 = above the target cell 5.
"""

import numpy as np

from .common import cabs, gauss_legendre

# ----------------------------------------------------------------------------
# Moment integrals of monomials over a neighbouring cell, in the target cell's
# scaled coordinate.  Cell at offset d covers [d - 1/2, d + 1/2]; its own
# scaled coordinate is s = xi - d.
# ----------------------------------------------------------------------------

_GX, _GW = gauss_legendre(8)   # exact for degree <= 15


def avg_integral(n, d):
    """int_{-1/2}^{1/2} (s + d)^n ds."""
    return float(np.sum(_GW * (_GX + d) ** n))


def mom_integral(n, d):
    """int_{-1/2}^{1/2} (s + d)^n s ds  (first scaled moment over that cell)."""
    return float(np.sum(_GW * (_GX + d) ** n * _GX))


def _weights(beta, gam, eps, tau):
    """Nonlinear weights of eqs. (A.3)/(A.6) from indicators beta[m, ...]."""
    wt = [g * (1.0 + tau / (b + eps)) for g, b in zip(gam, beta)]
    tot = sum(wt)
    return [w / tot for w in wt]


class Hweno1D:
    """1D unified-stencil HWENO (Appendix A.1).

    Input vector per cell (first axis of ``a``)::

        a = [abar0_{i-1}, abar0_i, abar0_{i+1}, abar1_{i-1}, abar1_{i+1}]

    p0 (quartic) satisfies all five conditions exactly (eq. (A.1)); p1 and p2
    are the linear polynomials matching the averages on {i-1, i} and
    {i, i+1} (eq. (A.2)).
    """

    DEG = 4
    NC = 5  # monomials 1, xi, ..., xi^4

    def __init__(self):
        n = np.arange(self.NC)
        M = np.array([[avg_integral(k, -1) for k in n],
                      [avg_integral(k, 0) for k in n],
                      [avg_integral(k, 1) for k in n],
                      [mom_integral(k, -1) for k in n],
                      [mom_integral(k, 1) for k in n]])
        self.Q = [np.linalg.solve(M, np.eye(5))]          # p0: coeffs = Q0 @ a
        for cells in ((-1, 0), (0, 1)):
            A = np.array([[avg_integral(k, d) for k in (0, 1)] for d in cells])
            Ainv = np.linalg.inv(A)
            Qm = np.zeros((self.NC, 5))
            for r, d in enumerate(cells):
                Qm[0:2, d + 1] = Ainv[:, r]               # input index d+1
            self.Q.append(Qm)
        # Sobolev Gram matrix: beta = c^T G c
        x, w = gauss_legendre(6)
        G = np.zeros((self.NC, self.NC))
        for order in range(1, self.DEG + 1):
            E = np.zeros((len(x), self.NC))
            for k in range(order, self.NC):
                coef = np.prod(np.arange(k - order + 1, k + 1))
                E[:, k] = coef * x ** (k - order)
            G += E.T @ (w[:, None] * E)
        self.G = G
        self.own_moment = np.array([mom_integral(k, 0) for k in n])

    def combined(self, a, opts, gradient=False):
        """Coefficients (5, ...) of the nonlinear combination of eq. (2.4)."""
        gam = opts.gamma1d
        c = [np.tensordot(Q, a, axes=1) for Q in self.Q]
        if opts.linear_weights or (gradient and opts.linear_gradients):
            om = list(gam)
        else:
            beta = [np.einsum('k...,kl,l...->...', cm, self.G, cm) for cm in c]
            tau = (0.5 * (cabs(beta[0] - beta[1]) + cabs(beta[0] - beta[2]))) ** 2
            om = _weights(beta, gam, opts.eps_weno, tau)
        C = (om[0] / gam[0]) * c[0]
        for m in (1, 2):
            C = C + (om[m] - om[0] * gam[m] / gam[0]) * c[m]
        return C

    @staticmethod
    def evaluate(C, pts):
        """Values of the polynomial with coefficients C at scaled points."""
        return np.stack([sum(C[k] * (x ** k) for k in range(C.shape[0])) for x in pts])

    @staticmethod
    def derivative(C, pts):
        """d/dxi of the polynomial with coefficients C at scaled points: with C
        the nonlinear combination of eq. (2.4), the combination of the
        candidates' derivatives with the same weights (eq. (2.5))."""
        return np.stack([sum(k * C[k] * (x ** (k - 1)) for k in range(1, C.shape[0]))
                         for x in pts])

    def moment(self, C):
        """Scaled first moment int u xi over the own cell (the hat-v of eq. (2.4))."""
        return np.tensordot(self.own_moment, C, axes=1)


class Hweno2D:
    """2D unified-stencil HWENO (Appendix A.2).

    Input vector per cell (first axis of ``a``), 17 entries::

        a[0:9]   = abar0 of cells 1..9 (row-major from (i-1, j-1))
        a[9:13]  = abar_xi  of cells 2, 4, 6, 8
        a[13:17] = abar_eta of cells 2, 4, 6, 8
    """

    DEG = 4
    MONOS = [(px, py) for tot in range(5) for py in range(tot + 1)
             for px in [tot - py]]                      # 15 monomials
    NC = 15
    CELL_OFF = {k + 1: (k % 3 - 1, k // 3 - 1) for k in range(9)}
    EDGE = (2, 4, 6, 8)

    def _row(self, kind, cell):
        dx, dy = self.CELL_OFF[cell]
        out = []
        for px, py in self.MONOS:
            if kind == 'avg':
                out.append(avg_integral(px, dx) * avg_integral(py, dy))
            elif kind == 'xi':
                out.append(mom_integral(px, dx) * avg_integral(py, dy))
            else:
                out.append(avg_integral(px, dx) * mom_integral(py, dy))
        return out

    @staticmethod
    def input_index(kind, cell):
        if kind == 'avg':
            return cell - 1
        base = 9 if kind == 'xi' else 13
        return base + Hweno2D.EDGE.index(cell)

    def __init__(self):
        nc = self.NC
        exact = [('avg', k) for k in range(1, 10)] + \
                [('xi', 4), ('xi', 6), ('eta', 2), ('eta', 8)]
        lsq = [('xi', 2), ('xi', 8), ('eta', 4), ('eta', 6)]
        A = np.array([self._row(*r) for r in exact])          # 13 x 15
        B = np.array([self._row(*r) for r in lsq])            # 4 x 15
        # KKT of  min |B c - b|^2  s.t.  A c = a
        K = np.zeros((nc + 13, nc + 13))
        K[:nc, :nc] = 2.0 * B.T @ B
        K[:nc, nc:] = A.T
        K[nc:, :nc] = A
        Kinv = np.linalg.inv(K)
        Q0 = np.zeros((nc, 17))
        for r, (kind, cell) in enumerate(lsq):
            Q0[:, self.input_index(kind, cell)] += (Kinv[:nc, :nc] @ (2.0 * B.T))[:, r]
        for r, (kind, cell) in enumerate(exact):
            Q0[:, self.input_index(kind, cell)] += Kinv[:nc, nc + r]
        self.Q = [Q0]
        lin = [self.MONOS.index(m) for m in ((0, 0), (1, 0), (0, 1))]
        for S in ((2, 4, 5), (2, 5, 6), (4, 5, 8), (5, 6, 8)):
            A3 = np.array([[self._row('avg', k)[i] for i in lin] for k in S])
            A3inv = np.linalg.inv(A3)
            Qm = np.zeros((nc, 17))
            for r, k in enumerate(S):
                Qm[lin, self.input_index('avg', k)] = A3inv[:, r]
            self.Q.append(Qm)
        # Sobolev Gram matrix over all multi-indices 1 <= |alpha| <= 4
        x, w = gauss_legendre(6)
        X, Y = np.meshgrid(x, x, indexing='ij')
        W = np.outer(w, w).ravel()
        X, Y = X.ravel(), Y.ravel()
        G = np.zeros((nc, nc))
        for ax in range(self.DEG + 1):
            for ay in range(self.DEG + 1 - ax):
                if ax + ay == 0:
                    continue
                E = np.zeros((len(W), nc))
                for k, (px, py) in enumerate(self.MONOS):
                    if px < ax or py < ay:
                        continue
                    cx = np.prod(np.arange(px - ax + 1, px + 1))
                    cy = np.prod(np.arange(py - ay + 1, py + 1))
                    E[:, k] = cx * cy * X ** (px - ax) * Y ** (py - ay)
                G += E.T @ (W[:, None] * E)
        self.G = G
        self.mom_xi = np.array(self._row('xi', 5))
        self.mom_eta = np.array(self._row('eta', 5))

    def combined(self, a, opts, gradient=False):
        """Coefficients (15, ...) of the nonlinear combination of eq. (3.4)."""
        gam = opts.gamma2d
        c = [np.tensordot(Q, a, axes=1) for Q in self.Q]
        if opts.linear_weights or (gradient and opts.linear_gradients):
            om = list(gam)
        else:
            beta = [np.einsum('k...,kl,l...->...', cm, self.G, cm) for cm in c]
            tau = (0.25 * sum(cabs(beta[0] - beta[s]) for s in range(1, 5))) ** 2
            om = _weights(beta, gam, opts.eps_weno, tau)
        C = (om[0] / gam[0]) * c[0]
        for m in range(1, 5):
            C = C + (om[m] - om[0] * gam[m] / gam[0]) * c[m]
        return C

    def evaluate(self, C, pts):
        """Values at scaled points pts = [(xi, eta), ...] -> (npts, ...)."""
        out = []
        for (x, y) in pts:
            acc = 0.0
            for k, (px, py) in enumerate(self.MONOS):
                acc = acc + C[k] * (x ** px) * (y ** py)
            out.append(acc)
        return np.stack(out)

    def derivatives(self, C, pts):
        """(d/dxi, d/deta) at scaled points pts = [(xi, eta), ...], each
        (npts, ...): for the nonlinear combination C of eq. (3.4), the
        derivatives of eq. (3.5) (candidates differentiated, weights reused)."""
        dxi, deta = [], []
        for (x, y) in pts:
            ax = 0.0
            ay = 0.0
            for k, (px, py) in enumerate(self.MONOS):
                if px:
                    ax = ax + C[k] * px * (x ** (px - 1)) * (y ** py)
                if py:
                    ay = ay + C[k] * py * (x ** px) * (y ** (py - 1))
            dxi.append(ax)
            deta.append(ay)
        return np.stack(dxi), np.stack(deta)

    def moments(self, C):
        """Scaled first moments (int u xi, int u eta) over the own cell."""
        return (np.tensordot(self.mom_xi, C, axes=1),
                np.tensordot(self.mom_eta, C, axes=1))
