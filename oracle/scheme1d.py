"""1D HWENO-GR semi-discrete residual (Sec. 2) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One call of :meth:`Scheme1D.residual` performs, in the paper's order
(flowchart of Sec. 4):

1. ghost cells of width 4 (Remark 4.1);
2. characteristic-wise HWENO reconstruction in every cell with a full
   stencil (Sec. 2.1, eq. (2.4)): point values at the four LGL points and the
   modified moment hat-v;
3. positivity limiter on the four LGL values (Sec. 2.1, last paragraph before
   the HWENO-DR description);
4. interface averages and weak-derivative moments (eqs. (2.6)-(2.8));
5. gradient reconstruction with the same scalar routine (eq. (2.9)); with
   ``Options.gradients = 'DR'`` steps 4-5 are replaced by the comparison
   scheme's derivatives of the convective reconstruction (eq. (2.5));
6. PP local Lax-Friedrichs fluxes (eq. (2.3)) and the volume term;
7. the residual F^1, F^2 of eq. (2.2).
"""

import numpy as np

from .common import (LGL_NODES, LGL_WEIGHTS, Options, Physics, cabs, cmax,
                     cmax_axis, cmin, cmin_axis, flux1d, beta_pp1d, invert_cells,
                     pressure, primitives, right_eigvecs1d, sound_speed)
from .recon import Hweno1D

HALO = 4
PARITY1D = np.array([1.0, -1.0, 1.0])   # rho even, m odd, E even at a wall


def pp_limit(Ubar, Upts, gamma, eps_pp):
    """Zhang-Shu scaling of point values about the cell average.

    Ubar[c, ...], Upts[p, c, ...].  Returns (limited points, theta1, theta2).
    eps = min(eps_pp, rhobar, p(ubar)).  theta1 keeps the point densities >=
    eps; theta2 keeps the point pressures >= eps, using the concavity of the
    pressure (linear interpolation bound) in place of the exact root.
    """
    rbar = Ubar[0]
    pbar = pressure(Ubar, gamma)
    eps = cmin(cmin(np.full_like(rbar, eps_pp), rbar), pbar)
    rmin = cmin_axis(Upts[:, 0], 0)
    low = np.real(rmin) < np.real(eps)
    den1 = np.where(low, rbar - rmin, 1.0)
    theta1 = np.where(low, (rbar - eps) / den1, 1.0)
    Ut = Upts.copy()
    Ut[:, 0] = rbar + theta1 * (Upts[:, 0] - rbar)
    pt = pressure(np.moveaxis(Ut, 0, 1), gamma)         # (p, ...)
    lowp = np.real(pt) < np.real(eps)
    den2 = np.where(lowp, pbar - pt, 1.0)
    t = np.where(lowp, (pbar - eps) / den2, 1.0)
    theta2 = cmin(cmin_axis(t, 0), np.ones_like(rbar))
    Ul = Ubar + theta2 * (Ut - Ubar)
    return Ul, theta1, theta2


class Scheme1D:
    """Uniform 1D grid on [x0, x1] with nx cells and ghost layers of width 4.

    ``bc`` is a pair of kinds for (left, right): 'periodic', 'outflow',
    'inflow', 'slip' or 'noslip' (both walls make the velocity odd in 1D).
    ``inflow`` maps a side index to a conservative state (rho, m, E).
    """

    def __init__(self, nx, x0, x1, phys=None, opts=None, bc=('periodic', 'periodic'),
                 inflow=None):
        self.nx = nx
        self.x0, self.x1 = x0, x1
        self.dx = (x1 - x0) / nx
        self.phys = phys or Physics()
        self.opts = opts or Options()
        self.bc = tuple(bc)
        self.inflow = inflow or {}
        self.rec = Hweno1D()

    # -- Remark 4.1 ---------------------------------------------------------
    def ghost(self, U):
        """U[2, 3, nx] -> ghosted Ug[2, 3, nx + 8]."""
        nx, H = self.nx, HALO
        Ug = np.zeros(U.shape[:2] + (nx + 2 * H,), dtype=U.dtype)
        Ug[..., H:H + nx] = U
        for side in (0, 1):
            kind = self.bc[side]
            for g in range(1, H + 1):
                dst = H - g if side == 0 else H + nx - 1 + g
                if kind == 'periodic':
                    src = nx - g if side == 0 else g - 1
                    Ug[..., dst] = U[..., src]
                elif kind == 'outflow':
                    src = 0 if side == 0 else nx - 1
                    Ug[..., dst] = U[..., src]
                elif kind in ('slip', 'noslip'):
                    src = g - 1 if side == 0 else nx - g
                    Ug[0, :, dst] = PARITY1D * U[0, :, src]
                    Ug[1, :, dst] = -PARITY1D * U[1, :, src]
                elif kind == 'inflow':
                    Ug[0, :, dst] = self.inflow[side]
                    Ug[1, :, dst] = 0.0
                else:
                    raise ValueError(kind)
        return Ug

    # -- Sec. 2.1 / 2.2 -----------------------------------------------------
    def residual(self, U, source=None):
        """Semi-discrete residual of eq. (2.2) and the modified moment.

        Returns ``(F, Vhat, diag)`` with F[2, 3, nx] = (F^1, F^2),
        Vhat[1, 3, nx] and diag = dict(alpha, beta_max, pp_cells).
        ``source`` (optional) is (Sbar, Sxi) added to (F^1, F^2).
        """
        ph, op, rec = self.phys, self.opts, self.rec
        g = ph.gamma
        dx, nx, H = self.dx, self.nx, HALO
        Ug = self.ghost(U)
        NG = nx + 2 * H

        # 2. characteristic reconstruction in cells 1 .. NG-2
        c = slice(1, NG - 1)
        ubar = Ug[0][:, c]
        R = right_eigvecs1d(ubar, g)                       # (c, k, n)
        L = invert_cells(R)                                # (k, c, n)
        stencil = np.stack([Ug[0][:, 0:NG - 2], Ug[0][:, 1:NG - 1], Ug[0][:, 2:NG],
                            Ug[1][:, 0:NG - 2], Ug[1][:, 2:NG]])   # (5, c, n)
        a = np.einsum('kcn,scn->skn', L, stencil)          # (5, k, n)
        C = rec.combined(a, op)                            # (5, k, n)
        vals = rec.evaluate(C, LGL_NODES)                  # (4, k, n)
        vh = rec.moment(C)                                 # (k, n)
        Upts = np.einsum('ckn,pkn->pcn', R, vals)          # (4, c, n)
        Vhat_all = np.einsum('ckn,kn->cn', R, vh)          # (c, n)

        # 3. positivity limiter on all four LGL values
        Ulim, th1, th2 = pp_limit(ubar, Upts, g, op.eps_pp)

        if op.gradients == 'DR':
            # 4'-5'. HWENO-DR (eq. (2.5)): d/dx of each field's nonlinear
            # combination, weights reused, transformed back to (rho, m, E)_x
            # and converted to (u_x, e_x) with the point values entering the
            # flux there (the limited LGL values)
            dvals = rec.derivative(C, LGL_NODES) / dx          # (4, k, n)
            dU = np.einsum('ckn,pkn->pcn', R, dvals)           # (4, c, n)
            rho, mom, E = Ulim[:, 0], Ulim[:, 1], Ulim[:, 2]
            u = mom / rho
            ux = (dU[:, 1] - u * dU[:, 0]) / rho
            ex = (dU[:, 2] - (E / rho) * dU[:, 0]) / rho - u * ux
            grads = np.stack([ux, ex], axis=1)[:, :, 2:-2]     # cells 3..NG-4
            rb0 = rb1 = None
        else:
            # 4. weak-derivative moments on cells 2 .. NG-3 (indices in region c)
            w_pts = np.stack(primitives(np.moveaxis(Ulim, 0, 1)))   # (2, 4, n)
            wbar = np.tensordot(w_pts, LGL_WEIGHTS, axes=([1], [0]))  # (2, n)
            what = 0.5 * (w_pts[:, 3, :-1] + w_pts[:, 0, 1:])      # faces between n, n+1
            rb0 = (what[:, 1:] - what[:, :-1]) / dx                 # cells 1..n-2 of c
            rb1 = (0.5 * (what[:, 1:] + what[:, :-1]) - wbar[:, 1:-1]) / dx

            # 5. gradient reconstruction on cells 3 .. NG-4
            ar = np.stack([rb0[:, :-2], rb0[:, 1:-1], rb0[:, 2:], rb1[:, :-2], rb1[:, 2:]])
            Cg = rec.combined(ar, op, gradient=True)           # (5, 2, m)
            grads = rec.evaluate(Cg, LGL_NODES)                # (4, 2, m) m: cells 3..NG-4
        # align region-c arrays with gradient cells: c index = ghosted - 1
        Ug_c = Ulim[:, :, 2:-2]                            # (4, c, m)

        # 6. fluxes on faces between gradient-cells m and m+1
        Um, Up = Ug_c[3, :, :-1], Ug_c[0, :, 1:]
        sm, sp = grads[3, :, :-1], grads[0, :, 1:]
        fm = flux1d(Um, sm[0], sm[1], ph)
        fp = flux1d(Up, sp[0], sp[1], ph)

        def speed(Uq, sq):
            p = pressure(Uq, g)
            return cmax(cabs(Uq[1] / Uq[0]) + sound_speed(Uq[0], p, g),
                        beta_pp1d(Uq, sq[0], sq[1], ph))

        beta = cmax(speed(Um, sm), speed(Up, sp))
        fhat = 0.5 * (fm + fp - beta * (Up - Um))           # (c, faces)

        # 7. assembly on interior cells: gradient-cell m = 1 .. nx
        inner = slice(1, nx + 1)
        F1 = -(fhat[:, 1:] - fhat[:, :-1]) / dx
        fvol = sum(LGL_WEIGHTS[q] * flux1d(Ug_c[q], grads[q, 0], grads[q, 1], ph)
                   for q in range(4))
        F2 = -(fhat[:, 1:] + fhat[:, :-1]) / (2.0 * dx) + fvol[:, inner] / dx
        F = np.stack([F1, F2])
        if source is not None:
            F = F + np.stack(source)
        Vhat = Vhat_all[None, :, 3:3 + nx]

        # internals kept for the pin tests: gradients (u_x, e_x) at the LGL
        # points of the interior cells, limited point values, weak moments
        self.last = dict(grads=grads[:, :, inner], points=Ug_c[:, :, inner],
                         rbar=None if rb0 is None else np.stack([rb0, rb1])[:, :, 2:2 + nx])

        # diagnostics: CFL wave speed from interior face traces, PP activity
        Uint = Ulim[:, :, 3:3 + nx]
        cs = []
        for q in (0, 3):
            p = pressure(Uint[q], g)
            cs.append(np.real(np.abs(Uint[q][1] / Uint[q][0]) + sound_speed(Uint[q][0], p, g)))
        alpha = float(np.max(np.maximum(cs[0], cs[1])))
        act = (np.real(th1[3:3 + nx]) < 1.0) | (np.real(th2[3:3 + nx]) < 1.0)
        diag = dict(alpha=alpha, beta_max=float(np.max(np.real(beta))),
                    pp_cells=int(np.count_nonzero(act)))
        return F, Vhat, diag
