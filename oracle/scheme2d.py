"""2D HWENO-GR semi-discrete residual (Sec. 3) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Order of one residual evaluation (flowchart of Sec. 4):

1. ghost cells of width 4 (Remark 4.1), x sweep on interior rows first, then
   the y sweep on every column (so corners compose both rules);
2. characteristic-wise HWENO reconstruction (eq. (3.4)) in two bases per cell
   (reading of "the relevant convective-flux Jacobian", Sec. 3.1):
   the x-Jacobian at the cell average gives the x-face traces, the nine
   volume values that feed f and the x weak moments, and hat-v; the
   y-Jacobian gives the y-face traces, the volume values that feed g and the
   y weak moments, and hat-w;
3. positivity limiter: checked on the 12 face and both bases' 9 volume
   points, applied to the 12 face values only (Sec. 3.1);
4. face moments and weak-derivative moments (eqs. (3.6)-(3.8)) from the
   limited face traces and the unlimited volume values;
5. gradient reconstruction, componentwise, same routine (eq. (3.9)), at the
   12 face and 9 volume points (with ``Options.gradients = 'DR'`` steps 4-5
   are the comparison scheme's derivatives of the convective reconstruction,
   eq. (3.5), each basis serving its own points and fluxes);
6. PP local Lax-Friedrichs fluxes at the face Gauss points (eq. (3.3)) and
   the volume fluxes;
7. the residual F^1, F^2, F^3 of eq. (3.2).
"""

import numpy as np

from .common import (GAUSS3_NODES, GAUSS3_WEIGHTS, Options, Physics, cabs, cmax,
                     cmax_axis, flux2d, beta_pp2d, invert_cells, pressure,
                     primitives, right_eigvecs2d, sound_speed)
from .recon import Hweno2D
from .scheme1d import pp_limit

HALO = 4
SLIP_X = np.array([1.0, -1.0, 1.0, 1.0])    # wall normal to x: u odd
SLIP_Y = np.array([1.0, 1.0, -1.0, 1.0])    # wall normal to y: v odd
NOSLIP = np.array([1.0, -1.0, -1.0, 1.0])   # adiabatic no-slip: u, v odd

G3, W3 = GAUSS3_NODES, GAUSS3_WEIGHTS
# scaled point sets of one cell
XFACE = [(-0.5, G3[g]) for g in range(3)] + [(0.5, G3[g]) for g in range(3)]
YFACE = [(G3[g], -0.5) for g in range(3)] + [(G3[g], 0.5) for g in range(3)]
VOL = [(G3[g], G3[h]) for h in range(3) for g in range(3)]   # index 3*h + g
WVOL = np.array([W3[g] * W3[h] for h in range(3) for g in range(3)])


class Scheme2D:
    """Uniform 2D grid, nx x ny cells on [x0,x1] x [y0,y1], halo 4.

    ``bc`` = (xlo, xhi, ylo, yhi) with kinds 'periodic', 'outflow', 'inflow',
    'slip' (reflective / symmetry) or 'noslip' (adiabatic no-slip wall).
    ``inflow`` maps a side index to a conservative state (4,), or to a profile
    (4, n) with one state per boundary cell along the side (n = ny for the x
    sides, bottom to top; n = nx for the y sides, left to right; the y-sweep's
    ghost columns take the end states).  Remark 4.1 prescribes the inflow
    state; Example 5.9 varies it along the boundary.
    """

    def __init__(self, nx, ny, x0, x1, y0, y1, phys=None, opts=None,
                 bc=('periodic',) * 4, inflow=None, solid=None, solid_wall='slip',
                 fixed=None, fixed_state=None):
        self.nx, self.ny = nx, ny
        self.dx = (x1 - x0) / nx
        self.dy = (y1 - y0) / ny
        self.phys = phys or Physics()
        self.opts = opts or Options()
        self.bc = tuple(bc)
        self.inflow = inflow or {}
        self.rec = Hweno2D()
        # masked domain (Examples 5.8, 5.10): solid cells of the grid; the
        # solid cells of `fixed` hold the conservative state `fixed_state`
        # (first moments zero) instead of a mirror image, as the ghost cells
        # of a prescribed-state boundary do (Remark 4.1)
        self.solid = None if solid is None else np.asarray(solid, dtype=bool)
        self.fixed = None if fixed is None else np.asarray(fixed, dtype=bool)
        if self.fixed is not None:
            assert self.solid is not None and not (self.fixed & ~self.solid).any()
        self.fixed_state = None if fixed_state is None else np.asarray(fixed_state)
        self.fixed_cells = []
        self.mirrors = [] if solid is None else self._mirror_map(solid_wall)

    # -- walls inside the grid (masked domains) ------------------------------
    def _mirror_map(self, wall):
        """(dst (j, i), src (j, i), signs (3, 4)) for every solid cell within
        HALO cells (in both directions) of a fluid cell: the mirror image, across
        the nearest wall face along +x, -x, +y, -y (ties in that order), of a
        fluid cell; reflective ('slip') or adiabatic no-slip wall signs as at
        the box walls (Remark 4.1).  A mirror that leaves the grid or lands in
        solid falls back to the first fluid cell in that direction."""
        S = self.solid
        ny, nx = S.shape
        out = []
        for j in range(ny):
            for i in range(nx):
                if not S[j, i]:
                    continue
                win = S[max(j - HALO, 0):j + HALO + 1, max(i - HALO, 0):i + HALO + 1]
                if win.all():
                    continue                      # deep inside the solid
                if self.fixed is not None and self.fixed[j, i]:
                    self.fixed_cells.append((j, i))
                    continue
                best = None
                for dj, di, axis in ((0, 1, 0), (0, -1, 0), (1, 0, 1), (-1, 0, 1)):
                    k = 1
                    while 0 <= j + k * dj < ny and 0 <= i + k * di < nx and S[j + k * dj, i + k * di]:
                        k += 1
                    if not (0 <= j + k * dj < ny and 0 <= i + k * di < nx):
                        continue                  # no fluid this way
                    if best is None or k < best[0]:
                        best = (k, dj, di, axis)
                if best is None:
                    continue                      # fluid only diagonally: left as it is
                k, dj, di, axis = best
                js, is_ = j + (2 * k - 1) * dj, i + (2 * k - 1) * di
                if not (0 <= js < ny and 0 <= is_ < nx) or S[js, is_]:
                    js, is_ = j + k * dj, i + k * di
                if wall == 'noslip':
                    par = NOSLIP
                else:
                    par = SLIP_X if axis == 0 else SLIP_Y
                mom = np.array([1.0, -1.0, 1.0]) if axis == 0 else np.array([1.0, 1.0, -1.0])
                out.append(((j, i), (js, is_), mom[:, None] * par[None, :]))
        return out

    # -- Remark 4.1 ---------------------------------------------------------
    def _fill(self, Ug, side, axis):
        H = HALO
        n = self.nx if axis == 0 else self.ny
        kind = self.bc[2 * axis + side]
        sl = [slice(None)] * 4
        if axis == 0:
            sl[2] = slice(H, H + self.ny)    # x sweep on interior rows only

        def at(idx):
            s = list(sl)
            s[3 - axis] = idx
            return tuple(s)

        for g in range(1, H + 1):
            dst = H - g if side == 0 else H + n - 1 + g
            if kind == 'periodic':
                src = H + n - g if side == 0 else H + g - 1
                Ug[at(dst)] = Ug[at(src)]
            elif kind == 'outflow':
                src = H if side == 0 else H + n - 1
                Ug[at(dst)] = Ug[at(src)]
            elif kind in ('slip', 'noslip'):
                src = H + g - 1 if side == 0 else H + n - g
                s = NOSLIP if kind == 'noslip' else (SLIP_X if axis == 0 else SLIP_Y)
                sgn = np.array([1.0, 1.0, 1.0])
                sgn[1 + axis] = -1.0                  # the normal moment flips
                for m in range(3):
                    Ug[(m,) + at(dst)[1:]] = (sgn[m] * s)[:, None] * Ug[(m,) + at(src)[1:]]
            elif kind == 'inflow':
                st = np.asarray(self.inflow[2 * axis + side])
                if st.ndim == 2:                      # one state per boundary cell
                    val = st if axis == 0 else np.pad(st, ((0, 0), (H, H)), mode='edge')
                else:
                    val = st[:, None]
                Ug[(0,) + at(dst)[1:]] = val
                for m in (1, 2):
                    Ug[(m,) + at(dst)[1:]] = 0.0
            else:
                raise ValueError(kind)

    def ghost(self, U):
        """U[3, 4, ny, nx] -> Ug[3, 4, ny + 8, nx + 8].  Solid cells next to the
        fluid are filled first (from fluid cells), then the box's halo."""
        H = HALO
        Ug = np.zeros(U.shape[:2] + (self.ny + 2 * H, self.nx + 2 * H), dtype=U.dtype)
        Ug[:, :, H:H + self.ny, H:H + self.nx] = U
        for (j, i), (js, is_), sg in self.mirrors:
            Ug[:, :, H + j, H + i] = sg * Ug[:, :, H + js, H + is_]
        for j, i in self.fixed_cells:
            Ug[0, :, H + j, H + i] = self.fixed_state
            Ug[1:, :, H + j, H + i] = 0.0
        for side in (0, 1):
            self._fill(Ug, side, 0)
        for side in (0, 1):
            self._fill(Ug, side, 1)
        return Ug

    # -- Sec. 3 -------------------------------------------------------------
    def reconstruct(self, Ug):
        """Step 2 and 3 on every cell with a full 3x3 stencil.

        Returns dict with (limited) 'xface', 'yface' [6, 4, ...], unlimited
        'xvol', 'yvol' [9, 4, ...], 'vhat' [2, 4, ...] (xi-, eta-moment),
        'theta1', 'theta2', 'ubar'.
        """
        ph, op, rec = self.phys, self.opts, self.rec
        g = ph.gamma
        NY, NX = Ug.shape[2], Ug.shape[3]

        def cell(m, k):
            dx, dy = Hweno2D.CELL_OFF[k]
            return Ug[m][:, 1 + dy:NY - 1 + dy, 1 + dx:NX - 1 + dx]

        stencil = np.stack([cell(0, k) for k in range(1, 10)] +
                           [cell(1, k) for k in Hweno2D.EDGE] +
                           [cell(2, k) for k in Hweno2D.EDGE])     # (17, c, ...)
        ubar = cell(0, 5)
        out = {'ubar': ubar}
        pts_sets = {0: XFACE, 1: YFACE}
        for b in (0, 1):
            R = right_eigvecs2d(ubar, g, b)
            L = invert_cells(R)
            a = np.einsum('kc...,sc...->sk...', L, stencil)
            C = rec.combined(a, op)
            vals = rec.evaluate(C, pts_sets[b] + VOL)              # (15, k, ...)
            U = np.einsum('ck...,pk...->pc...', R, vals)
            mxi, meta = rec.moments(C)
            out['face%d' % b] = U[:6]
            out['vol%d' % b] = U[6:]
            out['mom%d' % b] = np.einsum('ck...,k...->c...', R, mxi if b == 0 else meta)
            if op.gradients == 'DR':
                # eq. (3.5): derivatives of the same combination, back in
                # conservative variables, per unit length
                dxi, deta = rec.derivatives(C, pts_sets[b] + VOL)
                out['d%d' % b] = (np.einsum('ck...,pk...->pc...', R, dxi) / self.dx,
                                  np.einsum('ck...,pk...->pc...', R, deta) / self.dy)
        allpts = np.concatenate([out['face0'], out['face1'], out['vol0'], out['vol1']])
        Ulim, th1, th2 = pp_limit(ubar, allpts, g, op.eps_pp)
        res = dict(xface=Ulim[:6], yface=Ulim[6:12], xvol=out['vol0'], yvol=out['vol1'],
                   vhat=np.stack([out['mom0'], out['mom1']]), theta1=th1, theta2=th2,
                   ubar=ubar)
        if op.gradients == 'DR':
            res['dU'] = (out['d0'], out['d1'])
        return res

    def residual(self, U, source=None):
        """Semi-discrete residual of eq. (3.2) and the modified moments.

        Returns ``(F, Vhat, diag)`` with F[3, 4, ny, nx] = (F^1, F^2, F^3),
        Vhat[2, 4, ny, nx] = (hat-v, hat-w) and diag = dict(alpha, beta_max,
        pp_cells).  ``source`` (optional) is added to F.
        """
        return self.residual_ghosted(self.ghost(U), source)

    def residual_ghosted(self, Ug, source=None):
        """The residual of the interior of an already ghosted array (halo 4).

        Lets a window of a large grid be evaluated on its own: the interior of
        ``Ug`` may be any sub-block, its halo the true neighbours.
        """
        ph, op, rec = self.phys, self.opts, self.rec
        g = ph.gamma
        dx, dy = self.dx, self.dy
        ny, nx = Ug.shape[2] - 2 * HALO, Ug.shape[3] - 2 * HALO
        r = self.reconstruct(Ug)             # region c: ghosted index - 1

        # region-c arrays aligned to r1 (the cells whose gradients are
        # reconstructed; region c shrunk by 2)
        def c2r1(A):
            return A[..., 2:-2, 2:-2]

        if op.gradients == 'DR':
            s_xf, s_yf, s_volf, s_volg, s_last = self._dr_gradients(r, c2r1)
            rbar = None
        else:
            s_xf, s_yf, s_volf, s_volg, s_last, rbar = self._gr_gradients(r, dx, dy)
        return self._fluxes(r, c2r1, s_xf, s_yf, s_volf, s_volg, s_last, rbar, source, nx, ny)

    def _dr_gradients(self, r, c2r1):
        """HWENO-DR (eq. (3.5)): the conservative derivatives of each basis's
        reconstruction converted to s = (u_x, u_y, v_x, v_y, e_x, e_y) with the
        point values that enter the flux there: the limited face traces, and
        the (unlimited) volume values of the basis whose flux they feed."""
        def prim_grads(P, dU):
            rho, m, n, E = P[:, 0], P[:, 1], P[:, 2], P[:, 3]
            u, v = m / rho, n / rho
            comp = []
            for D in dU:                         # d/dx, then d/dy
                ul = (D[:, 1] - u * D[:, 0]) / rho
                vl = (D[:, 2] - v * D[:, 0]) / rho
                el = (D[:, 3] - (E / rho) * D[:, 0]) / rho - u * ul - v * vl
                comp.append((ul, vl, el))
            (ux, vx, ex), (uy, vy, ey) = comp
            return np.stack([ux, uy, vx, vy, ex, ey], axis=1)    # (P, 6, ...)
        d0, d1 = r['dU']
        s_xf = c2r1(prim_grads(r['xface'], (d0[0][:6], d0[1][:6])))
        s_yf = c2r1(prim_grads(r['yface'], (d1[0][:6], d1[1][:6])))
        s_volf = c2r1(prim_grads(r['xvol'], (d0[0][6:], d0[1][6:])))
        s_volg = c2r1(prim_grads(r['yvol'], (d1[0][6:], d1[1][6:])))
        return s_xf, s_yf, s_volf, s_volg, np.concatenate([s_xf, s_yf, s_volf])

    def _gr_gradients(self, r, dx, dy):
        """Steps 4-5 of HWENO-GR: weak-derivative moments and their
        reconstruction; gradients at the 12 face and 9 volume points of r1."""
        op, rec = self.opts, self.rec
        # 4. weak-derivative moments (eqs. (3.6)-(3.8)) on region c shrunk by 1
        wxf = np.stack(primitives(np.moveaxis(r['xface'], 0, 1)))   # (3, 6, ...)
        wyf = np.stack(primitives(np.moveaxis(r['yface'], 0, 1)))
        wbx = np.tensordot(np.stack(primitives(np.moveaxis(r['xvol'], 0, 1))), WVOL,
                           axes=([1], [0]))                        # (3, ...)
        wby = np.tensordot(np.stack(primitives(np.moveaxis(r['yvol'], 0, 1))), WVOL,
                           axes=([1], [0]))
        whx = 0.5 * (wxf[:, 3:6, :, :-1] + wxf[:, 0:3, :, 1:])       # (3, G, j, i+1/2)
        why = 0.5 * (wyf[:, 3:6, :-1, :] + wyf[:, 0:3, 1:, :])      # (3, G, j+1/2, i)
        Wx0 = np.tensordot(whx, W3, axes=([1], [0]))
        Wx1 = np.tensordot(whx, W3 * G3, axes=([1], [0]))
        Wy0 = np.tensordot(why, W3, axes=([1], [0]))
        Wy1 = np.tensordot(why, W3 * G3, axes=([1], [0]))
        rx0 = (Wx0[..., 1:] - Wx0[..., :-1]) / dx
        rxx = (0.5 * (Wx0[..., 1:] + Wx0[..., :-1]) - wbx[..., 1:-1]) / dx
        rxy = (Wx1[..., 1:] - Wx1[..., :-1]) / dx
        ry0 = (Wy0[:, 1:, :] - Wy0[:, :-1, :]) / dy
        ryx = (Wy1[:, 1:, :] - Wy1[:, :-1, :]) / dy
        ryy = (0.5 * (Wy0[:, 1:, :] + Wy0[:, :-1, :]) - wby[:, 1:-1, :]) / dy
        # restrict to region r2 = region c shrunk by one in both directions
        rbar = np.stack([np.stack([rx0, rxx, rxy])[:, :, 1:-1, :],
                         np.stack([ry0, ryx, ryy])[:, :, :, 1:-1]])  # (l, mom, w, j, i)

        # 5. gradient reconstruction on region r1 (= r2 shrunk by one)
        J, I = rbar.shape[3], rbar.shape[4]

        def rcell(mom, k):
            ox, oy = Hweno2D.CELL_OFF[k]
            return rbar[:, mom, :, 1 + oy:J - 1 + oy, 1 + ox:I - 1 + ox]   # (l, w, ...)

        ar = np.stack([rcell(0, k) for k in range(1, 10)] +
                      [rcell(1, k) for k in Hweno2D.EDGE] +
                      [rcell(2, k) for k in Hweno2D.EDGE])           # (17, l, w, ...)
        Cg = rec.combined(ar, op, gradient=True)
        gv = rec.evaluate(Cg, XFACE + YFACE + VOL)                    # (21, l, w, ...)
        # s = (u_x, u_y, v_x, v_y, e_x, e_y): index 2*w + l
        s = np.stack([gv[:, l, w] for w in range(3) for l in range(2)], axis=1)  # (21, 6, ...)
        return s[0:6], s[6:12], s[12:21], s[12:21], s, rbar

    def _fluxes(self, r, c2r1, s_xf, s_yf, s_volf, s_volg, s_last, rbar, source, nx, ny):
        """Steps 6-7: fluxes at the face Gauss points, volume fluxes, assembly."""
        ph = self.phys
        g = ph.gamma
        dx, dy = self.dx, self.dy
        xf, yf = c2r1(r['xface']), c2r1(r['yface'])
        xv, yv = c2r1(r['xvol']), c2r1(r['yvol'])

        # 6. x-faces between r1 cells (j, i) and (j, i+1), interior rows
        rows = slice(1, ny + 1)
        cols = slice(1, nx + 1)

        def wave(Uq, sq, d):
            p = pressure(Uq, g)
            un = Uq[1 + d] / Uq[0]
            return cmax(cabs(un) + sound_speed(Uq[0], p, g), beta_pp2d(Uq, sq, ph, d))

        Um = xf[3:6][:, :, rows, :-1]
        Up = xf[0:3][:, :, rows, 1:]
        sm = s_xf[3:6][:, :, rows, :-1]
        sp = s_xf[0:3][:, :, rows, 1:]
        fm = np.stack([flux2d(Um[q], sm[q], ph, 0) for q in range(3)])
        fp = np.stack([flux2d(Up[q], sp[q], ph, 0) for q in range(3)])
        bx = cmax_axis(np.concatenate([np.stack([wave(Um[q], sm[q], 0) for q in range(3)]),
                                       np.stack([wave(Up[q], sp[q], 0) for q in range(3)])]), 0)
        fhat = 0.5 * (fm + fp - bx * (Up - Um))                      # (G, c, ny, nx+1)

        # y-faces between r1 cells (j, i) and (j+1, i), interior columns
        Vm = yf[3:6][:, :, :-1, cols]
        Vp = yf[0:3][:, :, 1:, cols]
        tm = s_yf[3:6][:, :, :-1, cols]
        tp = s_yf[0:3][:, :, 1:, cols]
        gm = np.stack([flux2d(Vm[q], tm[q], ph, 1) for q in range(3)])
        gp = np.stack([flux2d(Vp[q], tp[q], ph, 1) for q in range(3)])
        by = cmax_axis(np.concatenate([np.stack([wave(Vm[q], tm[q], 1) for q in range(3)]),
                                       np.stack([wave(Vp[q], tp[q], 1) for q in range(3)])]), 0)
        ghat = 0.5 * (gm + gp - by * (Vp - Vm))                      # (G, c, ny+1, nx)

        # 7. assembly (eq. (3.2))
        fR, fL = fhat[..., 1:], fhat[..., :-1]
        gT, gB = ghat[:, :, 1:, :], ghat[:, :, :-1, :]

        def gsum(A, wts):
            return np.tensordot(wts, A, axes=([0], [0]))

        fvol = sum(WVOL[q] * flux2d(xv[q][:, rows, cols], s_volf[q][:, rows, cols], ph, 0)
                   for q in range(9))
        gvol = sum(WVOL[q] * flux2d(yv[q][:, rows, cols], s_volg[q][:, rows, cols], ph, 1)
                   for q in range(9))
        F1 = -gsum(fR - fL, W3) / dx - gsum(gT - gB, W3) / dy
        F2 = (-gsum(fL + fR, W3) / (2.0 * dx) - gsum(gT - gB, W3 * G3) / dy + fvol / dx)
        F3 = (-gsum(fR - fL, W3 * G3) / dx - gsum(gB + gT, W3) / (2.0 * dy) + gvol / dy)
        F = np.stack([F1, F2, F3])
        if source is not None:
            F = F + np.stack(source)
        inner = (Ellipsis, slice(3, 3 + ny), slice(3, 3 + nx))
        Vhat = r['vhat'][inner]
        if self.solid is not None and self.solid.shape == (ny, nx):
            F = np.where(self.solid, 0.0, F)            # solid cells carry no residual
            Vhat = np.where(self.solid, 0.0, Vhat)

        # internals kept for the pin tests: gradients s[21 points, 6] of the
        # interior cells (x-face, y-face, volume points), weak moments
        self.last = dict(grads=s_last[..., rows, cols],
                         rbar=None if rbar is None else rbar[..., 2:2 + ny, 2:2 + nx])

        # diagnostics
        fx = r['xface'][inner]
        fy = r['yface'][inner]
        speeds = []
        for P in (fx, fy):
            for q in range(6):
                Uq = np.real(P[q])
                p = pressure(Uq, g)
                c = sound_speed(Uq[0], p, g)
                speeds.append(np.maximum(np.abs(Uq[1] / Uq[0]), np.abs(Uq[2] / Uq[0])) + c)
        alpha = float(np.max(np.max(np.stack(speeds), axis=0)))
        th1 = np.real(r['theta1'][inner[1:]])
        th2 = np.real(r['theta2'][inner[1:]])
        diag = dict(alpha=alpha,
                    beta_max=float(max(np.max(np.real(bx)), np.max(np.real(by)))),
                    pp_cells=int(np.count_nonzero((th1 < 1.0) | (th2 < 1.0))))
        return F, Vhat, diag
