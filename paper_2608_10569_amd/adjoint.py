"""Differentiable SSP-RK3 rollouts on the HIP path.

``HwenoStep`` is a torch.autograd.Function whose forward is one
``hweno_rk_step`` with a fixed step and whose backward is one
``hweno_rk_step_vjp`` (the reverse mode of the three stages of eq. (2.12),
the step size held constant).  ``rollout`` advances ``nsteps`` steps and keeps
only every ``every``-th state; its backward recomputes each segment from its
checkpoint and runs the step adjoints in reverse.  All arithmetic of the
scheme and of its adjoint runs in the library's kernels; this module only
orders the calls.

The remaining helpers define the differentiable double-shear-layer
experiment: the initial state as the 6x6-point Gauss projection of the
primitive fields rho, u, v (p fixed) given at the quadrature nodes of every
cell, and the kinetic energy functional J = 1/2 sum dx dy |m|^2 / rho of the
final cell averages.
"""

import numpy as np
import torch

from . import hweno


def _check_mu(solver, mu):
    if mu is not None and abs(float(mu) - solver.mu_ref) > 1e-15 * max(1.0, solver.mu_ref):
        raise ValueError('mu = %r differs from the solver viscosity %r' % (float(mu), solver.mu_ref))


def _step(solver, dt):
    d = solver.rk_step(dt)
    if d['restarts']:
        raise hweno.HwenoError(4, 'a stage with the fixed step dt = %g was inadmissible' % dt)
    return d


class HwenoStep(torch.autograd.Function):
    """U_{n+1} = step(U_n; mu) for a fixed dt.  Usage:
    ``HwenoStep.apply(U, mu, solver, dt)`` with ``mu`` a 0-d float64 tensor
    equal to the solver's viscosity (its gradient is d/d mu_ref)."""

    @staticmethod
    def forward(ctx, U, mu, solver, dt):
        _check_mu(solver, mu)
        U = U.detach().contiguous()
        solver.set_state(U)
        _step(solver, dt)
        Un, _ = solver.get_state()
        ctx.solver, ctx.dt = solver, float(dt)
        ctx.save_for_backward(U)
        return Un

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        want_mu = ctx.needs_input_grad[1]
        Ub, mub = ctx.solver.rk_step_vjp(U, ctx.dt, gU.contiguous(), want_mu=want_mu)
        gmu = torch.tensor(mub, dtype=torch.float64, device=U.device) if want_mu else None
        return Ub, gmu, None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, mu, solver, dt, nsteps, every):
        _check_mu(solver, mu)
        U = U0.detach().contiguous()
        solver.set_state(U)
        cps = [U]
        for n in range(nsteps):
            _step(solver, dt)
            if (n + 1) % every == 0 and n + 1 < nsteps:
                cps.append(solver.get_state()[0])
        Un, _ = solver.get_state()
        ctx.solver, ctx.dt, ctx.nsteps, ctx.every = solver, float(dt), nsteps, every
        ctx.save_for_backward(*cps)
        return Un

    @staticmethod
    def backward(ctx, gU):
        cps = ctx.saved_tensors
        s, dt, every = ctx.solver, ctx.dt, ctx.every
        want_mu = ctx.needs_input_grad[1]
        g = gU.contiguous()
        mu_bar = 0.0
        record = getattr(s, 'record_slots', 0) >= every
        if record:
            return _Rollout._backward_recorded(ctx, cps, g, want_mu)
        for seg in reversed(range(len(cps))):
            start = seg * every
            stop = min(ctx.nsteps, start + every)
            states = [cps[seg]]
            s.set_state(cps[seg])
            for _ in range(start, stop - 1):     # recompute the segment
                _step(s, dt)
                states.append(s.get_state()[0])
            for U in reversed(states):
                g, mub = s.rk_step_vjp(U, dt, g, want_mu=want_mu)
                if want_mu:
                    mu_bar += mub
        gmu = torch.tensor(mu_bar, dtype=torch.float64, device=g.device) if want_mu else None
        return g, gmu, None, None, None, None

    @staticmethod
    def _backward_recorded(ctx, cps, g, want_mu):
        """Each segment is recomputed once more with every step recorded, and
        the step adjoints start from the recordings.  With two banks of
        ``every`` slots the recording of the segment before runs on a second
        stream while the current segment's adjoints run: bank seg % 2 holds
        segment seg, and a bank is recorded again only after the adjoints
        that read it (the second stream waits for everything the main
        stream has queued)."""
        s, dt, every, nsteps = ctx.solver, ctx.dt, ctx.every, ctx.nsteps
        main = torch.cuda.current_stream(g.device)
        overlap = s.record_slots >= 2 * every
        side = torch.cuda.Stream(g.device) if overlap else main

        def bank(seg):
            return (seg % 2) * every if overlap else 0

        def record(seg):
            start = seg * every
            stop = min(nsteps, start + every)
            side.wait_stream(main)
            try:
                with torch.cuda.stream(side):
                    s.set_stream(side.cuda_stream)
                    U = cps[seg]
                    for k in range(stop - start):
                        U = s.rk_step_record(bank(seg) + k, U, dt)
                    done = torch.cuda.Event()
                    done.record(side)
            finally:
                s.set_stream(main.cuda_stream)
            return done, stop - start

        s.take_mu_bar()                          # clear the device-side sum
        nseg = len(cps)
        pending = record(nseg - 1)
        for seg in reversed(range(nseg)):
            done, n = pending
            if overlap and seg > 0:
                pending = record(seg - 1)
            main.wait_event(done)
            for k in reversed(range(n)):         # mu-bar summed on the device
                g, _ = s.rk_step_vjp_recorded(bank(seg) + k, g, want_mu=False)
            if not overlap and seg > 0:
                pending = record(seg - 1)
        gmu = None
        if want_mu:
            gmu = torch.tensor(s.take_mu_bar(), dtype=torch.float64, device=g.device)
        return g, gmu, None, None, None, None


def rollout(solver, U0, mu, dt, nsteps, every=20):
    """U after ``nsteps`` fixed steps dt from U0, differentiable in U0 and mu;
    the backward keeps one state per ``every`` steps and recomputes the rest.
    With at least ``every`` recording slots on the solver (``set_record``)
    the recomputation records each step's stage intermediates and the step
    adjoints run from them (no second recomputation; the same step adjoints
    bit for bit); with ``2 every`` slots the recording of the next segment
    overlaps the adjoints of the current one on a second stream (the same
    bits as one bank)."""
    if nsteps < 1 or every < 1:
        raise ValueError('nsteps and every must be positive')
    if mu is None:
        mu = torch.tensor(solver.mu_ref, dtype=torch.float64, device=U0.device)
    return _Rollout.apply(U0, mu, solver, float(dt), int(nsteps), int(every))


# ---------------------------------------------------------------------------
# The double shear layer experiment
# ---------------------------------------------------------------------------
def _gauss6():
    x, w = np.polynomial.legendre.leggauss(6)
    return 0.5 * x, 0.5 * w


def gauss_nodes_2d(nx, ny, extent):
    """Coordinates (X, Y), each [6, 6, ny, nx] (eta node b, xi node a, j, i)."""
    x0, x1, y0, y1 = extent
    g, _ = _gauss6()
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    shape = (6, 6, ny, nx)
    X = np.broadcast_to(xc[None, None, None, :] + g[None, :, None, None] * dx, shape).copy()
    Y = np.broadcast_to(yc[None, None, :, None] + g[:, None, None, None] * dy, shape).copy()
    return X, Y


def project_fields(rho, u, v, p, gamma):
    """Cell averages and scaled first moments (3, 4, ny, nx) of the conserved
    variables from primitive fields at the 6x6 Gauss nodes ([6, 6, ny, nx]
    tensors, p may be a scalar); differentiable."""
    g, w = _gauss6()
    dev = rho.device
    W = torch.tensor(np.outer(w, w), dtype=torch.float64, device=dev)[:, :, None, None]
    XI = torch.tensor(g, dtype=torch.float64, device=dev)[None, :, None, None]
    ETA = torch.tensor(g, dtype=torch.float64, device=dev)[:, None, None, None]
    Q = torch.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
    avg = (W * Q).sum(dim=(1, 2))
    mxi = (W * XI * Q).sum(dim=(1, 2))
    meta = (W * ETA * Q).sum(dim=(1, 2))
    return torch.stack([avg, mxi, meta]).contiguous()


def kinetic_energy(U, dx, dy):
    """J = 1/2 sum dx dy (m^2 + n^2) / rho over the cell averages."""
    a = U[0]
    return 0.5 * dx * dy * ((a[1] ** 2 + a[2] ** 2) / a[0]).sum()


def shear_layer_fields(n=256, gamma=1.4):
    """(rho, u, v, p) of the double shear layer at the Gauss nodes of an n x n
    grid on [0,1]^2 (numpy, [6, 6, n, n]; p scalar)."""
    X, Y = gauss_nodes_2d(n, n, (0.0, 1.0, 0.0, 1.0))
    u = np.where(Y <= 0.5, np.tanh(80.0 * (Y - 0.25)), np.tanh(80.0 * (0.75 - Y)))
    return np.ones_like(X), u, 0.05 * np.sin(2 * np.pi * X), 1.0 / gamma
