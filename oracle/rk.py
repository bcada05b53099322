"""SSP-RK3 with modified moments, time-step rule and stage restart -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Stage structure (eq. (2.12); the 2D analogue in Sec. 3.1): every stage
combines the cell averages with the *modified* first-order moments hat-v
produced by the reconstruction of that stage's input, and the residual is
evaluated on the stage input itself:

    U1 = B(U^n)                    + dt F(U^n)
    U2 = 3/4 B(U^n) + 1/4 (B(U1)   + dt F(U1))
    U3 = 1/3 B(U^n) + 2/3 (B(U2)   + dt F(U2))

where B(U) = (ubar, hat-v(U)).  Time step (Sec. 5 preamble):
dt_trial = min(CFL h / alpha*, b Re h^2), alpha* from the stage-1 traces, the
last step clipped to t_final.  A stage whose cell averages have nonpositive
density or pressure rejects the step, which is redone from t^n with dt/2.
"""

import math

import numpy as np

from .common import pressure


class InadmissibleError(RuntimeError):
    """More restarts than ``Options.max_halvings`` were needed."""


def admissible(U, gamma, solid=None):
    """All cell averages finite with rho > 0 and p > 0 (strictly); solid cells
    of a masked domain are not checked."""
    Ub = np.real(U[0])
    if solid is not None:
        Ub = Ub[:, ~solid]
        U = U[..., ~solid]
    if not np.all(np.isfinite(np.real(U))):
        return False
    return bool(np.min(Ub[0]) > 0.0 and np.min(pressure(Ub, gamma)) > 0.0)


def _base(U, Vhat):
    return np.concatenate([U[0:1], Vhat], axis=0)


def grid_h(scheme):
    return min(scheme.dx, scheme.dy) if hasattr(scheme, 'dy') else scheme.dx


def trial_dt(scheme, alpha, t, rule='paper'):
    """dt_trial of the Sec. 5 preamble ('paper'), or CFL h^{5/3}/alpha ('h53')."""
    op, ph = scheme.opts, scheme.phys
    h = grid_h(scheme)
    if rule == 'paper':
        dt = op.cfl * h / alpha
        if ph.mu_ref > 0.0 and op.b_visc > 0.0:   # b <= 0 (or inf): no viscous bound
            dt = min(dt, op.b_visc * h * h / ph.mu_ref)
    elif rule == 'h53':
        dt = op.cfl * h ** (5.0 / 3.0) / alpha
    else:
        raise ValueError(rule)
    if math.isfinite(op.t_final):
        dt = min(dt, op.t_final - t)
    return dt


def rk3_step(scheme, U, t, dt=None, rule='paper', source=None, inflow=None):
    """One SSP-RK3 step.  Returns (U_new, dt_used, info).

    ``dt`` fixed, or None for the time-step rule.  ``source(t)`` returns the
    source moments to add to the residual at time t (manufactured solutions).
    ``inflow(t)`` returns {side: inflow state or profile} in force at time t
    (boundary data that vary in time, Example 5.11); each stage's residual
    sees the boundary data of its own time, as it sees the source.
    """
    g = scheme.phys.gamma
    src = (lambda tt: None) if source is None else source
    solid = getattr(scheme, 'solid', None)

    def keep_solid(V):
        """Solid cells of a masked domain keep U^n through the stages."""
        if solid is not None:
            V[..., solid] = U[..., solid]
        return V

    def residual(V, tt):
        if inflow is not None:
            scheme.inflow.update(inflow(tt))
        return scheme.residual(V, src(tt))
    F0, V0, d0 = residual(U, t)
    if dt is None:
        dt = trial_dt(scheme, d0['alpha'], t, rule)
    B0 = _base(U, V0)
    info = dict(alpha=d0['alpha'], beta_max=d0['beta_max'], restarts=0, pp_cells=0)
    while True:
        pp = d0['pp_cells']
        U1 = keep_solid(B0 + dt * F0)
        ok = admissible(U1, g, solid)
        if ok:
            F1, V1, d1 = residual(U1, t + dt)
            U2 = keep_solid(0.75 * B0 + 0.25 * (_base(U1, V1) + dt * F1))
            ok = admissible(U2, g, solid)
            pp += d1['pp_cells']
        if ok:
            F2, V2, d2 = residual(U2, t + 0.5 * dt)
            U3 = keep_solid((1.0 / 3.0) * B0 + (2.0 / 3.0) * (_base(U2, V2) + dt * F2))
            ok = admissible(U3, g, solid)
            pp += d2['pp_cells']
        if ok:
            info['pp_cells'] = pp
            return U3, dt, info
        info['restarts'] += 1
        if info['restarts'] > scheme.opts.max_halvings:
            raise InadmissibleError('stage admissibility failed after %d halvings'
                                    % scheme.opts.max_halvings)
        dt = 0.5 * dt


def run(scheme, U, t0, t1, rule='paper', source=None, dt=None, max_steps=10 ** 7, inflow=None):
    """Advance from t0 to t1 (the last step clipped).  Returns (U, t, nsteps)."""
    scheme.opts.t_final = t1
    t = t0
    n = 0
    while t < t1 - 1e-14 * max(1.0, abs(t1)) and n < max_steps:
        step_dt = None if dt is None else min(dt, t1 - t)
        U, used, _ = rk3_step(scheme, U, t, step_dt, rule, source, inflow)
        t += used
        n += 1
    return U, t, n
