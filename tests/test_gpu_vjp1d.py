"""Reverse mode of the 1D residual and RK step (Sec. 2) against the oracle's
complex-step tangent-linear model (dot-product tests), central differences
of the GPU forward, and bitwise determinism."""

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from oracle.common import Options, Physics  # noqa: E402
from oracle.rk import rk3_step  # noqa: E402
from oracle.scheme1d import Scheme1D  # noqa: E402
from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'
H = 1e-30


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _trough(U, lo=20, hi=21):
    """A near-vacuum cell at rest: the limiter acts there (a wider trough is
    handled by the weights alone)."""
    U = U.copy()
    U[0, 0, lo:hi] = 2e-3
    U[0, 1, lo:hi] = 0.0
    U[0, 2, lo:hi] = 2e-3
    U[1, :, lo:hi] = 0.0
    return U


CASES = {
    'periodic': dict(U=lambda: workloads.random_smooth_1d(40, seed=3), bc=('periodic',) * 2,
                     mu=0.01),
    'walls': dict(U=lambda: workloads.random_smooth_1d(36, seed=4), bc=('noslip', 'slip'),
                  mu=0.02),
    'outflow-inflow': dict(U=lambda: workloads.random_smooth_1d(36, seed=5),
                           bc=('inflow', 'outflow'), mu=0.01,
                           inflow={0: (1.1, 0.4, 0.9)}),
    'mu(T)': dict(U=lambda: workloads.random_smooth_1d(40, seed=6), bc=('periodic',) * 2,
                  mu=0.02, mu_exp=0.76),
    'limiter': dict(U=lambda: _trough(workloads.random_smooth_1d(48, seed=7)),
                    bc=('periodic',) * 2, mu=0.01),
}


def _cons(P, gamma=1.4):
    r, u, p = P
    return np.array([r, r * u, p / (gamma - 1.0) + 0.5 * r * u * u])


def _pair(case, **opt):
    c = CASES[case]
    U = c['U']()
    nx = U.shape[-1]
    kw = dict(mu_ref=c['mu'], mu_exp=c.get('mu_exp', 0.0), Pr=0.72)
    inflow = c.get('inflow')
    s = hweno.Solver(nx, extent=(0.0, 1.0), bc=c['bc'], inflow=inflow, **kw, **opt)

    def oracle(mu_ref):
        ph = Physics(mu_ref=mu_ref, mu_exp=kw['mu_exp'], Pr=0.72)
        inf = None if inflow is None else {k: _cons(v) for k, v in inflow.items()}
        return Scheme1D(nx, 0.0, 1.0, ph, Options(**opt), bc=c['bc'], inflow=inf)
    return s, oracle, U, kw['mu_ref']


def _directions(U, seed):
    rng = np.random.default_rng([2608, 98, seed])
    scale = np.abs(U).reshape(2, 3, -1).max(axis=-1)[..., None]
    return (rng.standard_normal(U.shape) * scale, rng.standard_normal(U.shape),
            rng.standard_normal((3, U.shape[-1])))


@pytest.mark.parametrize('case', list(CASES))
def test_vjp1d_dot_product(case):
    s, oracle, U, mu = _pair(case)
    dU, Rb, Vb = _directions(U, 1)
    Fc, Vc, dd = oracle(mu).residual(U + 1j * H * dU)
    lhs = np.sum(Fc.imag / H * Rb) + np.sum((Vc.imag / H).reshape(3, -1) * Vb)
    Ub, mub = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    Fm, _, _ = oracle(mu + 1j * H).residual(U.astype(complex))
    mref = np.sum(Fm.imag / H * Rb)
    print('1D %s (limiter cells %d): <J du, rb> %.15e  <du, J^T rb> %.15e  rel %.2e; mu %.6e vs '
          '%.6e rel %.2e' % (case, dd['pp_cells'], lhs, rhs, rel(lhs, rhs), mref, mub,
                             rel(mref, mub)))
    if case == 'limiter':
        assert dd['pp_cells'] > 0
    assert rel(lhs, rhs) < 1e-10
    assert rel(mref, mub) < 1e-10


def test_vjp1d_without_vbar_and_deterministic():
    s, oracle, U, mu = _pair('walls')
    dU, Rb, _ = _directions(U, 2)
    Fc, _, _ = oracle(mu).residual(U + 1j * H * dU)
    lhs = np.sum(Fc.imag / H * Rb)
    a, ma = s.residual_vjp(to_dev(U), to_dev(Rb))
    b, mb = s.residual_vjp(to_dev(U), to_dev(Rb))
    rhs = np.sum(dU * a.cpu().numpy())
    print('1D without Vbar: rel %.2e' % rel(lhs, rhs))
    assert rel(lhs, rhs) < 1e-10
    assert torch.equal(a, b) and ma == mb


def test_vjp1d_finite_differences_on_gpu():
    """Central differences cross the kinks of the weights (|beta_0 - beta_s|):
    the oracle's own differences of this state miss its exact tangent by
    1e-5 at eps = 1e-6 and by 1e-7 at eps = 1e-7, so eps = 1e-7."""
    s, _, U, _ = _pair('periodic')
    dU, Rb, Vb = _directions(U, 3)
    Ub, _ = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    eps = 1e-7
    Rp, Vp, _ = s.residual(to_dev(U + eps * dU))
    Rm, Vm, _ = s.residual(to_dev(U - eps * dU))
    fd = (np.sum((Rp - Rm).cpu().numpy() * Rb) + np.sum((Vp - Vm).cpu().numpy() * Vb)) / (2 * eps)
    print('1D finite differences: %.12e vs adjoint %.12e rel %.2e' % (fd, rhs, rel(fd, rhs)))
    assert rel(fd, rhs) < 1e-6


@pytest.mark.parametrize('case', ['periodic', 'walls', 'mu(T)'])
def test_step_vjp1d(case):
    """One SSP-RK3 step with dt fixed (the paper's rule at U0) against the
    oracle's complex-step tangent of its own step, in U0 and in mu_ref."""
    s, oracle, U, mu = _pair(case, cfl=0.3)
    s.set_state(to_dev(U))
    dt = s.rk_step(0.0)['dt']
    rng = np.random.default_rng([2608, 97])
    scale = np.abs(U).reshape(2, 3, -1).max(axis=-1)[..., None]
    dU = rng.standard_normal(U.shape) * scale
    Wb = rng.standard_normal(U.shape)
    U3c, used, info = rk3_step(oracle(mu), U + 1j * H * dU, 0.0, dt)
    assert used == dt and info['restarts'] == 0
    lhs = np.sum(U3c.imag / H * Wb)
    Ub, mub = s.rk_step_vjp(to_dev(U), dt, to_dev(Wb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    U3m, _, _ = rk3_step(oracle(mu + 1j * H), U.astype(complex), 0.0, dt)
    mref = np.sum(U3m.imag / H * Wb)
    print('1D step %s: rel %.2e mu rel %.2e' % (case, rel(lhs, rhs), rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10
    assert rel(mref, mub) < 1e-10
