"""Reverse-mode adjoint of the 2D residual against the oracle's complex-step
tangent-linear model (dot-product test) and against finite differences."""

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from oracle.common import Options, Physics  # noqa: E402
from oracle.scheme2d import Scheme2D  # noqa: E402
from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'
H = 1e-30


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


def directions(U, seed):
    rng = np.random.default_rng([2608, 99, seed])
    scale = np.abs(U).reshape(U.shape[0], U.shape[1], -1).max(axis=-1)[..., None, None]
    dU = rng.standard_normal(U.shape) * scale
    Rb = rng.standard_normal(U.shape)
    Vb = rng.standard_normal((8,) + U.shape[2:])
    return dU, Rb, Vb


def dot_test(U, bc, linear=False, extent=(0.0, 1.0, 0.0, 1.0), mu=0.01, seed=0, mu_exp=0.0):
    ny, nx = U.shape[2:]
    s = hweno.Solver(nx, ny, extent=extent, bc=bc, mu_ref=mu, mu_exp=mu_exp,
                     linear_weights=int(linear))
    sc = Scheme2D(nx, ny, *extent, Physics(mu_ref=mu, mu_exp=mu_exp),
                  Options(linear_weights=linear), bc=bc)
    dU, Rb, Vb = directions(U, seed)
    Fc, Vc, dd = sc.residual(U + 1j * H * dU)
    lhs = np.sum(Fc.imag / H * Rb) + np.sum((Vc.imag / H).reshape(8, ny, nx) * Vb)
    Ub, mub = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    # mu: complex step in mu_ref
    sm = Scheme2D(nx, ny, *extent, Physics(mu_ref=mu + 1j * H, mu_exp=mu_exp),
                  Options(linear_weights=linear), bc=bc)
    Fm, _, _ = sm.residual(U.astype(complex))
    mu_ref = np.sum(Fm.imag / H * Rb)
    return lhs, rhs, mu_ref, mub, dd


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize('linear', [False, True])
def test_vjp_dot_product_periodic(linear):
    U = workloads.random_smooth_2d(13, 11, seed=5, noise=1e-3)
    lhs, rhs, mref, mub, _ = dot_test(U, ('periodic',) * 4, linear=linear)
    print('periodic linear=%s: <J du, rb> %.15e  <du, J^T rb> %.15e  rel %.2e; mu %.6e vs %.6e rel %.2e'
          % (linear, lhs, rhs, rel(lhs, rhs), mref, mub, rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10
    assert rel(mref, mub) < 1e-10


@pytest.mark.parametrize('bc', [('noslip', 'noslip', 'noslip', 'slip'),
                                ('outflow', 'slip', 'slip', 'outflow')])
def test_vjp_dot_product_walls(bc):
    U = workloads.random_smooth_2d(12, 10, seed=6, noise=1e-3, extent=(0.0, 1.0, 0.0, 0.5))
    lhs, rhs, mref, mub, _ = dot_test(U, bc, extent=(0.0, 1.0, 0.0, 0.5), mu=1 / 200)
    print('bc %s: rel %.2e mu rel %.2e' % (bc, rel(lhs, rhs), rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10
    assert rel(mref, mub) < 1e-10


@pytest.mark.parametrize('case', ['periodic', 'walls'])
def test_vjp_dot_product_mu_T(case):
    """Temperature-dependent viscosity mu = mu_ref (T / T_ref)^0.76: the
    adjoint carries the viscosity's dependence on the state at every face
    and volume point, and mu-bar is the derivative in mu_ref of the whole
    law."""
    if case == 'periodic':
        U = workloads.random_smooth_2d(13, 11, seed=15, noise=1e-3)
        lhs, rhs, mref, mub, _ = dot_test(U, ('periodic',) * 4, mu=0.02, mu_exp=0.76)
    else:
        U = workloads.random_smooth_2d(12, 10, seed=16, noise=1e-3, extent=(0.0, 1.0, 0.0, 0.5))
        lhs, rhs, mref, mub, _ = dot_test(U, ('noslip', 'noslip', 'noslip', 'slip'),
                                          extent=(0.0, 1.0, 0.0, 0.5), mu=1 / 200, mu_exp=0.76)
    print('mu(T) %s: <J du, rb> %.15e  <du, J^T rb> %.15e  rel %.2e; mu %.6e vs %.6e rel %.2e'
          % (case, lhs, rhs, rel(lhs, rhs), mref, mub, rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10
    assert rel(mref, mub) < 1e-10


def test_vjp_dot_product_limiter_active():
    """A state with near-vacuum cells: the limiter acts in the oracle too."""
    U = workloads.random_smooth_2d(12, 12, seed=7, noise=1e-3)
    U[0, 0, 5:7, 4:8] = 2e-3                    # deep density trough
    U[0, 3, 5:7, 4:8] = 0.5 * (U[0, 1, 5:7, 4:8] ** 2 + U[0, 2, 5:7, 4:8] ** 2) / 2e-3 + 2e-3
    U[1:, :, 5:7, 4:8] = 0.0
    lhs, rhs, mref, mub, dd = dot_test(U, ('periodic',) * 4)
    print('limiter cells %d: rel %.2e mu rel %.2e' % (dd['pp_cells'], rel(lhs, rhs), rel(mref, mub)))
    assert dd['pp_cells'] > 0
    assert rel(lhs, rhs) < 1e-10


def test_vjp_finite_differences_on_gpu():
    """Central differences of the GPU residual along a direction."""
    nx, ny = 16, 14
    U = workloads.random_smooth_2d(nx, ny, seed=8, noise=1e-3)
    s = hweno.Solver(nx, ny, mu_ref=0.01)
    dU, Rb, Vb = directions(U, 3)
    Ub, _ = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    eps = 1e-6
    Rp, Vp, _ = s.residual(to_dev(U + eps * dU))
    Rm, Vm, _ = s.residual(to_dev(U - eps * dU))
    fd = (np.sum((Rp - Rm).cpu().numpy() * Rb) + np.sum((Vp - Vm).cpu().numpy() * Vb)) / (2 * eps)
    print('finite differences: %.12e vs adjoint %.12e rel %.2e' % (fd, rhs, rel(fd, rhs)))
    assert rel(fd, rhs) < 1e-6


def test_vjp_deterministic():
    U = workloads.random_smooth_2d(20, 18, seed=9, noise=1e-3)
    s = hweno.Solver(20, 18, mu_ref=0.01)
    _, Rb, Vb = directions(U, 4)
    a, ma = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    b, mb = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    assert torch.equal(a, b) and ma == mb
