"""Fused kernels against the split path: face fluxes formed inside the update
kernel (tiles flux = 0: one kernel per tile of 32 x 8 cells keeps the fluxes
of the tile's faces in LDS, against two face-flux kernels writing HBM, then
the update kernel), and weak moments formed inside the gradient kernel
(tiles grad = 0: per tile of 16 x 4 cells and its ring, in LDS, against the
weak-moment kernel writing HBM, then the gradient kernel).  The tiles change
no result, so the paths must give the same bits: residual, modified moments,
diagnostics and RK steps, on sizes whose last tile is ragged in x, in y or
both, with walls, outflow, a masked domain, source moments and a strong
shock where the positivity limiter acts."""

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'
SPLIT = dict(recon=16, grad=32, flux=64, order=0, xcd=1)
VARIANTS = {'flux': dict(SPLIT, flux=0), 'grad': dict(SPLIT, grad=0),
            'both': dict(SPLIT, grad=0, flux=0)}


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


def pair(nx, ny, variant='both', **kw):
    a = hweno.Solver(nx, ny, **kw)
    b = hweno.Solver(nx, ny, **kw)
    a.set_tiles(**SPLIT)
    b.set_tiles(**VARIANTS[variant])
    assert b.tiles() == VARIANTS[variant]
    return a, b


DIAG_KEYS = ('alpha_star', 'beta_max', 'min_rho', 'min_p', 'pp_cells', 'dt')


@pytest.mark.parametrize('variant', list(VARIANTS))
@pytest.mark.parametrize('shape', [(4, 4), (32, 8), (33, 9), (37, 13), (64, 16), (100, 41)])
@pytest.mark.parametrize('bc', [('periodic',) * 4, ('outflow', 'slip', 'noslip', 'outflow')])
def test_fused_residual_same_bits(shape, bc, variant):
    nx, ny = shape
    print('residual %dx%d %s %s' % (nx, ny, bc[0], variant), flush=True)
    U = to_dev(workloads.random_smooth_2d(nx, ny, seed=nx * 7 + ny, noise=1e-3))
    a, b = pair(nx, ny, variant, mu_ref=0.01, bc=bc)
    Ra, Va, da = a.residual(U)
    Rb, Vb, db = b.residual(U)
    assert torch.equal(Ra, Rb) and torch.equal(Va, Vb)
    for k in ('alpha_star', 'beta_max', 'pp_cells'):
        assert da[k] == db[k], k


def test_fused_steps_same_bits_strong_shock():
    """Viscous shock tube (pressure ratio 100, no-slip walls) with smooth
    perturbations, then the Sedov blast of Example 5.7 through its start,
    where the limiter acts and steps restart."""
    nx, ny = 120, 60
    print('shock tube %dx%d' % (nx, ny), flush=True)
    U = to_dev(workloads.viscous_shock_tube_2d(nx, ny, seed=5, amp=0.02))
    a, b = pair(nx, ny, extent=(0.0, 1.0, 0.0, 0.5), mu_ref=1.0 / 200.0, bc=('noslip',) * 4)
    steps_same_bits(a, b, U, 6)
    n = 40
    print('Sedov %dx%d' % (n, n), flush=True)
    a, b = pair(n, n, extent=(0.0, 1.1, 0.0, 1.1), bc=('slip', 'outflow', 'slip', 'outflow'),
                gamma=1.4, Pr=0.72, mu_ref=1e-4)
    pp, restarts = steps_same_bits(a, b, to_dev(workloads.sedov_2d(n)), 4)
    assert pp > 0 and restarts > 0


def steps_same_bits(a, b, U, nsteps):
    a.set_state(U)
    b.set_state(U)
    pp = restarts = 0
    for _ in range(nsteps):
        da, db = a.rk_step(0.0), b.rk_step(0.0)
        for k in DIAG_KEYS + ('restarts',):
            assert da[k] == db[k], k
        pp += da['pp_cells']
        restarts += da['restarts']
        assert torch.equal(a.get_state()[0], b.get_state()[0])
    return pp, restarts


def test_fused_masked_domain_and_source_same_bits():
    nx, ny = 45, 27
    print('masked %dx%d' % (nx, ny), flush=True)
    U = workloads.random_smooth_2d(nx, ny, seed=77, noise=1e-3)
    solid = np.zeros((ny, nx), bool)
    solid[9:17, 20:31] = True
    bc = ('outflow',) * 4
    a, b = pair(nx, ny, mu_ref=0.01, bc=bc)
    for s in (a, b):
        s.set_solid(solid, 'noslip')
        s.set_state(to_dev(U))
    for _ in range(3):
        da, db = a.rk_step(0.0), b.rk_step(0.0)
        for k in DIAG_KEYS:
            assert da[k] == db[k], k
    assert torch.equal(a.get_state()[0], b.get_state()[0])
    print('source %dx%d' % (nx, ny), flush=True)
    a, b = pair(nx, ny, mu_ref=0.01)
    rng = np.random.default_rng(3)
    src = [to_dev(1e-2 * rng.standard_normal((3, 4, ny, nx))) for _ in range(3)]
    for s in (a, b):
        s.set_state(to_dev(U))
        s.rk_step_source(1e-4, *src)
    assert torch.equal(a.get_state()[0], b.get_state()[0])
