"""Reverse mode on masked grids (walls inside the grid, Remark 4.1 applied to
the solid cells next to the fluid; Examples 5.8 and 5.10): the residual and
RK-step adjoints against the oracle's complex-step tangent of its masked
residual and step (dot-product tests), the step's solid cells against
central differences of the GPU step, and solid cells holding a prescribed
state."""

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from oracle.common import Options, Physics  # noqa: E402
from oracle.rk import rk3_step  # noqa: E402
from oracle.scheme2d import Scheme2D  # noqa: E402
from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'
H = 1e-30
NX, NY = 26, 20


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def masks():
    """A block in a corner (two of its sides on the box) and one away from
    the box's sides (all four wall directions and the block's corners), large
    enough to hold solid cells beyond the mirror band."""
    corner = np.zeros((NY, NX), bool)
    corner[:9, :10] = True
    inner = np.zeros((NY, NX), bool)
    inner[5:16, 6:18] = True
    return {'corner': corner, 'inner': inner}


def mirror_band(solid):
    """Solid cells within 4 cells of a fluid cell (the ones the fill lists)."""
    ny, nx = solid.shape
    out = np.zeros_like(solid)
    for j in range(ny):
        for i in range(nx):
            if solid[j, i]:
                w = solid[max(j - 4, 0):j + 5, max(i - 4, 0):i + 5]
                out[j, i] = not w.all()
    return out


def pair(solid, wall, mu=0.01, bc=('outflow',) * 4):
    s = hweno.Solver(NX, NY, mu_ref=mu, bc=bc)
    s.set_solid(solid, wall)
    sc = Scheme2D(NX, NY, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=mu), Options(), bc=bc, solid=solid,
                  solid_wall=wall)
    return s, sc


@pytest.mark.parametrize('wall', ['slip', 'noslip'])
@pytest.mark.parametrize('block', ['corner', 'inner'])
def test_masked_residual_vjp_dot_product(block, wall):
    solid = masks()[block]
    U = workloads.random_smooth_2d(NX, NY, seed=61, noise=1e-3)
    s, sc = pair(solid, wall)
    rng = np.random.default_rng([2608, 95, int(block == 'inner'), int(wall == 'noslip')])
    scale = np.abs(U).reshape(3, 4, -1).max(axis=-1)[..., None, None]
    dU = rng.standard_normal(U.shape) * scale
    Rb = rng.standard_normal(U.shape)
    Vb = rng.standard_normal((8, NY, NX))
    Fc, Vc, _ = sc.residual(U + 1j * H * dU)
    lhs = np.sum(Fc.imag / H * Rb) + np.sum((Vc.imag / H).reshape(8, NY, NX) * Vb)
    Ub, mub = s.residual_vjp(to_dev(U), to_dev(Rb), to_dev(Vb))
    Ub = Ub.cpu().numpy()
    rhs = np.sum(dU * Ub)
    Fm, _, _ = Scheme2D(NX, NY, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01 + 1j * H), Options(),
                        bc=('outflow',) * 4, solid=solid, solid_wall=wall).residual(
                            U.astype(complex))
    mref = np.sum(Fm.imag / H * Rb)
    print('masked residual %s %s: <J du, rb> %.15e  <du, J^T rb> %.15e  rel %.2e; mu rel %.2e'
          % (block, wall, lhs, rhs, rel(lhs, rhs), rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10 and rel(mref, mub) < 1e-10
    assert not Ub[..., solid].any()          # solid inputs are overwritten or unused


@pytest.mark.parametrize('wall', ['slip', 'noslip'])
@pytest.mark.parametrize('block', ['corner', 'inner'])
def test_masked_step_vjp_dot_product(block, wall):
    """U3bar on the fluid cells only: there the library's step and the
    oracle's agree (the two keep different values in solid cells)."""
    solid = masks()[block]
    U = workloads.random_smooth_2d(NX, NY, seed=62, noise=1e-3)
    s, sc = pair(solid, wall)
    s.set_state(to_dev(U))
    dt = s.rk_step(0.0)['dt']
    rng = np.random.default_rng([2608, 94, int(block == 'inner'), int(wall == 'noslip')])
    scale = np.abs(U).reshape(3, 4, -1).max(axis=-1)[..., None, None]
    dU = rng.standard_normal(U.shape) * scale
    Wb = rng.standard_normal(U.shape)
    Wb[..., solid] = 0.0
    U3c, used, info = rk3_step(sc, U + 1j * H * dU, 0.0, dt)
    assert used == dt and info['restarts'] == 0
    lhs = np.sum(U3c.imag / H * Wb)
    Ub, mub = s.rk_step_vjp(to_dev(U), dt, to_dev(Wb))
    rhs = np.sum(dU * Ub.cpu().numpy())
    sm = Scheme2D(NX, NY, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01 + 1j * H), Options(),
                  bc=('outflow',) * 4, solid=solid, solid_wall=wall)
    U3m, _, _ = rk3_step(sm, U.astype(complex), 0.0, dt)
    mref = np.sum(U3m.imag / H * Wb)
    print('masked step %s %s: rel %.2e mu rel %.2e' % (block, wall, rel(lhs, rhs), rel(mref, mub)))
    assert rel(lhs, rhs) < 1e-10 and rel(mref, mub) < 1e-10
    assert not Ub.cpu().numpy()[..., solid].any()


def test_masked_step_vjp_solid_cells_against_gpu_differences():
    """U3bar on every cell, solid ones included: the library's step leaves a
    solid cell next to the fluid at the mirror image of the last stage input
    and a solid cell beyond the band at its input, and the adjoint follows
    both; checked against central differences of the GPU step."""
    solid = masks()['inner']
    band = mirror_band(solid)
    assert band.any() and (solid & ~band).any()
    U = workloads.random_smooth_2d(NX, NY, seed=63, noise=1e-3)
    s, _ = pair(solid, 'noslip')
    s.set_state(to_dev(U))
    dt = s.rk_step(0.0)['dt']
    rng = np.random.default_rng([2608, 93])
    scale = np.abs(U).reshape(3, 4, -1).max(axis=-1)[..., None, None]
    dU = rng.standard_normal(U.shape) * scale
    Wb = rng.standard_normal(U.shape)
    Ub, _ = s.rk_step_vjp(to_dev(U), dt, to_dev(Wb))
    Ub = Ub.cpu().numpy()
    eps = 1e-7

    def step(V):
        s.set_state(to_dev(V))
        d = s.rk_step(dt)
        assert d['restarts'] == 0
        return s.get_state()[0].cpu().numpy()
    Up, Um = step(U + eps * dU), step(U - eps * dU)
    parts = {}
    for name, sel in (('fluid', ~solid), ('band', band), ('beyond', solid & ~band)):
        W = np.where(sel, Wb, 0.0)
        fd = np.sum((Up - Um) * W) / (2 * eps)
        Wd = to_dev(W)
        a, _ = s.rk_step_vjp(to_dev(U), dt, Wd)
        parts[name] = (fd, np.sum(dU * a.cpu().numpy()))
        print('%s outputs: differences %.12e adjoint %.12e rel %.2e'
              % (name, fd, parts[name][1], rel(fd, parts[name][1])))
    for name, (fd, ad) in parts.items():
        assert rel(fd, ad) < 1e-6, name
    # beyond the band the step carries the input through
    a, _ = s.rk_step_vjp(to_dev(U), dt, to_dev(np.where(solid & ~band, Wb, 0.0)))
    a = a.cpu().numpy()
    assert np.array_equal(a[..., solid & ~band], Wb[..., solid & ~band])
    assert np.allclose(np.sum(dU * Ub), sum(p[1] for p in parts.values()), rtol=1e-12, atol=0)


def test_masked_vjp_prescribed_solid_state():
    """Solid cells holding a prescribed state (hweno_set_solid_state) take
    nothing from the input: four rows of them below the fluid against the
    oracle's tangent."""
    nx, ny, pad = 16, 12, 4
    h = 1.0 / nx
    U = workloads.random_smooth_2d(nx, ny + pad, seed=64, noise=1e-3,
                                   extent=(0.0, 1.0, -pad * h, ny * h))
    solid = np.zeros((ny + pad, nx), bool)
    solid[:pad] = True
    Wp = (1.2, 0.3, -0.4, 0.9)
    bc = ('periodic', 'periodic', 'outflow', 'outflow')
    ext = (0.0, 1.0, -pad * h, ny * h)
    s = hweno.Solver(nx, ny + pad, extent=ext, mu_ref=0.01, bc=bc)
    s.set_solid(solid)
    s.set_solid_state(solid, Wp)
    g = 1.4
    cons = np.array([Wp[0], Wp[0] * Wp[1], Wp[0] * Wp[2],
                     Wp[3] / (g - 1) + 0.5 * Wp[0] * (Wp[1] ** 2 + Wp[2] ** 2)])
    sc = Scheme2D(nx, ny + pad, *ext, Physics(mu_ref=0.01), Options(), bc=bc, solid=solid,
                  fixed=solid, fixed_state=cons)
    rng = np.random.default_rng([2608, 92])
    scale = np.abs(U).reshape(3, 4, -1).max(axis=-1)[..., None, None]
    dU = rng.standard_normal(U.shape) * scale
    Rb = rng.standard_normal(U.shape)
    Fc, _, _ = sc.residual(U + 1j * H * dU)
    lhs = np.sum(Fc.imag / H * Rb)
    Ub, _ = s.residual_vjp(to_dev(U), to_dev(Rb))
    Ub = Ub.cpu().numpy()
    rhs = np.sum(dU * Ub)
    print('prescribed solid state: rel %.2e' % rel(lhs, rhs))
    assert rel(lhs, rhs) < 1e-10
    assert not Ub[..., solid].any()
