"""Solid cells that hold a prescribed state (the post-shock condition along
part of a wall inside the grid, Example 5.10): pinned to the prescribed-state
boundary of Remark 4.1.  Four rows of such cells below the fluid give the
fluid exactly the ghost data of an inflow side with that state, so the
residual of every fluid cell equals the box grid's bit for bit; a mirror
wall in their place does not."""

import numpy as np

from oracle.common import Options, Physics
from oracle.scheme2d import Scheme2D
from paper_2608_10569_amd import workloads


def _cons(rho, u, v, p, gamma=1.4):
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def test_fixed_cells_equal_a_prescribed_state_side():
    nx, ny, pad = 16, 12, 4
    h = 1.0 / nx                                   # a power of two: both grids' dy exact
    U = workloads.random_smooth_2d(nx, ny, seed=41, noise=1e-3, extent=(0.0, 1.0, 0.0, ny * h))
    W = _cons(1.2, 0.3, -0.4, 0.9)                 # flow into the boundary
    ph, op = Physics(mu_ref=0.01), Options()
    box = Scheme2D(nx, ny, 0.0, 1.0, 0.0, ny * h, ph, op,
                   bc=('periodic', 'periodic', 'inflow', 'outflow'), inflow={2: W})
    Rb, Vb, _ = box.residual(U)
    Um = np.zeros((3, 4, ny + pad, nx))
    Um[:, :, pad:] = U
    Um[0, :, :pad] = W[:, None, None]
    solid = np.zeros((ny + pad, nx), bool)
    solid[:pad] = True
    fixed = solid.copy()
    masked = Scheme2D(nx, ny + pad, 0.0, 1.0, -pad * h, ny * h, ph, op,
                      bc=('periodic', 'periodic', 'outflow', 'outflow'), solid=solid,
                      fixed=fixed, fixed_state=W)
    assert len(masked.fixed_cells) == pad * nx and not masked.mirrors
    Rm, Vm, _ = masked.residual(Um)
    assert np.array_equal(Rm[:, :, pad:], Rb)
    assert np.array_equal(Vm.reshape(8, ny + pad, nx)[:, pad:], Vb.reshape(8, ny, nx))
    assert not Rm[:, :, :pad].any()
    # the same cells as a reflective wall: the fluid next to them sees another boundary
    wall = Scheme2D(nx, ny + pad, 0.0, 1.0, -pad * h, ny * h, ph, op,
                    bc=('periodic', 'periodic', 'outflow', 'outflow'), solid=solid)
    Rw, _, _ = wall.residual(Um)
    assert np.abs(Rw[:, :, pad] - Rb[:, :, 0]).max() > 1e-2 * np.abs(Rb).max()


def test_fixed_cells_mixed_with_mirrors():
    """Fixed cells next to mirrored ones: every solid cell near the fluid is
    either in the mirror list or the fixed list, never both, and fixed cells
    are never a mirror's source."""
    nx, ny = 24, 16
    solid = np.zeros((ny, nx), bool)
    solid[:6, :10] = True
    fixed = solid.copy()
    fixed[:, 4:] = False
    sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(), Options(),
                  bc=('outflow',) * 4, solid=solid, fixed=fixed, fixed_state=_cons(1, 0, 0, 1))
    dst = {d for d, _, _ in sc.mirrors}
    fx = set(sc.fixed_cells)
    assert not (dst & fx) and fx and dst
    assert all(fixed[j, i] for j, i in fx) and not any(fixed[j, i] for j, i in dst)
    assert not any(solid[js, is_] for _, (js, is_), _ in sc.mirrors)
