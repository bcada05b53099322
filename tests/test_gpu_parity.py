"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Metric (per field = component x moment): max over cells of |gpu - oracle|
divided by max over cells of |oracle|.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from oracle import rk  # noqa: E402
from oracle.common import Options, Physics  # noqa: E402
from oracle.scheme1d import Scheme1D  # noqa: E402
from oracle.scheme2d import Scheme2D  # noqa: E402
from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = 'cuda:0'


def rel_err(A, B):
    """max over fields of max |A - B| / max |B|; A, B shaped (fields, cells)."""
    A, B = np.asarray(A), np.asarray(B)
    out = 0.0
    for k in range(A.shape[0]):
        den = np.abs(B[k]).max()
        num = np.abs(A[k] - B[k]).max()
        out = max(out, num / den if den > 0 else num)
    return out


def fields2d(U):
    return np.asarray(U).reshape(-1, U.shape[-2] * U.shape[-1])


def fields1d(U):
    return np.asarray(U).reshape(-1, U.shape[-1])


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


BCS_WALL = ('noslip', 'noslip', 'noslip', 'slip')


# weights: nonlinear (the paper), linear everywhere (test mode), and linear in
# the gradient reconstruction only (the counterpart discussed in Remark 3.1)
MODES = {'nonlinear': {}, 'linear': dict(linear_weights=True),
         'linear_gradients': dict(linear_gradients=True)}


@pytest.mark.parametrize('mode', list(MODES))
@pytest.mark.parametrize('shape', [(37, 29), (8, 5)])
def test_residual2d_periodic(mode, shape):
    nx, ny = shape
    U = workloads.random_smooth_2d(nx, ny, seed=3, noise=1e-3)
    opt = MODES[mode]
    s = hweno.Solver(nx, ny, extent=(0.0, 1.0, 0.0, 1.0), mu_ref=0.01, Pr=0.72,
                     **{k: int(v) for k, v in opt.items()})
    R, V, d = s.residual(to_dev(U))
    sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01, Pr=0.72), Options(**opt))
    Ro, Vo, do = sc.residual(U)
    eR = rel_err(fields2d(R.cpu().numpy()), fields2d(Ro))
    eV = rel_err(fields2d(V.cpu().numpy()), fields2d(Vo.reshape(8, ny, nx)))
    print('2D residual shape', shape, mode, 'R err %.2e V err %.2e' % (eR, eV))
    assert eR < 1e-11 and eV < 1e-12
    if mode == 'linear_gradients':
        # the option changes only the viscous part: visibly, and not the moments
        Rn, Vn, _ = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01, Pr=0.72),
                             Options()).residual(U)
        assert rel_err(fields2d(Rn), fields2d(Ro)) > 1e-8
        assert np.array_equal(Vn, Vo)
    assert abs(d['alpha_star'] - do['alpha']) < 1e-13 * do['alpha']
    assert abs(d['beta_max'] - do['beta_max']) < 1e-12 * do['beta_max']
    assert d['pp_cells'] == do['pp_cells']


def test_inviscid_limit_residual_and_step():
    """mu = 0 (the Euler limit): no viscous fluxes and no viscous step bound;
    the residual, the modified moments and one paper-rule step (Delta t from
    the wave speed alone) against the oracle, with walls."""
    nx, ny = 30, 22
    U = workloads.random_smooth_2d(nx, ny, seed=14, noise=1e-3, extent=(0.0, 1.0, 0.0, 0.5))
    ext = (0.0, 1.0, 0.0, 0.5)
    s = hweno.Solver(nx, ny, extent=ext, mu_ref=0.0, bc=BCS_WALL)
    sc = Scheme2D(nx, ny, *ext, Physics(mu_ref=0.0), Options(), bc=BCS_WALL)
    R, V, d = s.residual(to_dev(U))
    Ro, Vo, do = sc.residual(U)
    eR = rel_err(fields2d(R.cpu().numpy()), fields2d(Ro))
    eV = rel_err(fields2d(V.cpu().numpy()), fields2d(Vo.reshape(8, ny, nx)))
    s.set_state(to_dev(U))
    dg = s.rk_step(0.0)
    Uo, dto, _ = rk.rk3_step(sc, U, 0.0)
    eS = rel_err(fields2d(s.get_state()[0].cpu().numpy()), fields2d(Uo))
    print('mu = 0: residual %.2e, V %.2e, step %.2e, dt %.6e vs %.6e' % (eR, eV, eS, dg['dt'], dto))
    assert eR < 1e-11 and eV < 1e-12 and eS < 1e-12
    assert abs(dg['dt'] - dto) < 1e-13 * dto


@pytest.mark.parametrize('bc', [BCS_WALL, ('outflow', 'slip', 'slip', 'outflow')])
def test_residual2d_walls_and_outflow(bc):
    nx, ny = 24, 14
    U = workloads.random_smooth_2d(nx, ny, seed=5, noise=1e-3, extent=(0.0, 1.0, 0.0, 0.5))
    s = hweno.Solver(nx, ny, extent=(0.0, 1.0, 0.0, 0.5), mu_ref=1 / 200, Pr=0.73, bc=bc)
    R, V, _ = s.residual(to_dev(U))
    sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 0.5, Physics(mu_ref=1 / 200, Pr=0.73), Options(), bc=bc)
    Ro, Vo, _ = sc.residual(U)
    eR = rel_err(fields2d(R.cpu().numpy()), fields2d(Ro))
    eV = rel_err(fields2d(V.cpu().numpy()), fields2d(Vo.reshape(8, ny, nx)))
    print('2D residual bc', bc, 'R err %.2e V err %.2e' % (eR, eV))
    assert eR < 1e-11 and eV < 1e-12


def test_rk_step2d_one_step():
    nx, ny = 21, 18
    U = workloads.random_smooth_2d(nx, ny, seed=7, noise=1e-3)
    s = hweno.Solver(nx, ny, extent=(0.0, 1.0, 0.0, 1.0), mu_ref=0.01, cfl=0.6)
    s.set_state(to_dev(U))
    d = s.rk_step(0.0)
    Ug, t = s.get_state()
    sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01), Options(cfl=0.6))
    Uo, dto, info = rk.rk3_step(sc, U, 0.0)
    e = rel_err(fields2d(Ug.cpu().numpy()), fields2d(Uo))
    print('2D one RK3 step: dt gpu %.17g oracle %.17g, state err %.2e' % (d['dt'], dto, e))
    assert abs(d['dt'] - dto) < 1e-14 * dto
    assert e < 1e-12
    assert abs(t - dto) < 1e-14 * dto


@pytest.mark.parametrize('mode', list(MODES))
def test_residual1d(mode):
    nx = 150
    U = workloads.random_smooth_1d(nx, seed=1)
    opt = MODES[mode]
    s = hweno.Solver(nx, extent=(0.0, 1.0), mu_ref=0.01, **{k: int(v) for k, v in opt.items()})
    R, V, d = s.residual(to_dev(U))
    sc = Scheme1D(nx, 0.0, 1.0, Physics(mu_ref=0.01), Options(**opt))
    Ro, Vo, do = sc.residual(U)
    eR = rel_err(fields1d(R.cpu().numpy()), fields1d(Ro))
    eV = rel_err(fields1d(V.cpu().numpy()), fields1d(Vo[0]))
    print('1D residual', mode, 'R err %.2e V err %.2e' % (eR, eV))
    if mode == 'linear_gradients':
        Rn, _, _ = Scheme1D(nx, 0.0, 1.0, Physics(mu_ref=0.01), Options()).residual(U)
        assert rel_err(fields1d(Rn), fields1d(Ro)) > 1e-8
    assert eR < 1e-11 and eV < 1e-12
    assert abs(d['alpha_star'] - do['alpha']) < 1e-13 * do['alpha']


def test_rk1d_steps_smooth_wave():
    nx = 200
    U = workloads.smooth_wave_1d(nx, seed=0)
    kw = dict(extent=(0.0, 2 * np.pi), mu_ref=0.01, cfl=0.3, b_visc=0.0)
    s = hweno.Solver(nx, **kw)
    s.set_state(to_dev(U))
    sc = Scheme1D(nx, 0.0, 2 * np.pi, Physics(mu_ref=0.01), Options(cfl=0.3, b_visc=0.0),
                  bc=('periodic', 'periodic'))
    Uo, t = U, 0.0
    for n in range(20):
        d = s.rk_step(0.0)
        Uo, dto, _ = rk.rk3_step(sc, Uo, t)
        t += dto
    Ug, tg = s.get_state()
    e = rel_err(fields1d(Ug.cpu().numpy()), fields1d(Uo))
    print('1D 20 steps: t gpu %.17g oracle %.17g err %.2e' % (tg, t, e))
    assert e < 1e-10 and abs(tg - t) < 1e-13


def _cons(P, gamma=1.4):
    """(n, 4) primitive rows -> (4, n) conservative states."""
    r, u, v, p = P.T
    return np.stack([r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v)])


def test_inflow_profile_residual_step_and_errors():
    """Inflow that varies along two sides (x-low: one state per row, y-high:
    one per column) against the oracle's profile ghosts; clearing a profile
    restores the constant state; bad profiles are refused."""
    nx, ny = 24, 20
    U = workloads.random_smooth_2d(nx, ny, seed=9, noise=1e-3)
    rng = np.random.default_rng(9)

    def prof(n):
        return np.column_stack([1.0 + 0.2 * rng.random(n), 0.3 * rng.standard_normal(n),
                                0.3 * rng.standard_normal(n), 1.0 + 0.2 * rng.random(n)])
    px, py = prof(ny), prof(nx)
    bc = ('inflow', 'outflow', 'slip', 'inflow')
    const = (1.1, 0.2, 0.0, 0.9)
    s = hweno.Solver(nx, ny, mu_ref=0.01, bc=bc, inflow={0: const, 3: const})
    s.set_inflow_profile(0, px)
    s.set_inflow_profile(3, py)
    R, V, _ = s.residual(to_dev(U))
    sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01), Options(), bc=bc,
                  inflow={0: _cons(px), 3: _cons(py)})
    Ro, Vo, _ = sc.residual(U)
    eR = rel_err(fields2d(R.cpu().numpy()), fields2d(Ro))
    s.set_state(to_dev(U))
    d = s.rk_step(0.0)
    Uo, dto, _ = rk.rk3_step(sc, U, 0.0)
    eS = rel_err(fields2d(s.get_state()[0].cpu().numpy()), fields2d(Uo))
    print('inflow profiles: residual err %.2e, one step err %.2e' % (eR, eS))
    assert eR < 1e-11 and eS < 1e-12 and abs(d['dt'] - dto) < 1e-14 * dto
    # back to the constant state on both sides
    s.set_inflow_profile(0, None)
    s.set_inflow_profile(3, None)
    R2, _, _ = s.residual(to_dev(U))
    c = _cons(np.array([const]))[:, 0]
    Rc, _, _ = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01), Options(), bc=bc,
                        inflow={0: c, 3: c}).residual(U)
    assert rel_err(fields2d(R2.cpu().numpy()), fields2d(Rc)) < 1e-11
    for side, p in ((0, px[:-1]), (1, px), (3, px)):          # wrong n, wrong kinds
        with pytest.raises(hweno.HwenoError):
            s.set_inflow_profile(side, p)
    bad = px.copy()
    bad[3, 0] = -1.0
    with pytest.raises(hweno.HwenoError):
        s.set_inflow_profile(0, bad)
    b = hweno.Batch([dict(nx=8, ny=8, bc=bc, inflow={0: const, 3: const})])
    assert hweno.lib().hweno_set_inflow_profile(b._h, 0, None, 0) == 1


def _equivariance_errors(residual, U):
    """max field errors of residual(U) -> (F, V) under x -> -x and x <-> y."""
    F, V = residual(U)
    par = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None]
    sg = np.array([1.0, -1.0, 1.0])
    Um = np.stack([sg[m] * par * U[m][..., ::-1] for m in range(3)])
    Fm, _ = residual(np.ascontiguousarray(Um))
    want = np.stack([sg[m] * par * F[m][..., ::-1] for m in range(3)])
    e_ref = rel_err(fields2d(Fm), fields2d(want))
    perm = [0, 2, 1, 3]
    Us = np.stack([U[m][perm].swapaxes(-1, -2) for m in (0, 2, 1)])
    Fs, Vs = residual(np.ascontiguousarray(Us))
    want = np.stack([F[m][perm].swapaxes(-1, -2) for m in (0, 2, 1)])
    e_swap = rel_err(fields2d(Fs), fields2d(want))
    V4 = V.reshape(2, 4, *V.shape[-2:])
    wantV = np.stack([V4[m][perm].swapaxes(-1, -2) for m in (1, 0)])
    e_v = rel_err(fields2d(Vs.reshape(wantV.shape)), fields2d(wantV))
    return e_ref, e_swap, e_v


def test_gpu_residual_equivariance():
    """P13 on the device path: reflecting x (u odd, xi-moments flipped) or
    exchanging x and y (with u <-> v and the xi/eta moments) commutes with the
    GPU residual on a square no-slip box.  Smooth state: to rounding.  With
    the limiter active (the 2D Sedov blast after three oracle steps, beta up
    to 1e10) rounding is amplified, for the oracle as well: the GPU's error
    stays within 10x the oracle's own."""
    n = 28
    bc = ('noslip',) * 4
    s = hweno.Solver(n, n, mu_ref=0.01, bc=bc)

    def gpu(U):
        F, V, _ = s.residual(to_dev(U))
        return F.cpu().numpy(), V.cpu().numpy()
    sc = Scheme2D(n, n, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01), Options(), bc=bc)

    def ora(U):
        F, V, _ = sc.residual(U)
        return F, V
    U = workloads.random_smooth_2d(n, n, seed=21, noise=1e-3)
    e = _equivariance_errors(gpu, U)
    print('smooth: reflection %.2e, swap %.2e, swap of V %.2e' % e)
    assert max(e) < 1e-11
    ph = Physics(mu_ref=1e-3)
    sed = Scheme2D(n, n, 0.0, 1.1, 0.0, 1.1, ph, Options(), bc=('slip', 'outflow') * 2)
    X, t = workloads.sedov_2d(n), 0.0
    for _ in range(3):
        X, dt, _ = rk.rk3_step(sed, X, t)
        t += dt
    _, _, dg = s.residual(to_dev(X))
    eg, eo = _equivariance_errors(gpu, X), _equivariance_errors(ora, X)
    print('Sedov state (limiter cells %d): gpu %s, oracle %s'
          % (dg['pp_cells'], ['%.1e' % v for v in eg], ['%.1e' % v for v in eo]))
    assert dg['pp_cells'] > 0
    for a, b in zip(eg, eo):
        assert a < 10.0 * max(b, 1e-13)


def test_time_dependent_inflow_steps_and_errors():
    """Example 5.11's forced inflow: fixed steps with the left side's profile at
    the three stage times (and the post-shock state on top) against the
    oracle stepping with the same boundary data in time; refused inputs."""
    m = workloads.ShockMixingLayer(50, 20)
    g = 1.4
    ph = dict(gamma=g, Pr=0.72, mu_ref=1.0 / 500.0)
    s = hweno.Solver(m.nx, m.ny, extent=m.extent, bc=m.bc, inflow={0: m.top, 3: m.top}, **ph)
    U = m.initial()
    s.set_state(to_dev(U))
    sc = Scheme2D(m.nx, m.ny, *m.extent, Physics(**ph), Options(), bc=m.bc,
                  inflow={0: _cons(m.inflow(0.0), g), 3: _cons(np.array([m.top]), g)[:, 0]})
    _, _, d0 = sc.residual(U)
    dt = rk.trial_dt(sc, d0['alpha'], 0.0)
    Uo, t = U, 0.0
    for _ in range(4):
        s.set_inflow_stages(0, m.inflow(t), m.inflow(t + dt), m.inflow(t + 0.5 * dt))
        d = s.rk_step_inflow(dt)
        Uo, _, _ = rk.rk3_step(sc, Uo, t, dt=dt, inflow=lambda tt: {0: _cons(m.inflow(tt), g)})
        t += dt
        assert d['restarts'] == 0 and abs(d['t'] - t) < 1e-12 * t
    e = rel_err(fields2d(s.get_state()[0].cpu().numpy()), fields2d(Uo))
    print('time-dependent inflow, 4 steps: state err %.2e' % e)
    assert e < 1e-12
    p = m.inflow(t)
    with pytest.raises(hweno.HwenoError):
        s.rk_step_inflow(0.0)
    with pytest.raises(hweno.HwenoError):
        s.set_inflow_stages(0, p[:-1], p[:-1], p[:-1])
    with pytest.raises(hweno.HwenoError):
        s.set_inflow_stages(1, p, p, p)                       # an outflow side
    assert hweno.lib().hweno_set_inflow_stages(s._h, 0, None, None, None, 0) == 0


def test_prescribed_state_cells_equal_an_inflow_side():
    """Four rows of solid cells holding a state give the fluid the ghost data
    of an inflow side with that state: the fluid's residual and modified
    moments equal the box grid's bit for bit (as in the oracle); refused
    inputs."""
    nx, ny, pad = 16, 12, 4
    h = 1.0 / nx
    U = workloads.random_smooth_2d(nx, ny, seed=41, noise=1e-3, extent=(0.0, 1.0, 0.0, ny * h))
    Wp = (1.2, 0.3, -0.4, 0.9)                      # flow into the boundary
    box = hweno.Solver(nx, ny, extent=(0.0, 1.0, 0.0, ny * h), mu_ref=0.01, inflow={2: Wp},
                       bc=('periodic', 'periodic', 'inflow', 'outflow'))
    Rb, Vb, _ = box.residual(to_dev(U))
    Um = np.zeros((3, 4, ny + pad, nx))
    Um[:, :, pad:] = U
    solid = np.zeros((ny + pad, nx), bool)
    solid[:pad] = True
    s = hweno.Solver(nx, ny + pad, extent=(0.0, 1.0, -pad * h, ny * h), mu_ref=0.01,
                     bc=('periodic', 'periodic', 'outflow', 'outflow'))
    s.set_solid(solid)
    s.set_solid_state(solid, Wp)
    Rm, Vm, _ = s.residual(to_dev(Um))
    assert torch.equal(Rm[..., pad:, :], Rb) and torch.equal(Vm[..., pad:, :], Vb)
    assert not Rm[..., :pad, :].any()
    s.set_solid_state(None)                          # mirrors again: another boundary
    Rw, _, _ = s.residual(to_dev(Um))
    assert not torch.equal(Rw[..., pad:, :], Rb)
    with pytest.raises(hweno.HwenoError):
        s.set_solid_state(~solid, Wp)                # fluid cells
    with pytest.raises(hweno.HwenoError):
        s.set_solid_state(solid, (1.0, 0.0, 0.0, -1.0))
    with pytest.raises(hweno.HwenoError):
        hweno.Solver(8, 8).set_solid_state(np.zeros((8, 8), bool), Wp)   # no mask


def test_example_5_10_steps_match_oracle():
    """Example 5.10's set-up on a 48 x 32 grid: a masked domain with a step,
    reflective walls, solid cells holding the post-shock state and a top
    boundary that follows the exact shock at each stage's time; three steps
    against the oracle on the fluid cells."""
    m = workloads.Mach10Reflection(48, 32)
    g = 1.4
    ph = dict(gamma=g, Pr=0.72, mu_ref=1e-3)
    s = hweno.Solver(m.nx, m.ny, extent=m.extent, bc=m.bc, inflow={0: m.post, 3: m.post}, **ph)
    s.set_solid(m.solid)
    s.set_solid_state(m.fixed, m.post)
    U = m.initial()
    s.set_state(to_dev(U))
    post = _cons(np.array([m.post]), g)[:, 0]
    sc = Scheme2D(m.nx, m.ny, *m.extent, Physics(**ph), Options(), bc=m.bc,
                  inflow={0: post, 3: _cons(m.top(0.0), g)}, solid=m.solid, fixed=m.fixed,
                  fixed_state=post)
    _, _, d0 = sc.residual(U)
    dt = rk.trial_dt(sc, d0['alpha'], 0.0)
    Uo, t, pp = U, 0.0, 0
    for _ in range(3):
        s.set_inflow_stages(3, m.top(t), m.top(t + dt), m.top(t + 0.5 * dt))
        d = s.rk_step_inflow(dt)
        Uo, _, info = rk.rk3_step(sc, Uo, t, dt=dt, inflow=lambda tt: {3: _cons(m.top(tt), g)})
        t += dt
        pp += info['pp_cells']
        assert d['pp_cells'] == info['pp_cells']
    G = s.get_state()[0].cpu().numpy()
    fl = ~m.solid
    e = rel_err(G[..., fl].reshape(12, -1), Uo[..., fl].reshape(12, -1))
    print('Example 5.10 set-up, 3 steps of %.3e: fluid state err %.2e (limiter cell-stages %d)'
          % (dt, e, pp))
    assert e < 1e-12


@pytest.mark.parametrize('wall', ['slip', 'noslip'])
def test_masked_domain_residual_and_step(wall):
    """Solid cells inside the grid (a block in a corner, and one away from the
    box's sides so all four wall directions and the block's corners occur):
    residual (zero in solid cells) and one RK step against the oracle's masked
    domain; the step is compared on the fluid cells (the library keeps the
    last mirror fill in solid cells)."""
    nx, ny = 30, 24
    U = workloads.random_smooth_2d(nx, ny, seed=31, noise=1e-3)
    corner = np.zeros((ny, nx), bool)
    corner[:10, :9] = True
    inner = np.zeros((ny, nx), bool)
    inner[8:15, 11:21] = True
    for solid in (corner, inner):
        bc = ('outflow',) * 4
        s = hweno.Solver(nx, ny, mu_ref=0.01, bc=bc)
        s.set_solid(solid, wall)
        R, V, d = s.residual(to_dev(U))
        R, V = R.cpu().numpy(), V.cpu().numpy()
        sc = Scheme2D(nx, ny, 0.0, 1.0, 0.0, 1.0, Physics(mu_ref=0.01), Options(), bc=bc,
                      solid=solid, solid_wall=wall)
        Ro, Vo, do = sc.residual(U)
        eR = rel_err(fields2d(R), fields2d(Ro))
        eV = rel_err(fields2d(V), fields2d(Vo.reshape(8, ny, nx)))
        assert not R[..., solid].any() and not V[..., solid].any()
        s.set_state(to_dev(U))
        dg = s.rk_step(0.0)
        Uo, dto, _ = rk.rk3_step(sc, U, 0.0)
        G = s.get_state()[0].cpu().numpy()
        eS = rel_err(G[..., ~solid].reshape(12, -1), Uo[..., ~solid].reshape(12, -1))
        print('%s block, %s wall: residual %.2e, V %.2e, step %.2e' %
              ('corner' if solid is corner else 'inner', wall, eR, eV, eS))
        assert eR < 1e-11 and eV < 1e-12 and eS < 1e-12
        assert abs(dg['dt'] - dto) < 1e-13 * dto and abs(d['alpha_star'] - do['alpha']) < 1e-13 * do['alpha']


def test_masked_domain_refusals():
    nx, ny = 12, 10
    s = hweno.Solver(nx, ny, mu_ref=0.01, bc=('outflow',) * 4)
    m = np.zeros((ny, nx), bool)
    m[:4, :4] = True
    with pytest.raises(hweno.HwenoError):
        s.set_solid(m, 'outflow')                 # walls are reflective or no-slip
    with pytest.raises(hweno.HwenoError):
        s.set_solid(np.ones((ny, nx), bool))      # no fluid
    s.set_solid(m)
    U = workloads.random_smooth_2d(nx, ny, seed=2, noise=1e-3)
    z = torch.zeros((3, 4, ny, nx), dtype=torch.float64, device=DEV)
    s.residual_vjp(to_dev(U), z)                 # reverse mode on a masked grid
    s.set_solid(None)
    s.residual_vjp(to_dev(U), z)
    b = hweno.Batch([dict(nx=8, ny=8)])
    mm = np.zeros((8, 8), np.uint8)
    assert hweno.lib().hweno_set_solid(b._h, mm.ctypes.data_as(ctypes.c_void_p), 3) == 1
