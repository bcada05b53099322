"""Manufactured solutions on the GPU (Examples 5.1 and 5.2): the source hook
against the oracle step by step, and the accuracy tables at the paper's mesh
sizes run through the HIP path, for HWENO-GR and its comparison scheme
HWENO-DR.  Sources and exact moments come from the
oracle's symbolic fields (6-point Gauss moments); the GPU adds them in every
stage through hweno_rk_step_source."""

import math
import os

import numpy as np
import pytest

torch = pytest.importorskip('torch')
sp = pytest.importorskip('sympy')

from oracle import rk  # noqa: E402
from oracle.common import Options, Physics  # noqa: E402
from oracle.mms import MMS1D, MMS2D  # noqa: E402
from oracle.scheme1d import Scheme1D  # noqa: E402
from oracle.scheme2d import Scheme2D  # noqa: E402
from paper_2608_10569_amd import hweno  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden')
PH = dict(gamma=1.4, Pr=0.72, mu_ref=0.01)
T_END = 0.1
CFL = 0.6


def load_table(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith('#'):
                v = line.split()
                rows[int(v[0])] = (float(v[1]), float(v[2]))
    return rows


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


class PolySource:
    """Stage sources of a manufactured solution on the GPU.  The fields of
    Examples 5.1 and 5.2 depend on t only through exp(-t), so the source is a
    polynomial in z = exp(-t) whose coefficients depend on space alone:
    S(x, t) = sum_p z^p G_p(x).  The moments of every G_p are taken once per
    mesh with the oracle's own quadrature; a stage source is then a short
    polynomial evaluation on the device."""

    def __init__(self, mms):
        t = mms.symbols[-1]
        z = sp.Symbol('z')
        polys = [sp.Poly(sp.expand(e.subs(sp.exp(-t), z)), z) for e in mms.source_expr]
        for P in polys:
            assert t not in P.as_expr().free_symbols
        deg = max(P.degree() for P in polys)
        self.G = []
        for p in range(deg + 1):
            coeffs = [P.coeff_monomial(z ** p) for P in polys]
            fn = sp.lambdify(mms.symbols, coeffs, 'numpy')
            self.G.append(to_dev(np.stack(mms._moments(fn, 0.0))))

    def __call__(self, t):
        zt = math.exp(-t)
        out = self.G[-1].clone()
        for G in reversed(self.G[:-1]):       # Horner in z
            out = out * zt + G
        return out.contiguous()


def gpu_mms_run(s, U0, source, h, t_end):
    """The h^{5/3} rule of the convergence studies: dt = CFL h^{5/3} / alpha*
    from the stage-1 traces, the last step clipped to t_end."""
    s.set_state(U0)
    t = 0.0
    n = 0
    while t < t_end - 1e-14 * t_end:
        U, _ = s.get_state()
        _, _, d = s.residual(U)
        dt = min(CFL * h ** (5.0 / 3.0) / d['alpha_star'], t_end - t)
        s.rk_step_source(dt, source(t), source(t + dt), source(t + 0.5 * dt))
        t += dt
        n += 1
    U, tg = s.get_state()
    return U, tg, n


def test_source_step_matches_oracle_2d():
    n = 16
    sc = Scheme2D(n, n, 0.0, 1.0, 0.0, 1.0, Physics(**PH), Options(cfl=CFL))
    m = MMS2D(sc)
    s = hweno.Solver(n, n, **PH)
    U = m.exact(0.0)
    s.set_state(to_dev(U))
    t = 0.0
    worst = 0.0
    for k in range(6):
        _, _, d = sc.residual(U, m.source(t))
        dt = rk.trial_dt(sc, d['alpha'], t, rule='h53')
        srcs = [to_dev(np.stack(m.source(tt))) for tt in (t, t + dt, t + 0.5 * dt)]
        s.rk_step_source(dt, *srcs)
        U, used, info = rk.rk3_step(sc, U, t, dt, source=m.source)
        assert used == dt and info['restarts'] == 0
        t += dt
        G = s.get_state()[0].cpu().numpy()
        for mm in range(3):
            for c in range(4):
                worst = max(worst, np.abs(G[mm, c] - U[mm, c]).max() / np.abs(U[mm, c]).max())
    print('2D source steps: worst rel err per field %.2e after 6 steps' % worst)
    assert worst < 1e-12


def test_source_step_rejects_bad_arguments():
    s = hweno.Solver(8, 8, **PH)
    z = torch.zeros((3, 4, 8, 8), dtype=torch.float64, device=DEV)
    with pytest.raises(hweno.HwenoError):
        s.rk_step_source(1e-3, z, z, z)          # no state yet
    s.set_state(z + 1.0)
    with pytest.raises(hweno.HwenoError):
        s.rk_step_source(0.0, z, z, z)           # dt must be positive


def _rate(e0, e1, n0, n1):
    return math.log(e0 / e1) / math.log(n1 / n0)


def test_table_5_1_on_gpu():
    """Example 5.1 to T = 0.1 on the meshes of Table 5.1 from N = 80 to 280
    (N = 40 is pre-asymptotic): density errors within 3x of the printed GR
    column, fifth-order rates between consecutive meshes."""
    tab = load_table('table_5_1_gr.txt')
    res = {}
    for n in (80, 120, 160, 200, 240, 280):
        sc = Scheme1D(n, 0.0, 1.0, Physics(**PH), Options(cfl=CFL))
        m = MMS1D(sc)
        s = hweno.Solver(n, extent=(0.0, 1.0), **PH)
        src = PolySource(m)
        U, t, steps = gpu_mms_run(s, to_dev(m.exact(0.0)), src, 1.0 / n, T_END)
        err = U.cpu().numpy()[0, 0] - m.exact(t)[0, 0]
        res[n] = (np.abs(err).max(), np.abs(err).mean())
        print('1D N=%d: %d steps, Linf %.3e (paper %.3e)  L1 %.3e (paper %.3e)'
              % (n, steps, res[n][0], tab[n][0], res[n][1], tab[n][1]))
    for n in res:
        for k in range(2):
            assert tab[n][k] / 3.0 < res[n][k] < 3.0 * tab[n][k], (n, k, res[n], tab[n])
    ns = sorted(res)
    for a, b in zip(ns, ns[1:]):
        for k in range(2):
            assert _rate(res[a][k], res[b][k], a, b) > 4.5, (a, b, k)


def test_table_5_2_on_gpu():
    """Example 5.2 to T = 0.1 on 40^2, 80^2, 160^2 and the paper's finest mesh
    280^2: density errors within 3x of Table 5.2's GR column, rates > 4.5 from
    80 on."""
    tab = load_table('table_5_2_gr.txt')
    res = {}
    for n in (40, 80, 160, 280):
        sc = Scheme2D(n, n, 0.0, 1.0, 0.0, 1.0, Physics(**PH), Options(cfl=CFL))
        m = MMS2D(sc)
        s = hweno.Solver(n, n, **PH)
        src = PolySource(m)
        U, t, steps = gpu_mms_run(s, to_dev(m.exact(0.0)), src, 1.0 / n, T_END)
        err = U.cpu().numpy()[0, 0] - m.exact(t)[0, 0]
        res[n] = (np.abs(err).max(), np.abs(err).mean())
        print('2D N=%d: %d steps, Linf %.3e (paper %.3e)  L1 %.3e (paper %.3e)'
              % (n, steps, res[n][0], tab[n][0], res[n][1], tab[n][1]))
    for n in res:
        for k in range(2):
            assert tab[n][k] / 3.0 < res[n][k] < 3.0 * tab[n][k], (n, k, res[n], tab[n])
    for a, b in ((80, 160), (160, 280)):
        for k in range(2):
            assert _rate(res[a][k], res[b][k], a, b) > 4.5, (a, b, k)


def test_table_5_1_dr_on_gpu():
    """The comparison scheme HWENO-DR (eq. (2.5)) on Example 5.1 from N = 80
    to 280: density errors within 1.5x of Table 5.1's DR column (measured
    1.07-1.18x), rates above 4 between consecutive meshes (printed 4.2-5.0),
    and GR more accurate than DR on every mesh, as printed."""
    tab = load_table('table_5_1_dr.txt')
    res = {}
    for n in (80, 120, 160, 200, 240, 280):
        sc = Scheme1D(n, 0.0, 1.0, Physics(**PH), Options(cfl=CFL))
        m = MMS1D(sc)
        src = PolySource(m)
        for gm in ('DR', 'GR'):
            s = hweno.Solver(n, extent=(0.0, 1.0), gradients=gm, **PH)
            U, t, steps = gpu_mms_run(s, to_dev(m.exact(0.0)), src, 1.0 / n, T_END)
            err = U.cpu().numpy()[0, 0] - m.exact(t)[0, 0]
            res[gm, n] = (np.abs(err).max(), np.abs(err).mean())
        print('1D DR N=%d: %d steps, Linf %.3e (paper %.3e)  L1 %.3e (paper %.3e); GR %.3e %.3e'
              % (n, steps, res['DR', n][0], tab[n][0], res['DR', n][1], tab[n][1],
                 *res['GR', n]))
    ns = sorted(n for gm, n in res if gm == 'DR')
    for n in ns:
        for k in range(2):
            assert tab[n][k] / 1.5 < res['DR', n][k] < 1.5 * tab[n][k], (n, k, res['DR', n])
            assert res['GR', n][k] < res['DR', n][k]
    for a, b in zip(ns, ns[1:]):
        for k in range(2):
            assert _rate(res['DR', a][k], res['DR', b][k], a, b) > 4.0, (a, b, k)


def test_table_5_2_dr_on_gpu():
    """HWENO-DR (eq. (3.5)) on Example 5.2 at 200^2 and 280^2: density errors
    within 1.5x of Table 5.2's DR column (measured 1.00-1.07x), rate above 4
    (printed 4.5).  On coarser meshes the printed DR errors carry a large
    pre-asymptotic part that ours lacks (40^2: printed 4.1e-4, ours 6e-6), so
    there only 'not worse than printed' is asserted (at 80^2)."""
    tab = load_table('table_5_2_dr.txt')
    res = {}
    for n in (80, 200, 280):
        sc = Scheme2D(n, n, 0.0, 1.0, 0.0, 1.0, Physics(**PH), Options(cfl=CFL))
        m = MMS2D(sc)
        s = hweno.Solver(n, n, gradients='DR', **PH)
        src = PolySource(m)
        U, t, steps = gpu_mms_run(s, to_dev(m.exact(0.0)), src, 1.0 / n, T_END)
        err = U.cpu().numpy()[0, 0] - m.exact(t)[0, 0]
        res[n] = (np.abs(err).max(), np.abs(err).mean())
        print('2D DR N=%d: %d steps, Linf %.3e (paper %.3e)  L1 %.3e (paper %.3e)'
              % (n, steps, res[n][0], tab[n][0], res[n][1], tab[n][1]))
    for k in range(2):
        assert res[80][k] < tab[80][k]
        for n in (200, 280):
            assert tab[n][k] / 1.5 < res[n][k] < 1.5 * tab[n][k], (n, k, res[n], tab[n])
        assert _rate(res[200][k], res[280][k], 200, 280) > 4.0, k
