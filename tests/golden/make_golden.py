#!/usr/bin/env python3
"""Write stored oracle results used by the GPU parity tests.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_golden.py
Writes c1_smooth_wave_t1.txt: the smooth 1D wave (N = 200 on [0, 2 pi),
gamma 1.4, Pr 0.72, mu 0.01, CFL 0.3, the paper's time-step rule with
b = 0.001) advanced to t = 1 by the oracle; and c2_viscous_riemann_n800.txt:
the density averages of the two viscous Riemann problems of the N = 2000
configuration (Sod to t = 0.2, the (1,-2,0.4)|(1,2,0.4) double rarefaction to
t = 0.15, mu 1e-3, Pr 0.72, outflow sides) computed by the oracle on 800
cells with the CFL step alone (CFL 0.3; the explicit viscous limit is not
reached there), a mesh-converged reference of the viscous solution.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rk  # noqa: E402
from oracle.common import Options, Physics  # noqa: E402
from oracle.scheme1d import Scheme1D  # noqa: E402
from paper_2608_10569_amd import workloads  # noqa: E402


def c1():
    U = workloads.smooth_wave_1d(200)
    s = Scheme1D(200, 0.0, 2 * np.pi, Physics(gamma=1.4, Pr=0.72, mu_ref=0.01),
                 Options(cfl=0.3, b_visc=0.001))
    U, t, n = rk.run(s, U, 0.0, 1.0, rule='paper')
    path = os.path.join(HERE, 'c1_smooth_wave_t1.txt')
    header = ('oracle: smooth 1D wave N=200 [0,2pi) periodic, gamma 1.4, Pr 0.72, mu 0.01, '
              'CFL 0.3, b 0.001, to t=1\nsteps %d t %.17g\nrows: (m, c) = (0,rho) (0,m) (0,E) '
              '(1,rho) (1,m) (1,E), columns: cells' % (n, t))
    np.savetxt(path, U.reshape(6, -1), fmt='%.17e', header=header)
    print('wrote', path, 'steps', n, 't', t)


def c2():
    cases = {'sod': ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2),
             'double_rarefaction': ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.15)}
    rows, names = [], []
    for name, (left, right, T) in cases.items():
        s = Scheme1D(800, 0.0, 1.0, Physics(gamma=1.4, Pr=0.72, mu_ref=1e-3),
                     Options(cfl=0.3, b_visc=0.0), bc=('outflow', 'outflow'))
        U, t, n = rk.run(s, workloads.riemann_1d(left, right, 800), 0.0, T)
        rows.append(U[0, 0])
        names.append('%s t=%.17g steps=%d' % (name, t, n))
    path = os.path.join(HERE, 'c2_viscous_riemann_n800.txt')
    header = ('oracle: viscous Riemann problems on [0,1], 800 cells, outflow, gamma 1.4, Pr 0.72, '
              'mu 1e-3, CFL 0.3 (no viscous step bound)\nrows: density cell averages of ' +
              '; '.join(names))
    np.savetxt(path, np.stack(rows), fmt='%.17e', header=header)
    print('wrote', path)


if __name__ == '__main__':
    which = sys.argv[1:] or ['c1', 'c2']
    if 'c1' in which:
        c1()
    if 'c2' in which:
        c2()
