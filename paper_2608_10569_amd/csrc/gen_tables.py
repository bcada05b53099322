#!/usr/bin/env python3
"""Generate ``hweno_gen.h``: exact-rational stencil code for the HIP kernels.

Derives, with sympy in exact rational arithmetic, the maps of the unified
stencil HWENO reconstruction (Appendix A of the paper) and writes them as
straight-line device code with only the non-zero terms:

* 1D: the quartic p0 fixed by the averages of cells i-1, i, i+1 and the first
  moments of cells i-1, i+1 (eq. (A.1)) -> its five monomial coefficients.
* 2D: the quartic p0 of eq. (A.4): nine averages, the xi-moments of cells 4
  and 6 and the eta-moments of cells 2 and 8 imposed exactly, the other four
  first moments in the least-squares sense.  Derived by solving the exact
  conditions for 13 coefficients in terms of 2 free ones and minimising the
  least-squares residual over those two.
* The smoothness indicator of a quartic: the Sobolev sum over all
  derivatives of order 1..4 of the squared derivative integrated over the
  scaled cell, as a quadratic form in the coefficients.

Monomial order (both here and in the kernels): xi^a eta^b listed by total
degree, then by increasing b: (0,0),(1,0),(0,1),(2,0),(1,1),(0,2),(3,0),...

Run:  python gen_tables.py  (writes hweno_gen.h next to this file)
"""

import os
from collections import defaultdict

import sympy as sp

HERE = os.path.dirname(os.path.abspath(__file__))
MONOS2 = [(tot - b, b) for tot in range(5) for b in range(tot + 1)]
H = sp.Rational(1, 2)
xi, eta = sp.symbols('xi eta')


def cell_avg(expr, dx, dy):
    return sp.integrate(sp.integrate(expr, (xi, dx - H, dx + H)), (eta, dy - H, dy + H))


def cell_mom(expr, dx, dy, var):
    w = (xi - dx) if var == 'xi' else (eta - dy)
    return sp.integrate(sp.integrate(expr * w, (xi, dx - H, dx + H)), (eta, dy - H, dy + H))


def fmt(r):
    v = float(r)
    s = repr(v)
    if 'e' not in s and '.' not in s:
        s += '.0'
    return s


def linear_code(target, expr, inputs):
    """target = sum_k q_k * inputs_k, grouped by equal |q| to save products."""
    expr = sp.expand(expr)
    groups = defaultdict(list)
    for s in inputs:
        q = expr.coeff(s)
        if q != 0:
            groups[abs(q)].append(('+' if q > 0 else '-', s))
    terms = []
    for q, members in sorted(groups.items(), key=lambda t: -float(t[0])):
        inner = ' '.join('%s %s' % (sg, str(s)) for sg, s in members).lstrip('+ ').strip()
        if inner.startswith('- '):
            inner = '-' + inner[2:]
        terms.append('%s * (%s)' % (fmt(q), inner))
    if not terms:
        return '    %s = 0.0;' % target
    return '    %s = %s;' % (target, '\n        + '.join(terms))


def derive_1d():
    a = sp.symbols('c0:5')
    p = sum(a[k] * xi ** k for k in range(5))
    ins = sp.symbols('um uc up vm vp')
    eqs = [sp.integrate(p, (xi, d - H, d + H)) - v for d, v in zip((-1, 0, 1), ins[:3])]
    eqs += [sp.integrate(p * (xi - d), (xi, d - H, d + H)) - v for d, v in zip((-1, 1), ins[3:])]
    sol = sp.solve(eqs, a, dict=True)[0]
    coeffs = [sp.expand(sol[a[k]]) for k in range(5)]
    # self-check: P4 data reproduced exactly
    t = sp.symbols('t0:5')
    q = sum(t[k] * xi ** k for k in range(5))
    data = {ins[0]: sp.integrate(q, (xi, -1 - H, -1 + H)), ins[1]: sp.integrate(q, (xi, -H, H)),
            ins[2]: sp.integrate(q, (xi, 1 - H, 1 + H)),
            ins[3]: sp.integrate(q * (xi + 1), (xi, -1 - H, -1 + H)),
            ins[4]: sp.integrate(q * (xi - 1), (xi, 1 - H, 1 + H))}
    for k in range(5):
        assert sp.simplify(coeffs[k].subs(data) - t[k]) == 0
    return ins, coeffs


def derive_2d():
    c = {m: sp.Symbol('c_%d_%d' % m) for m in MONOS2}
    p = sum(c[m] * xi ** m[0] * eta ** m[1] for m in MONOS2)
    off = {k + 1: (k % 3 - 1, k // 3 - 1) for k in range(9)}
    A = sp.symbols('a1:10')
    X = {k: sp.Symbol('x%d' % k) for k in (2, 4, 6, 8)}
    Y = {k: sp.Symbol('y%d' % k) for k in (2, 4, 6, 8)}
    exact = [cell_avg(p, *off[k]) - A[k - 1] for k in range(1, 10)]
    exact += [cell_mom(p, *off[k], 'xi') - X[k] for k in (4, 6)]
    exact += [cell_mom(p, *off[k], 'eta') - Y[k] for k in (2, 8)]
    lsq = [cell_mom(p, *off[k], 'xi') - X[k] for k in (2, 8)]
    lsq += [cell_mom(p, *off[k], 'eta') - Y[k] for k in (4, 6)]
    unknowns = [c[m] for m in MONOS2]
    sol = sp.solve(exact, unknowns, dict=True)[0]
    free = [u for u in unknowns if u not in sol]
    assert len(free) == 2, free
    J = sum(sp.expand(r.subs(sol)) ** 2 for r in lsq)
    fs = sp.solve([sp.diff(J, f) for f in free], free, dict=True)[0]
    coeffs = {}
    for m in MONOS2:
        e = c[m].subs(sol).subs(fs) if c[m] in sol else fs[c[m]]
        coeffs[m] = sp.expand(e)
    inputs = list(A) + [X[k] for k in (2, 4, 6, 8)] + [Y[k] for k in (2, 4, 6, 8)]
    # self-check: P4 data reproduced exactly
    t = {m: sp.Symbol('t_%d_%d' % m) for m in MONOS2}
    q = sum(t[m] * xi ** m[0] * eta ** m[1] for m in MONOS2)
    data = {A[k - 1]: cell_avg(q, *off[k]) for k in range(1, 10)}
    data.update({X[k]: cell_mom(q, *off[k], 'xi') for k in (2, 4, 6, 8)})
    data.update({Y[k]: cell_mom(q, *off[k], 'eta') for k in (2, 4, 6, 8)})
    for m in MONOS2:
        assert sp.simplify(coeffs[m].subs(data) - t[m]) == 0
    return inputs, coeffs


def sobolev_form(monos, ndim):
    """Quadratic form G with beta = sum_{1<=|alpha|<=4} int (D^alpha p)^2."""
    syms = [sp.Symbol('k%d' % i) for i in range(len(monos))]
    if ndim == 1:
        p = sum(s * xi ** m for s, m in zip(syms, monos))
        beta = sum(sp.integrate(sp.diff(p, xi, o) ** 2, (xi, -H, H)) for o in range(1, 5))
    else:
        p = sum(s * xi ** m[0] * eta ** m[1] for s, m in zip(syms, monos))
        beta = 0
        for ax in range(5):
            for ay in range(5 - ax):
                if ax + ay == 0:
                    continue
                d = p
                if ax:
                    d = sp.diff(d, xi, ax)
                if ay:
                    d = sp.diff(d, eta, ay)
                beta += sp.integrate(sp.integrate(d ** 2, (xi, -H, H)), (eta, -H, H))
    return sp.expand(beta), syms


def quad_code(target, beta, syms, names):
    lines = ['    double %s = 0.0;' % target]
    poly = sp.Poly(beta, *syms)
    terms = []
    for i, si in enumerate(syms):
        for j in range(i, len(syms)):
            mono = [0] * len(syms)
            mono[i] += 1
            mono[j] += 1
            q = poly.coeff_monomial(tuple(mono))
            if q != 0:
                terms.append((q, names[i], names[j]))
    for q, ni, nj in terms:
        lines.append('    %s = fma(%s, %s * %s, %s);' % (target, fmt(q), ni, nj, target))
    return '\n'.join(lines)


def main():
    out = []
    out.append('// Generated by gen_tables.py from exact rational derivations of the')
    out.append('// unified-stencil HWENO candidate p0 (Appendix A of the paper).  Do not edit.')
    out.append('#pragma once')
    out.append('')
    out.append('namespace hweno_gen {')
    out.append('')
    # 1D
    ins1, co1 = derive_1d()
    out.append('// 1D quartic p0, eq. (A.1).  a = {ubar_{i-1}, ubar_i, ubar_{i+1}, vbar_{i-1},')
    out.append('// vbar_{i+1}} -> c[k], coefficient of xi^k.')
    out.append('__device__ __forceinline__ void p0_1d(const double* __restrict__ a, double* __restrict__ c) {')
    out.append('    const double um = a[0], uc = a[1], up = a[2], vm = a[3], vp = a[4];')
    for k in range(5):
        out.append(linear_code('c[%d]' % k, co1[k], ins1))
    out.append('}')
    out.append('')
    beta1, syms1 = sobolev_form(list(range(5)), 1)
    out.append('// Sobolev smoothness indicator of a 1D quartic with coefficients c.')
    out.append('__device__ __forceinline__ double sobolev_1d(const double* __restrict__ c) {')
    out.append(quad_code('b', beta1, syms1, ['c[%d]' % k for k in range(5)]))
    out.append('    return b;')
    out.append('}')
    out.append('')
    # 2D
    ins2, co2 = derive_2d()
    names2 = {s: ('a[%d]' % i) for i, s in enumerate(ins2)}
    out.append('// 2D quartic p0, eq. (A.4), constrained least squares.  a[0..8] = averages of')
    out.append('// cells 1..9 (row-major from (i-1,j-1)), a[9..12] = xi-moments of cells')
    out.append('// 2,4,6,8, a[13..16] = eta-moments of cells 2,4,6,8 -> c[15] in monomial order.')
    out.append('__device__ __forceinline__ void p0_2d(const double* __restrict__ a, double* __restrict__ c) {')
    for i, s in enumerate(ins2):
        out.append('    const double %s = a[%d];' % (s, i))
    for k, m in enumerate(MONOS2):
        out.append(linear_code('c[%d]' % k, co2[m], ins2))
    out.append('}')
    out.append('')
    beta2, syms2 = sobolev_form(MONOS2, 2)
    out.append('// Sobolev smoothness indicator of a 2D quartic with coefficients c.')
    out.append('__device__ __forceinline__ double sobolev_2d(const double* __restrict__ c) {')
    out.append(quad_code('b', beta2, syms2, ['c[%d]' % k for k in range(15)]))
    out.append('    return b;')
    out.append('}')
    out.append('')
    out.append('}  // namespace hweno_gen')
    del names2
    path = os.path.join(HERE, 'hweno_gen.h')
    with open(path, 'w') as f:
        f.write('\n'.join(out) + '\n')
    print('wrote', path)


if __name__ == '__main__':
    main()
