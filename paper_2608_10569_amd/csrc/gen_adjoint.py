#!/usr/bin/env python3
"""Generate ``hweno_gen_adj.h``: straight-line code for the reverse-mode
(vector-Jacobian) pieces of the HWENO-GR residual.

* transposed stencil maps of the quartic candidate p0 (1D, 2D) and the
  gradient of its Sobolev smoothness indicator;
* transposed point evaluations (x-face, y-face, volume Gauss points, own-cell
  moments; 1D LGL points);
* vector-Jacobian products of the pointwise physics of eqs. (2.1), (2.3),
  (3.1), (3.3): total fluxes, the two branches of the Lax-Friedrichs speed
  (|u_n| + c and the positivity bound), primitives (u, v, e), pressure;
* vector-Jacobian products of the characteristic bases (rows of L = R^-1
  and of R) with respect to the cell average.

Derivatives are taken symbolically (sympy) and emitted after common
subexpression elimination.  The forward maps are re-derived here from the
moment conditions (Appendix A) exactly as in gen_tables.py.

Run:  python gen_adjoint.py  (writes hweno_gen_adj.h next to this file)
"""

import os

import sympy as sp
from sympy.printing.c import C99CodePrinter

from gen_tables import MONOS2, derive_1d, derive_2d, fmt, sobolev_form

HERE = os.path.dirname(os.path.abspath(__file__))
S15 = sp.sqrt(15) / 10
T5 = sp.sqrt(5) / 10
H = sp.Rational(1, 2)


class CPrinter(C99CodePrinter):
    def _print_Float(self, expr):
        return fmt(expr)

    def _print_Rational(self, expr):
        return fmt(expr)

    def _print_Integer(self, expr):
        return fmt(expr)

    def _print_Pow(self, expr):
        b, e = expr.as_base_exp()
        x = '(%s)' % self._print(b)     # the base always in parentheses
        if e == 2:
            return '(%s * %s)' % (x, x)
        if e == -1:
            return '(1.0 / %s)' % x
        if e == -2:
            return '(1.0 / (%s * %s))' % (x, x)
        if e == 3:
            return '(%s * %s * %s)' % (x, x, x)
        if e == sp.Rational(1, 2):
            return 'sqrt%s' % x
        if e == -sp.Rational(1, 2):
            return '(1.0 / sqrt%s)' % x
        if e == sp.Rational(3, 2):
            return '(%s * sqrt%s)' % (x, x)
        if e == -sp.Rational(3, 2):
            return '(1.0 / (%s * sqrt%s))' % (x, x)
        return super()._print_Pow(expr)


PR = CPrinter()


def emit(targets, exprs, accumulate=True, indent='    '):
    """CSE + C code: target[i] (+)= exprs[i]."""
    reps, red = sp.cse([sp.expand(e) if e.is_polynomial() else e for e in exprs],
                       symbols=sp.numbered_symbols('t'))
    lines = []
    for sym, val in reps:
        lines.append('%sconst double %s = %s;' % (indent, sym, PR.doprint(val)))
    for t, e in zip(targets, red):
        if e == 0:
            if not accumulate:
                lines.append('%s%s = 0.0;' % (indent, t))
            continue
        lines.append('%s%s %s %s;' % (indent, t, '+=' if accumulate else '=', PR.doprint(e)))
    return lines


def linear_T(name, ins, outs_exprs, nin_name='cb', nout_name='ab'):
    """ab[s] = sum_k d outs_k / d ins_s * cb[k]   (transpose of a linear map)."""
    cb = sp.symbols('%s0:%d' % (nin_name, len(outs_exprs)))
    res = []
    for s in ins:
        res.append(sum(sp.diff(e, s) * cb[k] for k, e in enumerate(outs_exprs)))
    L = ['__device__ __forceinline__ void %s(const double* __restrict__ %s, '
         'double* __restrict__ %s) {' % (name, nin_name, nout_name)]
    for k in range(len(outs_exprs)):
        L.append('    const double %s%d = %s[%d];' % (nin_name, k, nin_name, k))
    L += emit(['%s[%d]' % (nout_name, s) for s in range(len(ins))], res, accumulate=False)
    L.append('}')
    return L


def point_eval_T(name, pts, monos, ndim):
    """Cb[k] += sum_p phi_k(x_p) yb[p] (transpose of the point evaluation)."""
    yb = sp.symbols('yb0:%d' % len(pts))
    res = []
    for m in monos:
        acc = 0
        for p, x in enumerate(pts):
            if ndim == 1:
                v = x ** m
            else:
                v = x[0] ** m[0] * x[1] ** m[1]
            acc += sp.nsimplify(v) * yb[p]
        res.append(acc)
    L = ['__device__ __forceinline__ void %s(const double* __restrict__ yb, '
         'double* __restrict__ Cb) {' % name]
    for p in range(len(pts)):
        L.append('    const double yb%d = yb[%d];' % (p, p))
    L += emit(['Cb[%d]' % k for k in range(len(monos))], res, accumulate=True)
    L.append('}')
    return L


def vjp_func(name, args_decl, inputs, outputs, out_bars, in_targets, pre=()):
    """Vector-Jacobian product: in_targets[i] += sum_j outbar_j d out_j / d in_i."""
    res = [sum(sp.diff(o, x) * ob for o, ob in zip(outputs, out_bars)) for x in inputs]
    L = ['__device__ __forceinline__ void %s(%s) {' % (name, args_decl)]
    L += ['    ' + p for p in pre]
    L += emit(in_targets, res, accumulate=True)
    L.append('}')
    return L


def physics():
    L = []
    r, m, n, E = sp.symbols('r m n E', positive=True)
    s = sp.symbols('s0:6')
    mu, gam, gm1, Pr = sp.symbols('mu gam gm1 Pr', positive=True)
    sgu, sgq = sp.symbols('sgu sgq')
    pre = ['const double gam = K.gamma, gm1 = K.gm1, Pr = K.Pr;',
           'const double r = U[0], m = U[1], n = U[2], E = U[3];',
           'const double s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3], s4 = s[4], s5 = s[5];']
    u, v = m / r, n / r
    p = gm1 * (E - (m * m + n * n) / (2 * r))
    txx = mu * (sp.Rational(4, 3) * s[0] - sp.Rational(2, 3) * s[3])
    txy = mu * (s[1] + s[2])
    tyy = mu * (sp.Rational(4, 3) * s[3] - sp.Rational(2, 3) * s[0])
    kq = gam * mu / Pr
    fx = [m, m * u + p - txx, n * u - txy, (E + p) * u - (txx * u + txy * v + kq * s[4])]
    gy = [n, m * v - txy, n * v + p - tyy, (E + p) * v - (txy * u + tyy * v + kq * s[5])]
    fb = sp.symbols('fb0:4')
    ins = [r, m, n, E] + list(s) + [mu]
    tg = ['Ub[0]', 'Ub[1]', 'Ub[2]', 'Ub[3]'] + ['sb[%d]' % z for z in range(6)] + ['mub']
    decl = ('const Consts& K, const double* __restrict__ U, const double* __restrict__ s, '
            'double mu, const double* __restrict__ fbv, double* __restrict__ Ub, '
            'double* __restrict__ sb, double& mub')
    for d, fl in ((0, fx), (1, gy)):
        L += vjp_func('flux2_vjp_%d' % d, decl, ins, fl, fb, tg,
                      pre + ['const double fb0 = fbv[0], fb1 = fbv[1], fb2 = fbv[2], fb3 = fbv[3];'])
        L.append('')
    # LF speed branches
    e = p / (gm1 * r)
    for d in (0, 1):
        un = u if d == 0 else v
        ac = sgu * un + sp.sqrt(gam * p / r)
        q = kq * s[4 + d]
        t2 = (txx - p) ** 2 + txy ** 2 if d == 0 else txy ** 2 + (tyy - p) ** 2
        r2e = r * r * e
        bpp = sgu * un + (sp.sqrt(r * r * q * q + 2 * r2e * t2) + r * sgq * q) / (2 * r2e)
        yb = sp.Symbol('yb')
        declA = ('const Consts& K, const double* __restrict__ U, double sgu, double yb, '
                 'double* __restrict__ Ub')
        L += vjp_func('speed2_ac_vjp_%d' % d, declA, [r, m, n, E], [ac], [yb],
                      ['Ub[0]', 'Ub[1]', 'Ub[2]', 'Ub[3]'],
                      ['const double gam = K.gamma, gm1 = K.gm1;',
                       'const double r = U[0], m = U[1], n = U[2], E = U[3];'])
        L.append('')
        declB = ('const Consts& K, const double* __restrict__ U, const double* __restrict__ s, '
                 'double mu, double sgu, double sgq, double yb, double* __restrict__ Ub, '
                 'double* __restrict__ sb, double& mub')
        L += vjp_func('speed2_bpp_vjp_%d' % d, declB, ins, [bpp], [yb], tg, pre)
        L.append('')
    # primitives and pressure
    wv = [u, v, E / r - (u * u + v * v) / 2]
    wb = sp.symbols('wb0:3')
    L += vjp_func('prim2_vjp', 'const double* __restrict__ U, const double* __restrict__ wbv, '
                  'double* __restrict__ Ub', [r, m, n, E], wv, wb,
                  ['Ub[0]', 'Ub[1]', 'Ub[2]', 'Ub[3]'],
                  ['const double r = U[0], m = U[1], n = U[2], E = U[3];',
                   'const double wb0 = wbv[0], wb1 = wbv[1], wb2 = wbv[2];'])
    L.append('')
    yb = sp.Symbol('yb')
    L += vjp_func('pres2_vjp', 'const Consts& K, const double* __restrict__ U, double yb, '
                  'double* __restrict__ Ub', [r, m, n, E], [p], [yb],
                  ['Ub[0]', 'Ub[1]', 'Ub[2]', 'Ub[3]'],
                  ['const double gm1 = K.gm1;',
                   'const double r = U[0], m = U[1], n = U[2], E = U[3];'])
    L.append('')
    # 1D
    ux, ex = sp.symbols('ux ex')
    u1 = m / r
    p1 = gm1 * (E - m * m / (2 * r))
    tau = sp.Rational(4, 3) * mu * ux
    q1 = -gam * mu * ex / Pr
    f1 = [m, m * u1 + p1 - tau, (E + p1) * u1 - (tau * u1 - q1)]
    pre1 = ['const double gam = K.gamma, gm1 = K.gm1, Pr = K.Pr;',
            'const double r = U[0], m = U[1], E = U[2];']
    ins1 = [r, m, E, ux, ex, mu]
    tg1 = ['Ub[0]', 'Ub[1]', 'Ub[2]', 'uxb', 'exb', 'mub']
    decl1 = ('const Consts& K, const double* __restrict__ U, double ux, double ex, double mu, '
             'const double* __restrict__ fbv, double* __restrict__ Ub, double& uxb, double& exb, '
             'double& mub')
    L += vjp_func('flux1_vjp', decl1, ins1, f1, fb[:3], tg1,
                  pre1 + ['const double fb0 = fbv[0], fb1 = fbv[1], fb2 = fbv[2];'])
    L.append('')
    ac1 = sgu * u1 + sp.sqrt(gam * p1 / r)
    L += vjp_func('speed1_ac_vjp', 'const Consts& K, const double* __restrict__ U, double sgu, '
                  'double yb, double* __restrict__ Ub', [r, m, E], [ac1], [yb],
                  ['Ub[0]', 'Ub[1]', 'Ub[2]'],
                  ['const double gam = K.gamma, gm1 = K.gm1;',
                   'const double r = U[0], m = U[1], E = U[2];'])
    L.append('')
    e1 = p1 / (gm1 * r)
    r2e1 = r * r * e1
    bpp1 = sgu * u1 + (sp.sqrt(r * r * q1 * q1 + 2 * r2e1 * (tau - p1) ** 2) + r * sgq * q1) / (2 * r2e1)
    L += vjp_func('speed1_bpp_vjp', 'const Consts& K, const double* __restrict__ U, double ux, '
                  'double ex, double mu, double sgu, double sgq, double yb, '
                  'double* __restrict__ Ub, double& uxb, double& exb, double& mub',
                  ins1, [bpp1], [yb], tg1, pre1)
    L.append('')
    w1 = [u1, E / r - u1 * u1 / 2]
    L += vjp_func('prim1_vjp', 'const double* __restrict__ U, const double* __restrict__ wbv, '
                  'double* __restrict__ Ub', [r, m, E], w1, wb[:2], ['Ub[0]', 'Ub[1]', 'Ub[2]'],
                  ['const double r = U[0], m = U[1], E = U[2];',
                   'const double wb0 = wbv[0], wb1 = wbv[1];'])
    L.append('')
    L += vjp_func('pres1_vjp', 'const Consts& K, const double* __restrict__ U, double yb, '
                  'double* __restrict__ Ub', [r, m, E], [p1], [yb], ['Ub[0]', 'Ub[1]', 'Ub[2]'],
                  ['const double gm1 = K.gm1;', 'const double r = U[0], m = U[1], E = U[2];'])
    L.append('')
    return L


def eigen():
    """VJP of row k of L and row k of R with respect to the cell average."""
    L = []
    r, m, n, E = sp.symbols('r m n E', positive=True)
    gam, gm1 = sp.symbols('gam gm1', positive=True)
    u, v = m / r, n / r
    q2 = u * u + v * v
    p = gm1 * (E - r * q2 / 2)
    c = sp.sqrt(gam * p / r)
    Hh = (E + p) / r
    b1 = gm1 / (c * c)
    b2 = b1 * q2 / 2
    lb = sp.symbols('lb0:4')
    rb = sp.symbols('rb0:4')
    for b in (0, 1):
        un, ut = (u, v) if b == 0 else (v, u)
        i_n, i_t = (1, 2) if b == 0 else (2, 1)
        Lrows = []
        for k in range(4):
            row = [0] * 4
            if k == 0:
                row[0], row[i_n], row[i_t], row[3] = (b2 + un / c) / 2, -(b1 * un + 1 / c) / 2, -b1 * ut / 2, b1 / 2
            elif k == 1:
                row[0], row[i_n], row[i_t], row[3] = 1 - b2, b1 * un, b1 * ut, -b1
            elif k == 2:
                row[0], row[i_n], row[i_t], row[3] = -ut, 0, 1, 0
            else:
                row[0], row[i_n], row[i_t], row[3] = (b2 - un / c) / 2, (1 / c - b1 * un) / 2, -b1 * ut / 2, b1 / 2
            Lrows.append(row)
        cols = [[1, un - c, ut, Hh - un * c], [1, un, ut, q2 / 2], [0, 0, 1, ut],
                [1, un + c, ut, Hh + un * c]]
        # R[comp][field]: reorder the (rho, m_n, m_t, E) column entries to (rho, m, n, E)
        R = [[0] * 4 for _ in range(4)]
        for f in range(4):
            col = cols[f]
            R[0][f] = col[0]
            R[i_n][f] = col[1]
            R[i_t][f] = col[2]
            R[3][f] = col[3]
        # self-check: L R = I
        Lm = sp.Matrix(Lrows)
        Rm = sp.Matrix(R)
        chk = sp.simplify((Lm * Rm).subs({gm1: sp.Rational(2, 5), gam: sp.Rational(7, 5),
                                          r: sp.Rational(3, 2), m: sp.Rational(1, 3),
                                          n: -sp.Rational(1, 5), E: 3}))
        assert chk == sp.eye(4), chk
        L.append('// d/d ubar of (row k of L) . lb + (row k of R) . rb, basis %d' % b)
        L.append('__device__ __forceinline__ void eig2_vjp_%d(const Consts& K, '
                 'const double* __restrict__ Ub, int k, const double* __restrict__ lbv, '
                 'const double* __restrict__ rbv, double* __restrict__ ub) {' % b)
        L.append('    const double gam = K.gamma, gm1 = K.gm1;')
        L.append('    const double r = Ub[0], m = Ub[1], n = Ub[2], E = Ub[3];')
        L.append('    const double lb0 = lbv[0], lb1 = lbv[1], lb2 = lbv[2], lb3 = lbv[3];')
        L.append('    const double rb0 = rbv[0], rb1 = rbv[1], rb2 = rbv[2], rb3 = rbv[3];')
        L.append('    switch (k) {')
        for k in range(4):
            obj = sum(Lrows[k][cc] * lb[cc] for cc in range(4)) + sum(R[k][f] * rb[f] for f in range(4))
            L.append('    case %d: {' % k)
            L += emit(['ub[%d]' % j for j in range(4)], [sp.diff(obj, x) for x in (r, m, n, E)],
                      indent='        ')
            L.append('        break; }')
        L.append('    }')
        L.append('}')
        L.append('')
    # 1D: full L, R
    u1 = m / r
    p1 = gm1 * (E - m * m / (2 * r))
    c1 = sp.sqrt(gam * p1 / r)
    H1 = (E + p1) / r
    b11 = gm1 / (c1 * c1)
    b21 = b11 * u1 * u1 / 2
    L1 = [[(b21 + u1 / c1) / 2, -(b11 * u1 + 1 / c1) / 2, b11 / 2],
          [1 - b21, b11 * u1, -b11],
          [(b21 - u1 / c1) / 2, (1 / c1 - b11 * u1) / 2, b11 / 2]]
    R1 = [[1, 1, 1], [u1 - c1, u1, u1 + c1], [H1 - u1 * c1, u1 * u1 / 2, H1 + u1 * c1]]
    lb9 = sp.symbols('lb0:9')
    rb9 = sp.symbols('rb0:9')
    obj = sum(L1[i][j] * lb9[3 * i + j] for i in range(3) for j in range(3)) + \
        sum(R1[i][j] * rb9[3 * i + j] for i in range(3) for j in range(3))
    L.append('// d/d ubar of sum L[i][j] lb[3i+j] + R[i][j] rb[3i+j] (1D)')
    L.append('__device__ __forceinline__ void eig1_vjp(const Consts& K, const double* __restrict__ Ub, '
             'const double* __restrict__ lbv, const double* __restrict__ rbv, '
             'double* __restrict__ ub) {')
    L.append('    const double gam = K.gamma, gm1 = K.gm1;')
    L.append('    const double r = Ub[0], m = Ub[1], E = Ub[2];')
    for i in range(9):
        L.append('    const double lb%d = lbv[%d], rb%d = rbv[%d];' % (i, i, i, i))
    L += emit(['ub[%d]' % j for j in range(3)], [sp.diff(obj, x) for x in (r, m, E)])
    L.append('}')
    L.append('')
    return L


def main():
    out = ['// Generated by gen_adjoint.py (sympy derivatives of the HWENO-GR pointwise maps).',
           '// Do not edit.', '#pragma once', '', 'namespace hw {', 'namespace adj {', '']
    ins1, co1 = derive_1d()
    out += linear_T('p0_1d_T', list(ins1), co1)
    out.append('')
    ins2, co2 = derive_2d()
    out += linear_T('p0_2d_T', list(ins2), [co2[m] for m in MONOS2])
    out.append('')
    beta1, syms1 = sobolev_form(list(range(5)), 1)
    out += ['// gradient of the 1D Sobolev indicator: g[k] = d beta / d c[k]',
            '__device__ __forceinline__ void sobolev_1d_grad(const double* __restrict__ c, '
            'double* __restrict__ g) {']
    out += ['    const double k%d = c[%d];' % (i, i) for i in range(5)]
    out += emit(['g[%d]' % i for i in range(5)], [sp.diff(beta1, x) for x in syms1],
                accumulate=False)
    out += ['}', '']
    beta2, syms2 = sobolev_form(MONOS2, 2)
    out += ['// gradient of the 2D Sobolev indicator: g[k] = d beta / d c[k]',
            '__device__ __forceinline__ void sobolev_2d_grad(const double* __restrict__ c, '
            'double* __restrict__ g) {']
    out += ['    const double k%d = c[%d];' % (i, i) for i in range(15)]
    out += emit(['g[%d]' % i for i in range(15)], [sp.diff(beta2, x) for x in syms2],
                accumulate=False)
    out += ['}', '']
    G = [-S15, 0, S15]
    xface = [(-H, G[g]) for g in range(3)] + [(H, G[g]) for g in range(3)]
    yface = [(G[g], -H) for g in range(3)] + [(G[g], H) for g in range(3)]
    vol = [(G[g], G[h]) for h in range(3) for g in range(3)]
    out += point_eval_T('xface_T', xface, MONOS2, 2) + ['']
    out += point_eval_T('yface_T', yface, MONOS2, 2) + ['']
    out += point_eval_T('vol_T', vol, MONOS2, 2) + ['']
    out += point_eval_T('lgl_T', [-H, -T5, T5, H], list(range(5)), 1) + ['']
    out += physics()
    out += eigen()
    out += ['}  // namespace adj', '}  // namespace hw']
    path = os.path.join(HERE, 'hweno_gen_adj.h')
    with open(path, 'w') as f:
        f.write('\n'.join(out) + '\n')
    print('wrote', path)


if __name__ == '__main__':
    main()
