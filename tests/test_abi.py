"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and validates arguments on the host."""

import ctypes
import os
import re

import pytest

from paper_2608_10569_amd import hweno

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, 'include')):
        if fn.endswith('.h'):
            text = open(os.path.join(ROOT, 'include', fn)).read()
            names |= set(re.findall(r'HWENO_API\s+[\w\s\*]+?\b(hweno_\w+)\s*\(', text))
    return names


def test_library_exports_every_declared_symbol():
    L = hweno.lib()
    decl = declared_symbols()
    assert decl, 'no declarations found'
    assert decl == set(hweno.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def _args(**kw):
    g = hweno.Grid(2, 16, 8, 0.0, 1.0, 0.0, 0.5)
    ph = hweno.PhysicsC(1.4, 0.73, 1.0 / 200, 0.0, 1.0)
    b = hweno.Bcs()
    for s, k in enumerate((4, 4, 4, 3)):
        b.kind[s] = k
    o = hweno.default_options()
    for k, v in kw.items():
        for st in (g, ph, o):
            if hasattr(st, k):
                setattr(st, k, v)
    return g, ph, b, o


def _create(g, ph, b, o):
    h = ctypes.c_void_p()
    code = hweno.lib().hweno_create(ctypes.byref(g), ctypes.byref(ph), ctypes.byref(b),
                                    ctypes.byref(o), ctypes.byref(h))
    if code == 0:
        hweno.lib().hweno_destroy(h)
    return code


def test_default_options_are_the_papers():
    o = hweno.default_options()
    assert (o.cfl, o.b_visc, o.eps_pp, o.eps_weno, o.max_halvings) == (0.6, 0.001, 1e-12, 1e-8, 64)


def test_create_validates_arguments():
    assert _create(*_args()) == 0
    for kw in (dict(dim=3), dict(nx=3), dict(ny=2), dict(gamma=1.0), dict(Pr=0.0),
               dict(mu_ref=-1e-3), dict(T_ref=0.0), dict(cfl=0.0), dict(eps_pp=0.0),
               dict(eps_weno=-1.0), dict(max_halvings=-1), dict(x1=0.0),
               dict(b_visc=float('nan')), dict(t_final=float('nan'))):
        assert _create(*_args(**kw)) == 1, kw
    g, ph, b, o = _args()
    b.kind[0] = 0          # periodic paired with a wall
    assert _create(g, ph, b, o) == 1
    b.kind[0] = 7          # unknown kind
    assert _create(g, ph, b, o) == 1
    b.kind[0] = 2          # inflow with zero density
    assert _create(g, ph, b, o) == 1
    b.inflow[0][0], b.inflow[0][3] = 1.0, 1.0
    assert _create(g, ph, b, o) == 0


def test_workspace_and_state_errors_without_device():
    g, ph, b, o = _args()
    h = ctypes.c_void_p()
    L = hweno.lib()
    assert L.hweno_create(ctypes.byref(g), ctypes.byref(ph), ctypes.byref(b), ctypes.byref(o),
                          ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert L.hweno_workspace_bytes(h, ctypes.byref(n)) == 0
    assert n.value >= (16 + 8) * (8 + 8) * 300 * 8
    d = hweno.Diag()
    assert L.hweno_rk_step(h, 0.0, ctypes.byref(d)) == 3          # no workspace
    assert L.hweno_set_workspace(h, ctypes.c_void_p(0), n.value) == 1
    assert L.hweno_set_workspace(h, ctypes.c_void_p(4096), n.value - 1) == 3
    assert L.hweno_set_workspace(h, ctypes.c_void_p(4096 + 8), n.value) == 3   # misaligned
    assert L.hweno_destroy(h) == 0
    assert L.hweno_status_string(4).decode().startswith('stage inadmissible')
    assert L.hweno_status_string(7).decode() == 'host memory allocation failed'


def test_tile_defaults_and_validation_without_device():
    """A new 2D context uses the fused face-flux path; tile values outside the
    documented sets are refused (checked on the host, before any upload)."""
    g, ph, b, o = _args()
    h = ctypes.c_void_p()
    L = hweno.lib()
    assert L.hweno_create(ctypes.byref(g), ctypes.byref(ph), ctypes.byref(b), ctypes.byref(o),
                          ctypes.byref(h)) == 0
    t = hweno.TilesC()
    assert L.hweno_get_tiles(h, ctypes.byref(t)) == 0
    base = t.as_dict()
    assert base == dict(recon=32, grad=32, flux=0, order=0, xcd=1)
    for change, code in ((dict(flux=64), 0), (dict(flux=128), 0), (dict(recon=16, grad=32), 0),
                         (dict(order=1, xcd=0), 0), (dict(grad=0), 0), (dict(recon=64), 1),
                         (dict(grad=16), 1),
                         (dict(flux=32), 1), (dict(order=2), 1), (dict(xcd=2), 1)):
        v = dict(base, **change)
        tt = hweno.TilesC(v['recon'], v['grad'], v['flux'], v['order'], v['xcd'])
        assert L.hweno_set_tiles(h, ctypes.byref(tt)) == code, change
        if code == 0:
            got = hweno.TilesC()
            assert L.hweno_get_tiles(h, ctypes.byref(got)) == 0 and got.as_dict() == v
    assert L.hweno_destroy(h) == 0


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(hweno, 'LIB_PATH', str(tmp_path / 'missing.so'))
    monkeypatch.setattr(hweno, '_lib', None)
    with pytest.raises(ImportError):
        hweno.lib()


_ALLOC_FAIL_SCRIPT = r'''
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2608_10569_amd import hweno
L = hweno.lib()
ny = 40_000_000                       # one inflow state per boundary row: 1.28 GB
g = hweno.Grid(2, 8, ny, 0.0, 1.0, 0.0, 1.0)
ph = hweno.PhysicsC(1.4, 0.72, 1e-3, 0.0, 1.0)
b = hweno.Bcs()
for s, k in enumerate((2, 1, 3, 3)):
    b.kind[s] = k
b.inflow[0][0], b.inflow[0][3] = 1.0, 1.0
o = hweno.default_options()
h = ctypes.c_void_p()
assert L.hweno_create(ctypes.byref(g), ctypes.byref(ph), ctypes.byref(b), ctypes.byref(o),
                      ctypes.byref(h)) == 0
prim = np.zeros(4 * ny)               # untouched pages: address space only
vm = [l for l in open('/proc/self/status') if l.startswith('VmSize')][0]
cur = int(vm.split()[1]) * 1024
resource.setrlimit(resource.RLIMIT_AS, (cur + (256 << 20), resource.RLIM_INFINITY))
code = L.hweno_set_inflow_profile(h, 0, prim.ctypes.data_as(ctypes.c_void_p), ny)
resource.setrlimit(resource.RLIMIT_AS, (resource.RLIM_INFINITY, resource.RLIM_INFINITY))
print('status', code, L.hweno_status_string(code).decode())
# the context is still usable and the side keeps its constant state
assert L.hweno_set_inflow_profile(h, 0, None, ny) == 0
assert L.hweno_destroy(h) == 0
sys.exit(0 if code == 7 else 1)
'''


def test_host_allocation_failure_is_a_status():
    """A failed host allocation inside a call comes back as HWENO_E_NOMEM
    instead of an exception crossing the C ABI (which would abort the
    process): the library's copy of a 40M-row inflow profile is made to fail
    by capping the address space of a child process."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, '-c', _ALLOC_FAIL_SCRIPT, ROOT], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert 'status 7 host memory allocation failed' in r.stdout


def test_noalloc_residual_host_checks_without_device():
    """The allocation-free residual refuses, before touching a device, a grid
    whose residual does not fit its static buffer (1776 bytes per ghosted
    cell in 2D: up to 380 x 380 cells), a batch context and NULL arrays."""
    L = hweno.lib()
    dummy = ctypes.c_void_p(4096)     # never dereferenced: the checks come first
    big = hweno.Grid(2, 381, 381, 0.0, 1.0, 0.0, 1.0)
    fits = hweno.Grid(2, 300, 300, 0.0, 1.0, 0.0, 1.0)
    assert 1776 * 389 * 389 > hweno.NOALLOC_BYTES > 1776 * 388 * 388 + 4096
    ph = hweno.PhysicsC(1.4, 0.72, 0.01, 0.0, 1.0)
    b = hweno.Bcs()
    o = hweno.default_options()
    h = ctypes.c_void_p()
    assert L.hweno_create(ctypes.byref(big), ctypes.byref(ph), ctypes.byref(b), ctypes.byref(o),
                          ctypes.byref(h)) == 0
    assert L.hweno_residual_noalloc(h, dummy, dummy, dummy, None) == 3
    assert L.hweno_residual_noalloc(h, None, dummy, dummy, None) == 1
    assert L.hweno_destroy(h) == 0
    g1 = hweno.Grid(1, 800000, 1, 0.0, 1.0, 0.0, 1.0)      # 1D: 352 bytes per ghosted cell
    assert L.hweno_create(ctypes.byref(g1), ctypes.byref(ph), ctypes.byref(b), ctypes.byref(o),
                          ctypes.byref(h)) == 0
    assert L.hweno_residual_noalloc(h, dummy, dummy, dummy, None) == 3
    assert L.hweno_destroy(h) == 0
    gs = (hweno.Grid * 2)(fits, fits)
    phs = (hweno.PhysicsC * 2)(ph, ph)
    bs = (hweno.Bcs * 2)(b, b)
    os_ = (hweno.OptionsC * 2)(o, o)
    assert L.hweno_batch_create(2, gs, phs, bs, os_, ctypes.byref(h)) == 0
    assert L.hweno_residual_noalloc(h, dummy, dummy, dummy, None) == 1
    assert L.hweno_destroy(h) == 0
