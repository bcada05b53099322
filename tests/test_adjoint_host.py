"""The library's adjoint building blocks on the CPU: every hand-written or
generated vector-Jacobian product of the device math against central
differences of the forward device function it reverses (both branches of the
LF wave-speed maximum included).  Compiles tests/host/adjoint_fd.cpp with g++
against a host stand-in of the HIP runtime header; no GPU needed."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), 'paper_2608_10569_amd', 'csrc')
CHECKS = ['p0_2d_T', 'p0_1d_T', 'xface_T', 'yface_T', 'vol_T', 'lgl_T', 'moment_xi_T',
          'moment_eta_T', 'moment1d_T', 'hweno2d_vjp', 'hweno2d_vjp_linear', 'hweno1d_vjp',
          'sobolev_2d_grad', 'sobolev_1d_grad', 'flux2_vjp_0', 'flux2_vjp_1', 'speed2_vjp_0',
          'speed2_vjp_1', 'pres2_vjp', 'prim2_vjp', 'eig2_vjp_0', 'eig2_vjp_1', 'flux1_vjp',
          'speed1_vjp', 'pres1_vjp', 'prim1_vjp', 'eig1_vjp']


@pytest.fixture(scope='module')
def report(tmp_path_factory):
    gxx = shutil.which('g++')
    if gxx is None:
        pytest.skip('g++ not available')
    exe = str(tmp_path_factory.mktemp('adjfd') / 'adjoint_fd')
    subprocess.run([gxx, '-O1', '-std=c++17', '-I', os.path.join(HERE, 'host'), '-I', CSRC,
                    os.path.join(HERE, 'host', 'adjoint_fd.cpp'), '-o', exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    lines = {}
    for ln in out.stdout.splitlines():
        parts = ln.split()
        if len(parts) >= 3 and parts[2] in ('OK', 'FAIL'):
            lines[parts[0]] = parts
    return out, lines


def test_every_adjoint_matches_finite_differences(report):
    out, lines = report
    assert set(CHECKS) <= set(lines), out.stdout
    bad = [ln for ln in lines.values() if ln[2] != 'OK']
    assert not bad and out.returncode == 0, out.stdout


def test_both_speed_branches_exercised(report):
    _, lines = report
    for name in ('speed2_vjp_0', 'speed2_vjp_1', 'speed1_vjp'):
        parts = lines[name]
        assert parts[3] == 'branches' and int(parts[4]) > 0 and int(parts[5]) > 0, parts
