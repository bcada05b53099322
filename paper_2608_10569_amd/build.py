"""Build libhweno.so (HIP, gfx950) in-tree.

Usage: python -m paper_2608_10569_amd.build   (or build() from Python)
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libhweno.so')
SOURCES = ['hweno2d.hip', 'hweno1d.hip', 'hweno2d_vjp.hip', 'hweno1d_vjp.hip', 'hweno_api.cpp']
ARCH = os.environ.get('HWENO_ARCH', 'gfx950')


def hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found')


def build(verbose=False):
    """Compile every source into paper_2608_10569_amd/libhweno.so."""
    tmp = LIB + '.tmp'
    cmd = [hipcc(), '--offload-arch=' + ARCH, '-O3', '-std=c++17', '-fPIC', '-shared',
           '-fvisibility=hidden', '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
           '-Wall', '-Wno-unused-function', '-Wno-unused-variable', '-o', tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(' '.join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    build(verbose='-v' in sys.argv)
    print(LIB)
