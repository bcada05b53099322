"""MI355X-native FP64 HWENO-GR (arXiv 2608.10569): residual and SSP-RK3 on HIP.

The compute path is libhweno.so (HIP kernels for gfx950 behind the C ABI of
include/hweno.h); ``hweno`` is its ctypes binding, ``workloads`` the seeded
synthetic inputs, ``build`` the in-tree build.
"""

from . import workloads  # noqa: F401
