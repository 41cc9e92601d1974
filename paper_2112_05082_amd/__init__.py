"""MI355X-native retrieved matvec of R3M-HPE (arXiv 2112.05082).

The library ``libr3m.so`` (HIP, gfx950) exposes the C ABI of include/r3m.h;
``r3m`` is its ctypes binding and ``pipeline`` builds device stores and
batches from workload descriptions using only those entry points.
"""
from . import r3m  # noqa: F401
