"""MI355X-native random batch Ewald (RBE) for periodic Coulomb systems.

The compute path is the C-ABI library ``librbe.so`` (hand-written HIP kernels
for gfx950, declared in ``include/rbe.h``); :mod:`paper_2010_01559_amd.rbe`
is a thin ctypes binding over it that passes torch device pointers and the
current HIP stream.  Importing this package loads nothing; the library is
loaded on first use and the binding raises if it is missing.
"""

__all__ = ["workloads"]
