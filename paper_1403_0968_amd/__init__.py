"""MI355X-native spectral-element Poisson operator (arXiv 1403.0968, sec. 4.2).

The computation lives in ``libsem.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/sem.h``); ``sem`` is its ctypes binding.
"""
from . import sem  # noqa: F401
