"""MI355X-native simulated p-bit Ising machine (arXiv 2510.23419 hot path).

The sweep runs in hand-written HIP kernels for gfx950 behind the C ABI of
``libpbit.so`` (declared in ``include/pbit.h``); ``paper_2510_23419_amd.pbit``
is its ctypes binding.  Importing this package loads nothing; the library is
opened on first use and a missing build is an error.
"""
__all__ = ["pbit"]
