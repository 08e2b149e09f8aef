"""qsd: sparse-tensor transposition (Quesadilla) on AMD Instinct MI355X.

The compute path is the native library ``libqsd.so`` (HIP kernels for gfx950 behind a
C ABI, declared in ``include/qsd.h``); ``qsd`` is its ctypes binding.
"""
