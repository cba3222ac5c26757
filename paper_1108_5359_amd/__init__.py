"""MI355X-native l1 filtering for Principal Component Pursuit.

The method's arithmetic lives in ``librpca.so`` (HIP kernels for gfx950 behind
the C ABI of ``include/rpca.h``); ``paper_1108_5359_amd.rpca`` is its ctypes
binding.  Build with ``python paper_1108_5359_amd/build.py``.
"""
__all__ = ["rpca"]
