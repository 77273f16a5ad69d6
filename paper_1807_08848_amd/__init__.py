"""MI355X-native random sampling for multiscale PDEs (offline sampling hot path).

The compute lives in ``libmsrs.so`` (HIP kernels for gfx950) behind the C ABI
of ``include/msrs.h``; :mod:`paper_1807_08848_amd.msrs` is the ctypes binding.
Build with ``python -m paper_1807_08848_amd.build``.
"""
__all__ = ["msrs", "build"]
