"""MI355X-native scenario-based robust reference governor.

The GPU library (``librg.so``, HIP for gfx950, C ABI in ``include/rg.h``) is
loaded lazily by :mod:`paper_2510_08288_amd.rg`; importing this package does not
touch the GPU.
"""
__all__ = ["workloads"]
