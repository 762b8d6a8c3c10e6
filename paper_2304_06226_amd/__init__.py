"""MI355X-native biased neutron history loop (HIP kernels behind a C-ABI).

The GPU library is loaded lazily by ``paper_2304_06226_amd.binding``; importing
the package itself loads nothing native.
"""
__all__ = ["workloads", "binding"]
