"""MI355X-native fractional-step pressure projection (HIP kernels behind a C ABI).

The native library ``libfsei.so`` is loaded lazily by ``paper_2103_15187_amd.fsei``;
importing this package does not touch the GPU.
"""
__all__ = ["fsei", "workloads"]
