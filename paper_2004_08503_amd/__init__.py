"""MI355X-native sparse IDP nodal DG stage (arXiv 2004.08503).

The compute path is the C-ABI library ``libidp_dg.so`` (HIP kernels for
gfx950); ``paper_2004_08503_amd.idp_dg`` is its ctypes binding.  Importing
the package itself loads nothing, so the seeded workload module can be used
without a GPU.
"""
__all__ = ["workloads"]
