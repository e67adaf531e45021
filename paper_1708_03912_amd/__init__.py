"""MI355X-native dense FEM assembly, matvec and CG for the integral
fractional Laplacian (Ainsworth & Glusa, arXiv:1708.03912).

The compute path is the HIP library ``libfraclap.so`` behind the C ABI in
``include/fraclap.h``; ``paper_1708_03912_amd.fraclap`` is its thin ctypes
binding.  Importing this package loads nothing; ``meshgen`` builds inputs.
"""
__all__ = ["fraclap", "meshgen"]
