"""MI355X-native Feynman path sum for Fock-state linear optics.

The compute path lives in the HIP/C++ library ``_lib/liblofp.so`` (C-ABI in
``include/lofp.h``); :mod:`paper_2510_26408_amd.lofp` is its ctypes binding and
:mod:`paper_2510_26408_amd.workloads` the seeded input generator.
"""
__all__ = ["lofp", "workloads"]
