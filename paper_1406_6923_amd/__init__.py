"""MI355X-native S-fraction multiscale finite-volume wave propagation (arXiv 1406.6923).

The compute path is the HIP library ``libsfm.so`` (C ABI in ``include/sfm.h``);
``paper_1406_6923_amd.sfm`` is its ctypes binding.  Importing the package does
not load the library; the first call does, and fails loudly if it is not built.
"""
from . import sfm  # noqa: F401

__all__ = ["sfm"]
