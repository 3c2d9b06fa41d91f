"""MI355X (gfx950) SGM stereo-disparity pipeline (arXiv 1610.04121).

The compute path is the HIP library ``libsgm.so`` behind the C ABI in
``include/sgm.h``; :mod:`paper_1610_04121_amd.sgm` is its ctypes binding and
:mod:`paper_1610_04121_amd.synth` the seeded synthetic input generator.
Importing the package loads nothing; the library is loaded on first use.
"""
from .sgm import SGM, SGMError, INVALID, footprint_bytes, validate, path_walk  # noqa: F401

__all__ = ["SGM", "SGMError", "INVALID", "footprint_bytes", "validate", "path_walk"]
