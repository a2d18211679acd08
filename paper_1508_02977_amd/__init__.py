"""Overlapping-Schwarz optical flow with varying illumination on MI355X.

The compute path is the HIP library ``libsfdd.so`` (C ABI in
``include/sfdd.h``); :mod:`paper_1508_02977_amd.api` is its Python binding and
:mod:`paper_1508_02977_amd.synth` draws seeded synthetic frame pairs.
Importing this package loads nothing; the first binding call loads the library
and fails loudly if it has not been built.
"""

__all__ = ["api", "synth", "build"]
