"""MI355X-native multiresolution contact detection between triangulated
rigid particles (Noble & Weinzierl, arXiv 2105.12415), behind a C ABI
(include/dem.h) implemented in hand-written HIP for gfx950 (libdem.so).
"""
from ._abi import DemError, lib, EXPORTS, LIB_PATH  # noqa: F401
from . import api  # noqa: F401

__all__ = ["DemError", "lib", "EXPORTS", "LIB_PATH", "api"]
