"""geolik: exact Gaussian log-likelihood of Matérn random fields on AMD MI355X.

The computation lives in the HIP/C++ library libgeolik.so (C ABI in
include/geolik.h); this package is its ctypes binding.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import GeolikError, lib  # noqa: F401
