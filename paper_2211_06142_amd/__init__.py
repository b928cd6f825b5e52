"""MI355X-native DEM + fluid-coupling hot path of arXiv:2211.06142.

The product is libdem.so (HIP kernels for gfx950 behind the C ABI of
include/dem.h); ``paper_2211_06142_amd.dem`` is its ctypes binding.
"""
from . import dem  # noqa: F401
