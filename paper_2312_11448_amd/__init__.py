"""MI355X-native Monte-Carlo Lyman-alpha packet transport.

Python face of libmclya.so (HIP kernels for gfx950 behind the C ABI of
include/mc_lya.h). ``_abi`` mirrors the C calls one for one; ``Simulation``
holds the device arrays (torch tensors) that the calls read and write.
"""
from ._abi import *  # noqa: F401,F403
from ._abi import load, MCLyaError, LIB_PATH  # noqa: F401
from .sim import Simulation, desc_from_spec  # noqa: F401
from .mlp import Mlp  # noqa: F401
