"""MI355X-native population-parallel local search (cuGenOpt hot path).

The engine is the HIP library libgx.so (sources in csrc/, interface in
include/gx.h); ``gx`` is its ctypes binding.
"""
from . import gx  # noqa: F401

__all__ = ["gx"]
