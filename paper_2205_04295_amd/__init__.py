"""MI355X-native (gfx950) multi-mode rPIE hot path.

The computation lives in the HIP library ``libmrpie.so`` (C ABI in
include/mrpie.h); ``api`` holds thin torch-facing wrappers.
"""
from ._abi import MrpieError, Problem, Params, make_params, load  # noqa: F401

__all__ = ["MrpieError", "Problem", "Params", "make_params", "load"]
