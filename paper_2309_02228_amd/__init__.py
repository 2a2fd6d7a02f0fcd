"""MI355X-native matrix power kernel (MPK) with algebraic temporal blocking.

The compute path is libmpk.so (HIP kernels for gfx950, C++ host planner, C
ABI declared in include/mpk.h); ``mpk`` is its thin ctypes binding.
"""
from . import mpk  # noqa: F401  (raises ImportError if libmpk.so is not built)
from .mpk import Plan, PlanCache, MPKError, version  # noqa: F401
