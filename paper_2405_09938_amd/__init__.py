"""MI355X (gfx950) facet-sum raw-data generator (HEEPS/MARE hot path).

The computation lives in libheeps_sim.so (hand-written HIP for gfx950, C ABI
in include/heeps_sim.h); this package is its PyTorch-facing binding.
"""
from .sim import FACET_KEYS, GRAD_KEYS, Plan, SimForward, Simulator, simulate  # noqa: F401
from ._native import SimError, load  # noqa: F401
