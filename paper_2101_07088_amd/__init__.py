"""MI355X-native doubly-periodic spectral Ewald (DP-SE) electrostatics.

Thin Python binding of libdpse.so (the C ABI declared in include/dpse.h).
It only marshals arguments: every stage of a solve runs in the library's HIP
kernels. PyTorch supplies device memory and streams. If the library has not
been built, importing the binding raises -- there is no CPU fallback.
"""
from .native import (DPSE_FP64, DPSE_MIXED, DPSE_GAUGE_NONE, DPSE_KMAX_GT, DPSE_UNIFORM_FAST, DPSE_ONE_JUMP, DPSE_TRIPLY, DPSE_DETERMINISTIC, Stage, BatchGraph,
                     DpseError, Plan, derive, library_path, solve_batch, workspace_size)

__all__ = ["DPSE_FP64", "DPSE_MIXED", "DPSE_GAUGE_NONE", "DPSE_KMAX_GT", "DPSE_UNIFORM_FAST", "DPSE_ONE_JUMP", "DPSE_TRIPLY", "DPSE_DETERMINISTIC", "Stage", "DpseError",
           "Plan", "BatchGraph", "derive", "library_path", "solve_batch", "workspace_size"]
