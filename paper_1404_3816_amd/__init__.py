"""MI355X-native HiKF hot path: Q H^T by an H^2 / FMM product and the
cross-covariance Kalman step, in hand-written HIP for gfx950.

``hikf`` is the ctypes binding of include/hikf.h; ``filter`` wraps it with
torch-allocated device workspaces.  Both load libhikf.so on first use and
fail loudly if it is missing; ``build`` compiles it and needs neither.
"""

import importlib

__all__ = ["hikf", "filter", "HikfFilter", "problem_from_csr", "step_batch"]


def __getattr__(name):
    if name in ("hikf", "filter"):
        return importlib.import_module(f".{name}", __name__)
    if name in ("HikfFilter", "problem_from_csr", "step_batch"):
        return getattr(importlib.import_module(".filter", __name__), name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
