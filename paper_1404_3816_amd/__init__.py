"""MI355X-native HiKF hot path: Q H^T by an H^2 / FMM product and the
cross-covariance Kalman step, in hand-written HIP for gfx950.

``hikf`` is the ctypes binding of include/hikf.h; ``filter`` wraps it with
torch-allocated device workspaces.
"""

from . import hikf  # noqa: F401  (fails loudly if libhikf.so is missing)
from .filter import HikfFilter, problem_from_csr  # noqa: F401
