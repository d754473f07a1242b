"""Seeded random draws, a synthetic plume truth and the workload table.

Random numbers are drawn here with numpy's PCG64 generator and handed to
whoever needs them, so the oracle and the GPU path never need a shared
random-number implementation.
"""

import numpy as np

from .grid import cell_centres, grid_size

# The five workloads (grids, kernels, ray counts, filter lengths) the build is
# exercised on.  Kernel K(r) = theta * exp(-(r/ell)^gamma) (Sec. 4.2, eq.
# ``equation_Q``), R = r_var * I (eq. ``equation_R``), prior x0 = 0, P0 = Q.
WORKLOADS = {
    "crosswell-32x32-p16": dict(
        dim=2, n=32, p=16, theta=1.0, ell=0.3, gamma=1.0, r_var=1e-4,
        steps=10, n_c=4, seed=0, prior="kernel"),
    "crosswell-256x256-p64": dict(
        dim=2, n=256, p=64, theta=1.0, ell=0.1, gamma=1.0, r_var=1e-4,
        steps=100, n_c=4, seed=0, prior="kernel"),
    "crosswell-1024x1024-p256": dict(
        dim=2, n=1024, p=256, theta=1.0, ell=0.05, gamma=2.0, r_var=1e-4,
        steps=50, n_c=5, seed=0, prior="kernel"),
    "crosswell-128cube-p512": dict(
        dim=3, n=128, p=512, theta=1.0, ell=0.2, gamma=1.0, r_var=1e-4,
        steps=20, n_c=4, seed=0, prior="kernel"),
}


def workload(name: str) -> dict:
    """A copy of one workload's parameters (with m filled in)."""
    w = dict(WORKLOADS[name])
    w["m"] = grid_size(w["dim"], w["n"])
    w["name"] = name
    return w


def normal_draws(seed: int, *shape) -> np.ndarray:
    """Standard-normal draws from numpy's PCG64 stream for ``seed``."""
    return np.random.default_rng(seed).standard_normal(shape)


def plume_truth(dim: int, n: int, steps: int, amplitude: float = 1.0, cells=None):
    """(steps, m) slowness perturbations of a plume spreading from x = 0.

    A stand-in for the paper's CO2 plume (Sec. 4.1, which is not public): a
    smooth bump attached to the injection well at mid depth whose lateral
    and vertical extents grow like sqrt(k).  Row k-1 is the state at step k.
    With ``cells`` (grid indices) only those columns are produced.
    """
    pts = cell_centres(dim, n)
    if cells is not None:
        pts = pts[np.asarray(cells)]
    out = np.empty((steps, pts.shape[0]))
    depth = pts[:, dim - 1]
    for k in range(1, steps + 1):
        frac = np.sqrt(k / steps)
        a = 0.05 + 0.75 * frac            # lateral reach from the well
        b = 0.03 + 0.20 * frac            # vertical half-thickness
        q = (pts[:, 0] / a) ** 2 + ((depth - 0.5) / b) ** 2
        if dim == 3:
            q = q + ((pts[:, 1] - 0.5) / b) ** 2
        out[k - 1] = amplitude * np.exp(-q)
    return out


def observations(rowptr, col, val, truth, r_var, seed: int):
    """y_k = H x_k + sqrt(r_var) * eps_k for every row x_k of ``truth``.

    This is the measurement equation of the state-space model (Sec. 2.1, eq.
    ``equation_measurement``) used to synthesise data.
    """
    steps = truth.shape[0]
    p = len(rowptr) - 1
    eps = normal_draws(seed, steps, p)
    y = np.empty((steps, p))
    rows = np.repeat(np.arange(p), np.diff(rowptr))
    for k in range(steps):
        hx = np.bincount(rows, weights=val * truth[k, col], minlength=p)
        y[k] = hx + np.sqrt(r_var) * eps[k]
    return y


def plume_observations(dim, n, rowptr, col, val, steps, r_var, seed: int):
    """``observations`` of ``plume_truth`` evaluated only at the ray cells,
    for grids where a dense (steps, m) truth would be wasteful."""
    cells, inv = np.unique(np.asarray(col), return_inverse=True)
    truth = plume_truth(dim, n, steps, cells=cells)
    return observations(rowptr, inv, val, truth, r_var, seed)


def serving_streams(count: int = 64, seed: int = 1):
    """Filter configurations of a serving mix: per stream a 2-D grid with
    m log-uniform in [16384, 1048576] (N = round(sqrt(m))), p drawn from
    {32, 64, 128, 256, 512}, ell ~ U[0.05, 0.3] and the kernel exponential
    or Gaussian with probability 1/2 each (drawn in that order per stream);
    R = 1e-4 I and P_0 = Q as in the other workloads.

    The Chebyshev order and arithmetic follow the kernel: exponential
    streams use n_c = 4 with the FP32 FMM; Gaussian streams use the largest
    order, n_c = 8, the FP64 FMM and the PSD guard, because the H^2
    approximation of a smooth kernel leaves H Q H^T indefinite at every
    order up to 8 (the innovation covariance of the literal filter then
    fails within 3 to 52 steps on these streams), and FP32 rounding of C_Q
    alone moves its smallest eigenvalues by more than their size."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        m = float(np.exp(rng.uniform(np.log(16384.0), np.log(1048576.0))))
        n = int(round(np.sqrt(m)))
        p = int(rng.choice([32, 64, 128, 256, 512]))
        ell = float(rng.uniform(0.05, 0.3))
        gauss = bool(rng.uniform() < 0.5)
        out.append(dict(dim=2, n=n, m=n * n, p=p, theta=1.0, ell=ell,
                        gamma=2.0 if gauss else 1.0, n_c=8 if gauss else 4,
                        precision="f64" if gauss else "f32", psd_guard=gauss,
                        r_var=1e-4, prior="kernel", seed=seed + 1 + s))
    return out


def poisson_requests(count: int, streams: int, rate, seed: int = 1):
    """Arrival times (seconds; all zero when rate is None) and stream ids
    (uniform over the streams) of a request sequence."""
    rng = np.random.default_rng(seed)
    sid = rng.integers(streams, size=count)
    if rate is None:
        return np.zeros(count), sid
    return np.cumsum(rng.exponential(1.0 / rate, size=count)), sid
