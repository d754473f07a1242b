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
