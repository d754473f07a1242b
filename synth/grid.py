"""Uniform cell-centred grids on the unit square / cube.

Points are the centres ((i+1/2)h, (j+1/2)h[, (k+1/2)h]) with h = 1/N.  The
linear index is lexicographic with the first coordinate (x, the inter-well
distance) fastest, then the second (2-D: depth z; 3-D: y), then the third
(3-D: depth z).
"""

import numpy as np


def grid_size(dim: int, n: int) -> int:
    """Number of unknowns m = N^dim."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1:
        raise ValueError("n must be positive")
    return n ** dim


def grid_shape(dim: int, n: int):
    """Array shape of a grid-ordered field, slowest axis first."""
    return (n,) * dim


def cell_centres(dim: int, n: int) -> np.ndarray:
    """(m, dim) array of cell centres; column 0 is x (fastest index)."""
    m = grid_size(dim, n)
    idx = np.arange(m, dtype=np.int64)
    out = np.empty((m, dim), dtype=np.float64)
    for ax in range(dim):
        out[:, ax] = ((idx // (n ** ax)) % n + 0.5) / n
    return out
