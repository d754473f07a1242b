"""Straight-ray crosswell measurement operator H (Sec. 4.1).

The paper's traveltime y = integral of the slowness along the ray equals H s,
where H_ij is the length of ray i inside cell j (eq.
``equation_traveltimeintegral``).  Sources sit on the well x = 0 and
receivers on the well x = 1 at uniform depths; every source is paired with
every receiver, as in the paper's 6 x 48 survey (Sec. 4.1).

In 3-D the same 2-D survey is repeated in ``planes`` vertical planes
y = (o + 1/2) / planes, so every ray stays inside its plane.

Tie-break for a ray that runs along a cell face: each straight piece between
consecutive grid-line crossings goes to the cell that contains the piece's
midpoint under floor(coord * N), clamped to N - 1.
"""

import math

import numpy as np


def _default_split(p: int):
    """Sources x receivers with sources = largest power of two <= sqrt(p)
    that divides p (16 = 4x4, 64 = 8x8, 256 = 16x16, 512 = 16x32)."""
    ns = 1 << int(math.floor(math.log2(p) / 2)) if p > 0 else 1
    while ns > 1 and p % ns:
        ns //= 2
    return ns, p // ns


def crosswell_geometry(dim: int, p: int, planes: int = 8, sources=None):
    """Return (start, end) arrays of shape (p, dim) for the p rays.

    2-D: ray a = s * n_r + r joins (0, z_s) to (1, z_r) with
    z_s = (s + 1/2) / n_s and z_r = (r + 1/2) / n_r.
    3-D: ray a = o * (n_s n_r) + s * n_r + r lies in plane y_o.
    ``sources`` overrides the number of sources (receivers = rays / sources).
    """
    if dim == 2:
        per_plane, nplanes = p, 1
    elif dim == 3:
        if p % planes:
            raise ValueError("p must be a multiple of the number of planes")
        per_plane, nplanes = p // planes, planes
    else:
        raise ValueError("dim must be 2 or 3")
    if sources is None:
        ns, nr = _default_split(per_plane)
    else:
        ns = int(sources)
        if per_plane % ns:
            raise ValueError("rays per plane must be a multiple of sources")
        nr = per_plane // ns
    start = np.zeros((p, dim))
    end = np.zeros((p, dim))
    a = 0
    for o in range(nplanes):
        for s in range(ns):
            for r in range(nr):
                zs = (s + 0.5) / ns
                zr = (r + 0.5) / nr
                start[a, 0], end[a, 0] = 0.0, 1.0
                start[a, dim - 1], end[a, dim - 1] = zs, zr
                if dim == 3:
                    y = (o + 0.5) / nplanes
                    start[a, 1] = end[a, 1] = y
                a += 1
    return start, end


def _trace(p0, p1, n):
    """Cells crossed by the segment p0 -> p1 and the length inside each.

    Returns (cells, lengths) with cells as grid-order linear indices, sorted.
    """
    dim = p0.shape[0]
    d = p1 - p0
    seglen = float(np.sqrt(np.dot(d, d)))
    ts = [0.0, 1.0]
    for ax in range(dim):
        if d[ax] != 0.0:
            lines = np.arange(1, n) / n
            t = (lines - p0[ax]) / d[ax]
            ts.extend(t[(t > 0.0) & (t < 1.0)].tolist())
    ts = np.unique(np.asarray(ts))
    t0, t1 = ts[:-1], ts[1:]
    keep = (t1 - t0) > 1e-12
    t0, t1 = t0[keep], t1[keep]
    mid = p0[None, :] + 0.5 * (t0 + t1)[:, None] * d[None, :]
    ijk = np.clip(np.floor(mid * n).astype(np.int64), 0, n - 1)
    lin = np.zeros(len(t0), dtype=np.int64)
    for ax in range(dim):
        lin += ijk[:, ax] * (n ** ax)
    lens = (t1 - t0) * seglen
    cells, inv = np.unique(lin, return_inverse=True)
    acc = np.zeros(len(cells))
    np.add.at(acc, inv, lens)
    return cells, acc


def crosswell_h(dim: int, n: int, p: int, planes: int = 8, sources=None):
    """CSR arrays (rowptr int64[p+1], col int32[nnz], val float64[nnz]) of H.

    Row a holds the path lengths of ray a in the cells it crosses, in domain
    units, with columns in increasing grid order.
    """
    start, end = crosswell_geometry(dim, p, planes, sources)
    rows_c, rows_v = [], []
    for a in range(p):
        c, v = _trace(start[a], end[a], n)
        rows_c.append(c)
        rows_v.append(v)
    rowptr = np.zeros(p + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(c) for c in rows_c])
    col = np.concatenate(rows_c).astype(np.int32) if p else np.zeros(0, np.int32)
    val = np.concatenate(rows_v) if p else np.zeros(0)
    return rowptr, col, val


def ray_lengths(dim: int, p: int, planes: int = 8, sources=None):
    """Euclidean length of each ray (the row sums of H)."""
    start, end = crosswell_geometry(dim, p, planes, sources)
    return np.sqrt(((end - start) ** 2).sum(axis=1))
