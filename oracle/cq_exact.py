"""Tier C: the exact product C_Q = Q H^T -- test infrastructure only.

Sec. 3.2 writes Q H^T column by column, (Q h^(k))_i = sum_j K(x_i, x_j)
h^(k)_j.  Three independent routes compute it exactly (up to rounding):

* ``cq_dense``: form Q and multiply (small m).
* ``cq_fft``: on a uniform grid Q is block Toeplitz; embedding it in a
  circulant of twice the size per axis turns Q w into a periodic
  convolution evaluated with FFTs (the FFT route Sec. 1 mentions for
  regular grids).
* ``cq_rows``: the defining sum evaluated directly for chosen rows i, over
  the nonzeros of H only: C_Q[i, a] = sum_{j in ray a} K(|x_i - x_j|) H_aj.
"""

import numpy as np

from .kernels import kernel, dense_q


def _dense_from_csr(rowptr, col, val, m):
    p = len(rowptr) - 1
    H = np.zeros((p, m))
    for a in range(p):
        sl = slice(rowptr[a], rowptr[a + 1])
        H[a, col[sl]] = val[sl]
    return H


def cq_dense(points, W, family="powexp", theta=1.0, ell=1.0, gamma=1.0):
    """Q @ W with Q formed densely; W is (m, p) (W = H^T for C_Q)."""
    return dense_q(points, family, theta, ell, gamma) @ np.asarray(W, np.float64)


def cq_fft(dim, n, W, family="powexp", theta=1.0, ell=1.0, gamma=1.0,
           chunk=16):
    """Q @ W on the N^dim cell-centred grid by circulant embedding.

    W is (m, p) in grid order (x fastest).  The embedding holds K at the
    periodic offsets u - 2N*[u >= N] (times h) on a (2N)^dim grid; the linear
    convolution of an N^dim field with it is exact on the first N^dim
    entries because every true offset lies in (-N, N).
    """
    W = np.asarray(W, np.float64)
    m, p = W.shape
    h = 1.0 / n
    K = kernel(family, theta, ell, gamma)
    off = np.arange(2 * n)
    off = np.where(off < n, off, off - 2 * n) * h
    grids = np.meshgrid(*([off] * dim), indexing="ij")
    dist = np.sqrt(sum(g * g for g in grids))
    kf = np.fft.rfftn(K(dist))
    out = np.empty((m, p))
    shape = (n,) * dim
    big = (2 * n,) * dim
    axes = tuple(range(dim))
    for c0 in range(0, p, chunk):
        c1 = min(p, c0 + chunk)
        for c in range(c0, c1):
            f = W[:, c].reshape(shape)
            y = np.fft.irfftn(np.fft.rfftn(f, s=big, axes=axes) * kf, s=big, axes=axes)
            out[:, c] = y[tuple(slice(0, n) for _ in range(dim))].reshape(m)
    return out


def cq_rows(dim, n, rowptr, col, val, rows, family="powexp", theta=1.0,
            ell=1.0, gamma=1.0, chunk=32):
    """Exact C_Q[rows, :] by the defining sum over the nonzeros of H."""
    rows = np.asarray(rows, np.int64)
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    val = np.asarray(val, np.float64)
    p = len(rowptr) - 1
    K = kernel(family, theta, ell, gamma)
    h = 1.0 / n

    def coords(idx):
        return np.stack([((idx // (n ** ax)) % n + 0.5) * h
                         for ax in range(dim)], axis=1)

    src = coords(col)
    out = np.zeros((len(rows), p))
    for r0 in range(0, len(rows), chunk):
        tgt = coords(rows[r0:r0 + chunk])
        d = tgt[:, None, :] - src[None, :, :]
        kv = K(np.sqrt((d * d).sum(-1))) * val[None, :]
        for a in range(p):
            out[r0:r0 + chunk, a] = kv[:, rowptr[a]:rowptr[a + 1]].sum(axis=1)
    return out


def h_dense(rowptr, col, val, m):
    """Dense (p, m) H from CSR arrays."""
    return _dense_from_csr(rowptr, col, val, m)
