"""Covariance kernels Q_ij = K(|x_i - x_j|) -- test infrastructure only.

* ``powexp``: K(r) = theta * exp(-(r / ell)^gamma), the model-error kernel of
  Sec. 4.2 (eq. ``equation_Q``; the paper calls the exponent p, here gamma).
  gamma = 1 is the exponential kernel and gamma = 2 the Gaussian kernel of
  the Sec. 3.3 list (there written sigma^2 exp(-r^2/L^2) and exp(-r/L)).
* ``r2``: K(r) = theta * r^2, a test-only kernel that is a polynomial of
  degree 2 in every coordinate, so Chebyshev interpolation with 3 or more
  nodes per axis reproduces it exactly.
"""

import numpy as np


def powexp(r, theta=1.0, ell=1.0, gamma=1.0):
    r = np.asarray(r, dtype=np.float64)
    return theta * np.exp(-np.power(r / ell, gamma))


def r2(r, theta=1.0, ell=1.0, gamma=1.0):
    r = np.asarray(r, dtype=np.float64)
    return theta * r * r


FAMILIES = {"powexp": powexp, "r2": r2}


def kernel(family="powexp", theta=1.0, ell=1.0, gamma=1.0):
    """Return K as a function of distance arrays."""
    f = FAMILIES[family]
    return lambda r: f(r, theta, ell, gamma)


def diag_value(family="powexp", theta=1.0, ell=1.0, gamma=1.0):
    """K(0), the diagonal of Q (the same for every cell)."""
    return float(kernel(family, theta, ell, gamma)(0.0))


def dense_q(points, family="powexp", theta=1.0, ell=1.0, gamma=1.0):
    """The dense m x m matrix Q_ij = K(|x_i - x_j|)."""
    d = points[:, None, :] - points[None, :, :]
    return kernel(family, theta, ell, gamma)(np.sqrt((d * d).sum(-1)))
