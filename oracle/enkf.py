"""Perturbed-observation ensemble Kalman filter -- test infrastructure only.

Sec. 2.3 (eqs. ``equation_samplemean``, ``equation_samplecov1``,
``equation_samplegain_enkf``) on the random-walk model of Sec. 2.1 (eq.
``equation_random_walk``), in the stochastic form the paper compares against
(Houtekamer and Mitchell 1998; Burgers, van Leeuwen and Evensen 1998): every
member is forecast and corrected like the Kalman filter's mean, with its own
model-error draw and its own perturbed copy of the data.  One step, for the
ensemble X = [x^1 ... x^N] (m x N):

  forecast   x^j <- x^j + w^j,           w^j a draw from N(0, Q)
  mean       x~ = (1/N) sum_j x^j                        (eq. samplemean)
  anomalies  A = (X - x~ 1^T) / sqrt(N - 1),  Sigma~ = A A^T  (eq. samplecov1)
  gain       K~ = A A^T H^T (H A A^T H^T + R)^{-1}       (eq. samplegain_enkf)
  analysis   x^j <- x^j + K~ (y + v^j - H x^j),  v^j a draw from N(0, R)

Sigma~ is never formed: the m x p gain K~ = A (H A)^T S^{-1} with
S = (H A)(H A)^T + R (Cholesky factorisation and solves, as in ``kf_dense``)
is applied to the innovations of all members.  The draws are
inputs (E = [w^1 ... w^N], V = [v^1 ... v^N]); the oracle draws nothing.
Outputs per step: the analysis sample mean and the diagonal of the analysis
sample covariance (the 1/(N-1) normalisation of eq. samplecov1).
FP64 NumPy / SciPy; H may be a dense array or a SciPy sparse matrix.
"""

import numpy as np
import scipy.linalg as sla


def enkf_step(X, E, H, y, V, r_diag):
    """One forecast + analysis step.  X (m, N) is not modified; returns
    (X_analysis, mean, variance)."""
    X = np.asarray(X, np.float64)
    N = X.shape[1]
    if N < 2:
        raise ValueError("the sample covariance needs N >= 2 members")
    Xf = X + np.asarray(E, np.float64) if E is not None else X.copy()
    xm = Xf.mean(axis=1)
    A = (Xf - xm[:, None]) / np.sqrt(N - 1.0)
    HA = np.asarray(H @ A)
    S = HA @ HA.T + np.diag(np.asarray(r_diag, np.float64))
    cf = sla.cho_factor(S, lower=True)
    D = np.asarray(y, np.float64)[:, None] + np.asarray(V, np.float64) - np.asarray(H @ Xf)
    K = sla.cho_solve(cf, HA @ A.T).T                     # K~ = A (H A)^T S^{-1}
    Xa = Xf + K @ D                                       # x^j + K~ (d^j - H x^j), all j
    mean = Xa.mean(axis=1)
    var = ((Xa - mean[:, None]) ** 2).sum(axis=1) / (N - 1.0)
    return Xa, mean, var


def enkf_run(X0, H, r_diag, ys, Es, Vs):
    """Steps k = 1..K with data ys[k-1] (p,), model-error draws Es[k-1]
    (m, N; None for no forecast noise) and observation draws Vs[k-1] (p, N).
    Returns (X_K, means (K, m), variances (K, m))."""
    X = np.array(X0, np.float64, copy=True)
    means, vars_ = [], []
    for k in range(len(ys)):
        X, mu, va = enkf_step(X, None if Es is None else Es[k], H, ys[k], Vs[k], r_diag)
        means.append(mu)
        vars_.append(va)
    return X, np.array(means), np.array(vars_)
