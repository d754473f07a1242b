"""Tier B: the cross-covariance (HiKF) filter in FP64 -- test infrastructure.

Follows Algorithm ``Algorithm_HiKF`` and Sec. 3.1 with an exact or given
C_Q = Q H^T:

  predict   s_{t+1|t} = s_{t|t};  C_{t+1|t} = C_{t|t} + C_Q  (eq. eqn_KF_forecast_new)
            var_{t+1|t} = var_{t|t} + diag Q                   (reading: the
            algorithm prints no variance prediction; diag Q = K(0))
  gain      K = C_{t+1|t} (H C_{t+1|t} + R)^{-1}               (eq. eqn_kalmangin_new)
  state     s_{t+1|t+1} = s_{t+1|t} + K (y_{t+1} - H s_{t+1|t})
  cross-cov C_{t+1|t+1} = C_{t+1|t} - K (H C_{t+1|t})          (eq. eqn_KF_pred_new)
  variance  var_i -= sum_j K_ij (C_{t+1|t})_ij                  (Sec. 3.1)

Readings: H C is symmetric only in exact arithmetic, so the innovation
covariance is taken as S = (G + G^T)/2 + R with G = H C_{t+1|t}; S^{-1} is
applied by Cholesky solves.  Rows are independent given G, so the filter may
be run on any row subset that contains every cell a ray crosses (the
columns where H is nonzero); the other rows are then exact samples.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _as_operator(H):
    return H.tocsr() if sp.issparse(H) else np.asarray(H, np.float64)


def crosscov_kf(CQ, H, R, x0, C0, var0, qdiag, ys, return_C=False, return_Z=False):
    """Run tier B over the rows of ``ys``.

    CQ (m,p) = Q H^T; H (p,m) dense or scipy-sparse; R (p,p); x0 (m,);
    C0 (m,p) = P0 H^T; var0 (m,) = diag P0; qdiag = K(0) (scalar or (m,)).
    Returns (xs, variances) of shape (steps, m) [and the final C] [and the
    list of Z_s = C_{s|s-1} L_s^{-T}, S_s = L_s L_s^T].  The covariance update
    P_{s|s} = P_{s|s-1} - K_s H P_{s|s-1} equals P_{s|s-1} - Z_s Z_s^T, so
    P_t = P_0 + t Q - sum_s Z_s Z_s^T can be rebuilt from the Z history
    without ever holding an m x m matrix during the filter.
    """
    H = _as_operator(H)
    R = np.asarray(R, np.float64)
    C = np.array(C0, np.float64, copy=True)
    x = np.array(x0, np.float64, copy=True)
    var = np.array(var0, np.float64, copy=True)
    xs, vs, zs = [], [], []
    for y in np.atleast_2d(ys):
        C = C + CQ                                   # predict
        var = var + qdiag
        G = H @ C                                    # H C_{t+1|t}, (p,p)
        S = 0.5 * (G + G.T) + R
        cf = sla.cho_factor(S, lower=True)
        K = sla.cho_solve(cf, C.T).T                 # C S^{-1}
        if return_Z:
            L = np.tril(cf[0])
            zs.append(sla.solve_triangular(L, C.T, lower=True).T)
        x = x + K @ (y - H @ x)
        var = var - np.einsum("ij,ij->i", K, C)
        C = C - K @ G
        xs.append(x.copy())
        vs.append(var.copy())
    out = (np.array(xs), np.array(vs))
    if return_C:
        out = out + (C,)
    if return_Z:
        out = out + (zs,)
    return out


def crosscov_gain_identity(C_prior, G, R):
    """Both forms of the posterior cross-covariance for one step.

    Returns (C - K G, K R) with K = C S^{-1}, S = (G+G^T)/2 + R.  They agree
    because S - R = G (for symmetric G), so C - C S^{-1} G = C S^{-1} R; the
    second form (P_post H^T = K R) is the one that avoids cancellation.
    """
    S = 0.5 * (G + G.T) + R
    cf = sla.cho_factor(S, lower=True)
    K = sla.cho_solve(cf, C_prior.T).T
    return C_prior - K @ G, K @ R


def psd_part(A):
    """The nearest symmetric positive semidefinite matrix to sym(A) in the
    Frobenius norm: its eigendecomposition with the negative eigenvalues set
    to zero (LAPACK symmetric eigensolver via NumPy)."""
    A = 0.5 * (np.asarray(A, np.float64) + np.asarray(A, np.float64).T)
    w, V = np.linalg.eigh(A)
    return (V * np.clip(w, 0.0, None)) @ V.T


def crosscov_kf_guarded(CQ, H, R, x0, C0, var0, qdiag, ys, G0=None):
    """Tier B with the measurement-space prior kept positive semidefinite.

    The H^2 approximation of a smooth kernel makes H Q H^T (which enters
    every step's G = H C_prior) indefinite; the random walk adds it every
    step, so S = (G + G^T)/2 + R eventually fails its Cholesky.  This variant
    carries G and h = H x_hat by the exact recursions of the cross-covariance
    update (C_post = K R gives H C_post = G S^{-1} R, and H x_hat_post =
    h + G S^{-1} nu), with H Q H^T replaced by its PSD part GQp:
        G_{t+1|t} = G_{t|t-1} S^{-1} R + GQp,   h <- h + G S^{-1} nu,
    starting from G_{1|0} = H C_0 + GQp (G0, when given, overrides it; for
    the kernel prior P_0 = Q the start is 2 GQp) and h = H x_0.  Both p-space
    quantities then describe one PSD measurement-space model, so S stays SPD
    and the innovation loop is stable; the rows of C, x_hat and the variances
    are updated as in ``crosscov_kf`` (with C_post = K R).
    Returns (xs, variances).
    """
    H = _as_operator(H)
    R = np.asarray(R, np.float64)
    C = np.array(C0, np.float64, copy=True)
    x = np.array(x0, np.float64, copy=True)
    var = np.array(var0, np.float64, copy=True)
    GQp = psd_part(H @ CQ)
    G = np.array(G0, np.float64, copy=True) if G0 is not None else H @ C + GQp
    h = H @ x
    xs, vs = [], []
    for y in np.atleast_2d(ys):
        C = C + CQ
        var = var + qdiag
        S = 0.5 * (G + G.T) + R
        cf = sla.cho_factor(S, lower=True)
        K = sla.cho_solve(cf, C.T).T
        nu = y - h
        x = x + K @ nu
        var = var - np.einsum("ij,ij->i", K, C)
        C = K @ R
        h = h + G @ sla.cho_solve(cf, nu)
        G = G @ sla.cho_solve(cf, R) + GQp
        xs.append(x.copy())
        vs.append(var.copy())
    return np.array(xs), np.array(vs)
