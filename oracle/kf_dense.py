"""Tier A: the conventional random-walk Kalman filter -- test infrastructure.

Follows Sec. 2.2 (Algorithm ``algorithm_Kalman``) with F = I (Sec. 2.1, eq.
``equation_random_walk``) and stationary Q, R, H:

  predict   x_{t+1|t} = x_{t|t};  P_{t+1|t} = P_{t|t} + Q     (eq. KF_forecast)
  gain      K = P_{t+1|t} H^T (H P_{t+1|t} H^T + R)^{-1}      (eq. eqn_kalmangin)
  state     x_{t+1|t+1} = x_{t+1|t} + K (y_{t+1} - H x_{t+1|t})
  covar.    P_{t+1|t+1} = P_{t+1|t} - K H P_{t+1|t}           (eq. eqn_KF_Pa)

The inverse is applied through a Cholesky factorisation of the innovation
covariance and triangular solves (LAPACK via SciPy), never formed.
"""

import numpy as np
import scipy.linalg as sla


def dense_kf(Q, H, R, x0, P0, ys):
    """Run the filter over the rows of ``ys``.

    Q (m,m), H (p,m), R (p,p), x0 (m,), P0 (m,m), ys (steps,p).
    Returns (xs, variances, covariances): arrays (steps,m), (steps,m),
    (steps,m,m) holding x_{k|k}, diag P_{k|k} and P_{k|k} for k = 1..steps.
    """
    Q = np.asarray(Q, np.float64)
    H = np.asarray(H, np.float64)
    R = np.asarray(R, np.float64)
    x = np.array(x0, np.float64, copy=True)
    P = np.array(P0, np.float64, copy=True)
    xs, vs, Ps = [], [], []
    for y in np.atleast_2d(ys):
        P = P + Q                                   # predict
        S = H @ P @ H.T + R
        cf = sla.cho_factor(S, lower=True)
        K = sla.cho_solve(cf, H @ P.T).T            # P H^T S^{-1}
        x = x + K @ (y - H @ x)
        P = P - K @ (H @ P)
        xs.append(x.copy())
        vs.append(np.diag(P).copy())
        Ps.append(P.copy())
    return np.array(xs), np.array(vs), np.array(Ps)
