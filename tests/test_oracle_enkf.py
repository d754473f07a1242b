"""Pins for the oracle's perturbed-observation EnKF (Sec. 2.3).

The EnKF is pinned against the Kalman filter (tier A, itself pinned in
test_oracle_kf.py) by two routes that do not use its own formulas:

* exact moments: when the forecast anomalies have sample covariance exactly
  P_f and the observation perturbations have zero sample mean, sample
  covariance exactly R and no sample correlation with the anomalies, one
  analysis gives exactly the Kalman posterior mean and covariance (the
  stochastic EnKF's analysis covariance is the Joseph form of the update,
  which equals (I - K H) P_f for the optimal gain);
* convergence: with draws from N(0, P_0), N(0, Q), N(0, R) the ensemble mean
  and variance approach the Kalman filter's as N grows, at the Monte Carlo
  rate 1/sqrt(N).
"""

import numpy as np
import pytest

from oracle import enkf, kernels, kf_dense


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _centred_orthonormal(N, k, rng):
    """(N, k) with orthonormal columns, every column orthogonal to ones."""
    M = np.hstack([np.ones((N, 1)), rng.standard_normal((N, k))])
    Qm, _ = np.linalg.qr(M)
    return Qm[:, 1:k + 1]


def _problem(m=7, p=3, seed=5):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(size=(m, 2))
    Pf = kernels.dense_q(pts, "powexp", 1.1, 0.5, 1.0) + 0.05 * np.eye(m)
    H = rng.uniform(-1.0, 1.0, size=(p, m))
    r = rng.uniform(0.05, 0.3, size=p)
    xbar = rng.standard_normal(m)
    y = rng.standard_normal(p)
    return rng, Pf, H, r, xbar, y


@pytest.mark.parametrize("N", [11, 24])
def test_exact_moments_reproduce_the_kalman_update(N):
    rng, Pf, H, r, xbar, y = _problem()
    m, p = len(xbar), len(y)
    Z = _centred_orthonormal(N, m + p, rng) * np.sqrt(N - 1.0)
    X = xbar[:, None] + np.linalg.cholesky(Pf) @ Z[:, :m].T
    V = np.sqrt(r)[:, None] * Z[:, m:].T
    Xa, mean, var = enkf.enkf_step(X, None, H, y, V, r)
    xk, vk, Pk = kf_dense.dense_kf(np.zeros((m, m)), H, np.diag(r), xbar, Pf, y[None, :])
    assert _rel(mean, xk[0]) < 1e-12
    assert _rel(var, vk[0]) < 1e-12
    Aa = Xa - mean[:, None]
    assert _rel(Aa @ Aa.T / (N - 1.0), Pk[0]) < 1e-12


def test_unperturbed_observations_shrink_the_spread_too_much():
    # without the v^j the analysis covariance is (I-KH) P_f (I-KH)^T, which
    # lacks K R K^T: the exact-moment test above fails for that mistake
    rng, Pf, H, r, xbar, y = _problem()
    m, p, N = len(xbar), len(y), 24
    Z = _centred_orthonormal(N, m, rng) * np.sqrt(N - 1.0)
    X = xbar[:, None] + np.linalg.cholesky(Pf) @ Z.T
    _, _, var = enkf.enkf_step(X, None, H, y, np.zeros((p, N)), r)
    _, vk, _ = kf_dense.dense_kf(np.zeros((m, m)), H, np.diag(r), xbar, Pf, y[None, :])
    assert np.all(var < vk[0])


def test_no_information_keeps_the_forecast():
    # H = 0: the gain vanishes and the analysis is the forecast X + E
    rng = np.random.default_rng(2)
    m, p, N = 9, 4, 6
    X, E = rng.standard_normal((m, N)), rng.standard_normal((m, N))
    Xa, mean, var = enkf.enkf_step(X, E, np.zeros((p, m)), rng.standard_normal(p),
                                   rng.standard_normal((p, N)), np.full(p, 0.1))
    assert np.array_equal(Xa, X + E)
    assert np.allclose(mean, (X + E).sum(axis=1) / N, rtol=0, atol=1e-15)


def test_converges_to_the_kalman_filter():
    rng = np.random.default_rng(11)
    m, p, K = 5, 2, 4
    pts = rng.uniform(size=(m, 2))
    Q = kernels.dense_q(pts, "powexp", 0.4, 0.3, 1.0)
    P0 = kernels.dense_q(pts, "powexp", 1.0, 0.3, 1.0)
    H = rng.uniform(0.0, 1.0, size=(p, m))
    r = np.array([0.2, 0.1])
    x0 = rng.standard_normal(m)
    ys = rng.standard_normal((K, p))
    xk, vk, _ = kf_dense.dense_kf(Q, H, np.diag(r), x0, P0, ys)
    LQ, LP = np.linalg.cholesky(Q + 1e-12 * np.eye(m)), np.linalg.cholesky(P0)
    errs = {}
    for N in (2000, 200000):
        g = np.random.default_rng(N)
        X0 = x0[:, None] + LP @ g.standard_normal((m, N))
        Es = [LQ @ g.standard_normal((m, N)) for _ in range(K)]
        Vs = [np.sqrt(r)[:, None] * g.standard_normal((p, N)) for _ in range(K)]
        _, means, vars_ = enkf.enkf_run(X0, H, r, ys, Es, Vs)
        errs[N] = (max(_rel(means[k], xk[k]) for k in range(K)),
                   max(_rel(vars_[k], vk[k]) for k in range(K)))
    assert errs[200000][0] < 0.02 and errs[200000][1] < 0.01
    # Monte Carlo rate: 100x the members, about 10x smaller errors
    assert errs[200000][0] < errs[2000][0] / 3
    assert errs[200000][1] < errs[2000][1] / 3


def test_one_member_is_rejected():
    with pytest.raises(ValueError):
        enkf.enkf_step(np.zeros((3, 1)), None, np.zeros((1, 3)), [0.0], np.zeros((1, 1)), [1.0])
