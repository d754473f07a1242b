"""Pins for oracle tiers A (dense KF) and B (cross-covariance KF).

Tier A (Sec. 2.2) is pinned against results obtained by routes other than
its own recursion: the steady state of the scalar local-level model, the
H = 0 and R -> 0 limits, and brute-force Gaussian conditioning of the whole
state-space model (Sec. 2.1).  Tier B (Sec. 3.1) is pinned by its claimed
equivalence to tier A.
"""

import numpy as np
import pytest

import synth
from oracle import cq_exact, kernels, kf_crosscov, kf_dense, truth


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _small_problem(m=12, p=4, seed=3):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(size=(m, 2))
    Q = kernels.dense_q(pts, "powexp", 0.7, 0.4, 1.0)
    H = rng.uniform(0.0, 1.0, size=(p, m)) * (rng.uniform(size=(p, m)) < 0.6)
    R = np.diag(rng.uniform(0.05, 0.2, size=p))
    P0 = kernels.dense_q(pts, "powexp", 1.3, 0.2, 1.0)
    mu0 = rng.standard_normal(m)
    ys = rng.standard_normal((5, p))
    return Q, H, R, P0, mu0, ys


def test_scalar_steady_state():
    # local-level model x_t = x_{t-1} + w, y = h x + v; the prior variance
    # converges to the positive root of P^2 - qP - qr/h^2 = 0.
    q, r, h = 0.3, 0.5, 2.0
    ys = np.zeros((400, 1))
    _, var, _ = kf_dense.dense_kf([[q]], [[h]], [[r]], [0.0], [[7.0]], ys)
    pm = 0.5 * (q + np.sqrt(q * q + 4.0 * q * r / h ** 2))
    post = pm * r / (h * h * pm + r)
    assert abs(var[-1, 0] - post) < 1e-14 * post * 10


def test_h_zero_keeps_mean_and_adds_q():
    Q, H, R, P0, mu0, ys = _small_problem()
    H0 = np.zeros_like(H)
    xs, var, Ps = kf_dense.dense_kf(Q, H0, R, mu0, P0, ys)
    for k in range(len(ys)):
        np.testing.assert_array_equal(xs[k], mu0)
        np.testing.assert_allclose(Ps[k], P0 + (k + 1) * Q, rtol=1e-14, atol=1e-14)
    # tier B with H = 0: C stays zero, variance grows by K(0) per step
    xb, vb = kf_crosscov.crosscov_kf(Q @ H0.T, H0, R, mu0, P0 @ H0.T,
                                     np.diag(P0), np.diag(Q), ys)
    np.testing.assert_array_equal(xb[-1], mu0)
    np.testing.assert_allclose(vb[-1], np.diag(P0 + len(ys) * Q), rtol=1e-14)


def test_r_to_zero_interpolates():
    Q, H, R, P0, mu0, ys = _small_problem()
    assert np.linalg.matrix_rank(H) == H.shape[0]
    xs, _, _ = kf_dense.dense_kf(Q, H, 1e-13 * np.eye(H.shape[0]), mu0, P0, ys)
    for k in range(len(ys)):
        np.testing.assert_allclose(H @ xs[k], ys[k], atol=1e-9)


def _brute_force_posterior(Q, H, R, P0, mu0, ys, k):
    """Condition x_k on y_1..y_k through the joint Gaussian of
    z = (x_0, w_1..w_k, v_1..v_k), by a Schur complement."""
    m, p = Q.shape[0], H.shape[0]
    nz = m + k * m + k * p
    cov = np.zeros((nz, nz))
    cov[:m, :m] = P0
    for s in range(k):
        a = m + s * m
        cov[a:a + m, a:a + m] = Q
        b = m + k * m + s * p
        cov[b:b + p, b:b + p] = R
    mean = np.zeros(nz)
    mean[:m] = mu0
    A = np.zeros((m, nz))                      # x_k = x_0 + sum_s w_s
    A[:, :m] = np.eye(m)
    for s in range(k):
        A[:, m + s * m:m + (s + 1) * m] = np.eye(m)
    B = np.zeros((k * p, nz))                  # y_t = H x_t + v_t
    for t in range(k):
        B[t * p:(t + 1) * p, :m] = H
        for s in range(t + 1):
            B[t * p:(t + 1) * p, m + s * m:m + (s + 1) * m] = H
        B[t * p:(t + 1) * p, m + k * m + t * p:m + k * m + (t + 1) * p] = np.eye(p)
    cxy = A @ cov @ B.T
    cyy = B @ cov @ B.T
    Y = np.concatenate(ys[:k])
    gain = np.linalg.solve(cyy, cxy.T).T
    post_mean = A @ mean + gain @ (Y - B @ mean)
    post_cov = A @ cov @ A.T - gain @ cxy.T
    return post_mean, post_cov


@pytest.mark.parametrize("k", [1, 2, 5])
def test_brute_force_conditioning(k):
    Q, H, R, P0, mu0, ys = _small_problem()
    xs, var, Ps = kf_dense.dense_kf(Q, H, R, mu0, P0, ys)
    pm, pc = _brute_force_posterior(Q, H, R, P0, mu0, ys, k)
    assert _rel(xs[k - 1], pm) < 1e-11
    assert _rel(Ps[k - 1], pc) < 1e-11


def test_covariance_psd_and_variance_shrinks():
    Q, H, R, P0, mu0, ys = _small_problem()
    xs, var, Ps = kf_dense.dense_kf(Q, H, R, mu0, P0, ys)
    prev = np.diag(P0)
    for k in range(len(ys)):
        P = Ps[k]
        assert np.abs(P - P.T).max() < 1e-12 * np.abs(P).max()
        assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > -1e-12 * np.abs(P).max()
        assert np.all(var[k] <= prev + np.diag(Q) + 1e-14)
        prev = var[k]


def test_tier_b_equals_tier_a_small():
    Q, H, R, P0, mu0, ys = _small_problem()
    xa, va, _ = kf_dense.dense_kf(Q, H, R, mu0, P0, ys)
    xb, vb = kf_crosscov.crosscov_kf(Q @ H.T, H, R, mu0, P0 @ H.T,
                                     np.diag(P0), np.diag(Q), ys)
    assert _rel(xb, xa) < 1e-12
    assert _rel(vb, va) < 1e-12


def test_tier_b_equals_tier_a_crosswell():
    w = synth.workload("crosswell-32x32-p16")
    n, p, m = w["n"], w["p"], w["m"]
    rp, col, val = synth.crosswell_h(2, n, p)
    pts = synth.cell_centres(2, n)
    H = cq_exact.h_dense(rp, col, val, m)
    Q = kernels.dense_q(pts, "powexp", w["theta"], w["ell"], w["gamma"])
    R = w["r_var"] * np.eye(p)
    _, ys = truth.random_walk_stream(Q, H, w["r_var"], 4, w["seed"])
    xa, va, _ = kf_dense.dense_kf(Q, H, R, np.zeros(m), Q, ys)
    CQ = Q @ H.T
    xb, vb = kf_crosscov.crosscov_kf(CQ, H, R, np.zeros(m), CQ, np.diag(Q),
                                     w["theta"], ys)
    for k in range(len(ys)):
        assert _rel(xb[k], xa[k]) < 1e-11
        assert _rel(vb[k], va[k]) < 1e-11


def test_tier_b_z_history_rebuilds_tier_a_covariance():
    # P_t = P_0 + t Q - sum_s Z_s Z_s^T with Z_s = C_{s|s-1} L_s^{-T}: the
    # cross-covariance filter carries enough to rebuild tier A's full P_t
    Q, H, R, P0, mu0, ys = _small_problem()
    _, _, Ps = kf_dense.dense_kf(Q, H, R, mu0, P0, ys)
    _, _, zs = kf_crosscov.crosscov_kf(Q @ H.T, H, R, mu0, P0 @ H.T, np.diag(P0),
                                       np.diag(Q), ys, return_Z=True)
    for t in range(1, len(ys) + 1):
        P = P0 + t * Q - sum(z @ z.T for z in zs[:t])
        assert _rel(P, Ps[t - 1]) < 1e-12, t


def test_tier_b_row_subset_is_exact():
    # rows outside the ray cells do not influence the update (Sec. 3.1)
    w = synth.workload("crosswell-32x32-p16")
    n, p, m = w["n"], w["p"], w["m"]
    rp, col, val = synth.crosswell_h(2, n, p)
    pts = synth.cell_centres(2, n)
    H = cq_exact.h_dense(rp, col, val, m)
    Q = kernels.dense_q(pts, "powexp", 1.0, 0.3, 1.0)
    CQ = Q @ H.T
    ys = np.random.default_rng(0).standard_normal((3, p))
    R = 1e-4 * np.eye(p)
    xf, vf = kf_crosscov.crosscov_kf(CQ, H, R, np.zeros(m), CQ, np.ones(m), 1.0, ys)
    rows = np.union1d(np.unique(col), np.arange(0, m, 37))
    xs, vs = kf_crosscov.crosscov_kf(CQ[rows], H[:, rows], R, np.zeros(len(rows)),
                                     CQ[rows], np.ones(len(rows)), 1.0, ys)
    np.testing.assert_allclose(xs, xf[:, rows], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(vs, vf[:, rows], rtol=1e-12, atol=1e-13)


def test_posterior_crosscov_identity():
    Q, H, R, P0, mu0, ys = _small_problem()
    C = (P0 + Q) @ H.T
    literal, kr = kf_crosscov.crosscov_gain_identity(C, H @ C, R)
    assert _rel(kr, literal) < 1e-12


def test_storage_matches_paper_table():
    # Table "table_computationtimeC++": HiKF keeps one m x n FP64
    # cross-covariance; with n = 288 rays that is 8 m n bytes.
    rows = np.loadtxt(__file__.replace("test_oracle_kf.py", "golden/storage_table.txt"))
    rng = np.random.default_rng(0)
    for nx, nz, kf_mb, _enkf, hikf_mb in rows:
        m, n = int(nx * nz), 288
        Hs = np.zeros((n, 4))
        CQ = rng.standard_normal((4, n))
        _, _, C = kf_crosscov.crosscov_kf(CQ, Hs, np.eye(n), np.zeros(4), CQ,
                                          np.ones(4), 1.0, np.zeros((1, n)),
                                          return_C=True)
        per_row = C.nbytes / C.shape[0]
        assert per_row == 8 * n
        assert round(per_row * m / 1e6, 1) == pytest.approx(hikf_mb, abs=0.06)
    # the smallest grid's KF storage is exactly one m x m FP64 matrix
    assert round(8 * 3245 ** 2 / 1e6, 1) == rows[0][2]


def test_random_walk_truth_follows_the_model():
    # Sec. 2.1: x_k = x_{k-1} + w_k, w_k ~ N(0, Q); y_k = H x_k + v_k,
    # v_k ~ N(0, R).  With a diagonal Q the square root is elementwise, so
    # the stream is fixed by the standard-normal draws taken in the order
    # x_0, then (w_k, v_k) for every k.
    m, p, steps, r_var = 5, 3, 4, 0.04
    q = np.array([0.5, 1.0, 2.0, 0.25, 3.0])
    H = np.arange(1.0, 16.0).reshape(p, m) / 10.0
    xs, ys = truth.random_walk_stream(np.diag(q), H, r_var, steps, seed=11)
    z = synth.normal_draws(11, m + steps * (m + p))
    x = np.sqrt(q) * z[:m]                     # x_0 ~ N(0, P_0 = Q)
    off = m
    for k in range(steps):
        x = x + np.sqrt(q) * z[off:off + m]
        y = H @ x + np.sqrt(r_var) * z[off + m:off + m + p]
        off += m + p
        np.testing.assert_allclose(xs[k], x, rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(ys[k], y, rtol=1e-14, atol=1e-14)


def test_pspace_recursion_identity():
    # The GPU may carry G = H C_prior and h = H x_hat across steps instead of
    # gathering them from the rows of C.  Both follow from the posterior
    # cross-covariance identity C_post = K R (= C_prior - K G, Sec. 3.1 eq.
    # eqn_KF_pred_new with S - R = G):  H C_post = G S^{-1} R, so the next
    # prior G is G S^{-1} R + H C_Q; and H x_hat_post = h + G S^{-1} nu.
    # Pinned here on the literal tier-B recursion, without any GPU.
    w = synth.workload("crosswell-32x32-p16")
    n, p, m = w["n"], w["p"], w["m"]
    rp, col, val = synth.crosswell_h(2, n, p)
    H = cq_exact.h_dense(rp, col, val, m)
    Q = kernels.dense_q(synth.cell_centres(2, n), "powexp", 1.0, 0.3, 1.0)
    CQ = Q @ H.T
    GQ = H @ CQ
    R = 1e-4 * np.eye(p)
    _, ys = truth.random_walk_stream(Q, H, 1e-4, 5, 0)
    C, x = CQ.copy(), np.zeros(m)
    G_rec = h_rec = None
    for y in ys:
        C = C + CQ
        G = H @ C
        h = H @ x
        if G_rec is not None:
            assert _rel(G_rec, G) < 1e-12 and _rel(h_rec, h) < 1e-12
        S = 0.5 * (G + G.T) + R
        K = np.linalg.solve(S, C.T).T
        nu = y - h
        Sinv = np.linalg.inv(S)
        G_rec = G @ Sinv @ R + GQ
        h_rec = h + G @ Sinv @ nu
        x = x + K @ nu
        C = C - K @ G
        # the recursion's value for H C_post, before the next prediction
        assert _rel(H @ C, G @ Sinv @ R) < 1e-11


def test_psd_part_is_the_nearest_psd_matrix():
    # PSD, idempotent, identity on PSD matrices, and never farther from a PSD
    # matrix than its argument (projection onto a convex set)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((12, 12))
    P = B @ B.T
    E = rng.standard_normal((12, 12)) * 0.3
    A = P + 0.5 * (E + E.T)
    Ap = kf_crosscov.psd_part(A)
    assert np.linalg.eigvalsh(Ap).min() > -1e-12 * np.abs(Ap).max()
    assert _rel(kf_crosscov.psd_part(Ap), Ap) < 1e-13
    assert _rel(kf_crosscov.psd_part(P), P) < 1e-13
    assert np.linalg.norm(Ap - P) <= np.linalg.norm(A - P) + 1e-12
    # the nearest PSD matrix: any other PSD candidate is at least as far
    for _ in range(5):
        Z = rng.standard_normal((12, 12))
        cand = Ap + 0.01 * Z @ Z.T
        assert np.linalg.norm(A - cand) >= np.linalg.norm(A - Ap) - 1e-12


def test_guarded_filter_equals_tier_b_when_hqh_is_psd():
    # with the exact C_Q the measurement-space prior H Q H^T is PSD, the
    # projection changes nothing and the carried G equals H C_prior: the
    # guarded filter is tier B
    w = synth.workload("crosswell-32x32-p16")
    n, p, m = w["n"], w["p"], w["m"]
    rp, col, val = synth.crosswell_h(2, n, p)
    H = cq_exact.h_dense(rp, col, val, m)
    Q = kernels.dense_q(synth.cell_centres(2, n), "powexp", 1.0, 0.3, 1.0)
    CQ = Q @ H.T
    R = 1e-4 * np.eye(p)
    _, ys = truth.random_walk_stream(Q, H, 1e-4, 6, 0)
    assert np.linalg.eigvalsh(0.5 * (H @ CQ + (H @ CQ).T)).min() > 0
    xb, vb = kf_crosscov.crosscov_kf(CQ, H, R, np.zeros(m), CQ, np.ones(m), 1.0, ys)
    xg, vg = kf_crosscov.crosscov_kf_guarded(CQ, H, R, np.zeros(m), CQ, np.ones(m), 1.0, ys,
                                             G0=2.0 * kf_crosscov.psd_part(H @ CQ))
    assert _rel(xg, xb) < 1e-9 and _rel(vg, vb) < 1e-11


def test_guard_keeps_s_positive_definite_where_the_fmm_prior_fails():
    # A smooth Gaussian kernel (ell = 0.2 on 64 x 64, p = 64): the oracle's
    # FP64 bbFMM C_Q at n_c = 6 makes H Q H^T indefinite, and the literal
    # filter's S loses definiteness within the 40 steps; the guarded filter
    # runs on with positive variances.  Its variances stay within 2e-2 of
    # the guarded filter on the exact C_Q; x_hat does not (the gain
    # amplifies the H^2 error of n_c = 6 into O(1) errors on this
    # ill-conditioned problem), which is the accuracy side of the same
    # limitation and is reported, not hidden.
    from oracle import bbfmm
    n, p = 64, 64
    rp, col, val = synth.crosswell_h(2, n, p)
    m = n * n
    H = cq_exact.h_dense(rp, col, val, m)
    cq = bbfmm.bbfmm_apply(2, n, H.T, 6, 8, "powexp", 1.0, 0.2, 2.0)
    cqe = cq_exact.cq_fft(2, n, H.T, "powexp", 1.0, 0.2, 2.0)
    assert np.linalg.eigvalsh(0.5 * (H @ cq + (H @ cq).T)).min() < 0
    R = 1e-4 * np.eye(p)
    ys = np.random.default_rng(4).standard_normal((40, p)) * 1e-2
    with pytest.raises(np.linalg.LinAlgError):
        kf_crosscov.crosscov_kf(cq, H, R, np.zeros(m), cq, np.ones(m), 1.0, ys)
    xg, vg = kf_crosscov.crosscov_kf_guarded(cq, H, R, np.zeros(m), cq, np.ones(m), 1.0, ys,
                                             G0=2.0 * kf_crosscov.psd_part(H @ cq))
    xe, ve = kf_crosscov.crosscov_kf_guarded(cqe, H, R, np.zeros(m), cqe, np.ones(m), 1.0, ys,
                                             G0=2.0 * kf_crosscov.psd_part(H @ cqe))
    assert np.all(np.isfinite(xg)) and np.all(vg > 0)
    assert max(_rel(vg[k], ve[k]) for k in range(len(ys))) < 2e-2
