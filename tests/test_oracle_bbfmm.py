"""Pins for the FP64 black-box FMM oracle (Sec. 3.2).

* Chebyshev interpolation with n_c >= 3 nodes per axis reproduces a kernel
  of degree 2 in every coordinate exactly, so every pass and list must give
  the dense product to rounding (catches a wrong operator, sign, index or
  list).
* The approximate Q is symmetric (M2L for offset -o is the transpose of
  offset o, L2L the transpose of M2M), so u^T (Q v) = v^T (Q u).
* The error against the exact product falls geometrically with n_c (the
  trend of Table ``table_bbfmm``; its values are parity unpinned).
* The near and interaction-list pair totals equal closed-form counts.
"""

import os

import numpy as np
import pytest

import synth
from oracle import bbfmm, cq_exact, kernels


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dim,n,leaf,nc", [(2, 32, 8, 3), (2, 64, 8, 4),
                                           (2, 64, 8, 5), (3, 16, 4, 3),
                                           (3, 16, 4, 4)])
def test_polynomial_kernel_is_exact(dim, n, leaf, nc):
    rng = np.random.default_rng(7)
    W = rng.standard_normal((n ** dim, 3))
    pts = synth.cell_centres(dim, n)
    exact = cq_exact.cq_dense(pts, W, "r2", 1.0)
    approx = bbfmm.bbfmm_apply(dim, n, W, nc, leaf, "r2", 1.0)
    assert _rel(approx, exact) < 1e-13


def test_symmetry():
    rng = np.random.default_rng(2)
    n = 64
    u = rng.standard_normal((n * n, 1))
    v = rng.standard_normal((n * n, 1))
    Qu = bbfmm.bbfmm_apply(2, n, u, 4, 8, "powexp", 1.0, 0.1, 1.0)
    Qv = bbfmm.bbfmm_apply(2, n, v, 4, 8, "powexp", 1.0, 0.1, 1.0)
    a, b = float((u.T @ Qv)[0, 0]), float((v.T @ Qu)[0, 0])
    assert abs(a - b) < 1e-13 * (abs(a) + abs(b) + np.abs(u).sum() * np.abs(Qv).max())


def test_linearity():
    rng = np.random.default_rng(4)
    n = 32
    W = rng.standard_normal((n * n, 2))
    F = bbfmm.bbfmm_apply(2, n, W, 4, 8, "powexp", 1.0, 0.2, 1.0)
    G = bbfmm.bbfmm_apply(2, n, W @ np.array([[2.0], [-3.0]]), 4, 8, "powexp", 1.0, 0.2, 1.0)
    assert _rel(G, F @ np.array([[2.0], [-3.0]])) < 1e-13


@pytest.mark.parametrize("n,ell,gamma", [(256, 0.05, 2.0), (64, 0.3, 1.0)])
def test_geometric_convergence(n, ell, gamma):
    rng = np.random.default_rng(5)
    W = rng.standard_normal((n * n, 2))
    exact = cq_exact.cq_fft(2, n, W, "powexp", 1.0, ell, gamma)
    errs = [_rel(bbfmm.bbfmm_apply(2, n, W, nc, 8, "powexp", 1.0, ell, gamma), exact)
            for nc in (3, 4, 5, 6, 7)]
    for a, b in zip(errs, errs[1:]):
        assert b < a * 0.6
    # Table "table_bbfmm" reports ~1e-9 at 5 nodes and ~3e-11 at 7 nodes for
    # a Gaussian kernel on an unstated workload; here only the geometric
    # decay is checked.
    assert errs[-1] < 1e-5


@pytest.mark.parametrize("dim,n,leaf", [(2, 256, 8), (2, 1024, 8), (3, 128, 4), (2, 32, 8)])
def test_pair_counts_closed_form(dim, n, leaf):
    near, far = bbfmm.interaction_counts(dim, n, leaf)
    nl = n // leaf
    assert near == (nl + 2 * (nl - 1)) ** dim
    D = int(np.log2(nl))
    # per axis and level: pairs whose parents are within one box, minus
    # pairs that are themselves within one box
    closed = sum((6 * 2 ** l - 8) ** dim - (3 * 2 ** l - 2) ** dim
                 for l in range(2, D + 1))
    assert far == closed


def test_interior_list_sizes():
    # an interior box has 27 (2-D) / 189 (3-D) interaction-list entries
    for dim in (2, 3):
        counts = 0
        for o in bbfmm.il_offsets(dim):
            if all(len(bbfmm._il_axis_targets(16, v)) and
                   (5 in bbfmm._il_axis_targets(16, v)) for v in o):
                counts += 1
        assert counts == (27 if dim == 2 else 189)


@pytest.mark.parametrize("dim,n,nc", [(2, 40, 3), (2, 20, 4), (3, 12, 3), (3, 6, 3)])
def test_padded_tree_polynomial_kernel_exact(dim, n, nc):
    # N not of the form leaf * 2^D: the tree is padded with zero-weight cells
    # (root box Npad / N); Chebyshev interpolation is still exact for K = r^2,
    # so the product must equal the dense one (catches padding, scaling and
    # index mistakes)
    rng = np.random.default_rng(5)
    m = n ** dim
    W = rng.standard_normal((m, 3))
    Q = kernels.dense_q(synth.cell_centres(dim, n), "r2", 1.0, 1.0, 1.0)
    got = bbfmm.bbfmm_apply(dim, n, W, nc, None, "r2", 1.0, 1.0, 1.0)
    np.testing.assert_allclose(got, Q @ W, rtol=1e-12, atol=1e-12 * np.abs(Q @ W).max())


def test_padded_tree_converges_for_smooth_kernel():
    n = 40
    pts = synth.cell_centres(2, n)
    W = np.random.default_rng(6).standard_normal((n * n, 2))
    ref = kernels.dense_q(pts, "powexp", 1.0, 0.3, 1.0) @ W
    errs = [np.linalg.norm(bbfmm.bbfmm_apply(2, n, W, nc, None, "powexp", 1.0, 0.3, 1.0) - ref)
            / np.linalg.norm(ref) for nc in (3, 4, 5, 6)]
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(3)), errs


def _paper_table():
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "bbfmm_table.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            dim_s, nodes, err = line.split()
            rows.append((int(dim_s), int(nodes), float(err)))
    return rows


def test_convergence_trend_of_paper_table():
    # Table "table_bbfmm" (Sec. 3.3): for a Gaussian kernel the relative
    # accuracy improves by a factor that grows with the node count (x7.0 from
    # 5 to 6 nodes, x17.8 from 6 to 7 at state dimension 1e4), and at 7 nodes
    # it is the same for 1e4 and 1e5 unknowns.  Its point set, kernel length
    # and error definition are not stated (values parity unpinned), so the
    # oracle is checked for the same trend on a Gaussian of length 0.5 on
    # 128^2 and 256^2 grids (1.6e4 and 6.6e4 unknowns).
    table = _paper_table()
    t4 = {nodes: err for dim_s, nodes, err in table if dim_s == 10000}
    paper_ratio = [t4[5] / t4[6], t4[6] / t4[7]]
    assert paper_ratio[1] > paper_ratio[0] > 1.0
    errs = {}
    for n in (128, 256):
        W = np.random.default_rng(5).standard_normal((n * n, 1))
        exact = cq_exact.cq_fft(2, n, W, "powexp", 1.0, 0.5, 2.0)
        errs[n] = [_rel(bbfmm.bbfmm_apply(2, n, W, nc, 8, "powexp", 1.0, 0.5, 2.0), exact)
                   for nc in (5, 6, 7)]
    ratio = [errs[128][0] / errs[128][1], errs[128][1] / errs[128][2]]
    assert ratio[1] > ratio[0] > 1.0
    for ours, theirs in zip(ratio, paper_ratio):
        assert theirs / 4 < ours < theirs * 4, (ratio, paper_ratio)
    # like the table's 1e4 / 1e5 rows at 7 nodes: the accuracy does not
    # depend on the number of unknowns at a fixed kernel and node count
    assert abs(np.log10(errs[256][2] / errs[128][2])) < 0.5


def test_lowrank_m2l_full_rank_is_the_plain_fmm():
    # a threshold of 0 keeps every singular vector: U is orthogonal and
    # U (U^T T U)(U^T M) = T M
    rng = np.random.default_rng(9)
    W = rng.standard_normal((64 * 64, 2))
    plain = bbfmm.bbfmm_apply(2, 64, W, 4, 8, "powexp", 1.0, 0.1, 1.0)
    full = bbfmm.bbfmm_apply(2, 64, W, 4, 8, "powexp", 1.0, 0.1, 1.0, svd_eps=0.0)
    assert _rel(full, plain) < 1e-13


@pytest.mark.parametrize("dim,n,nc,ell,gamma", [(2, 128, 5, 0.05, 2.0), (3, 32, 4, 0.2, 1.0)])
def test_lowrank_m2l_error_follows_the_threshold(dim, n, nc, ell, gamma):
    # the compressed M2L adds an error of about the threshold (relative to the
    # far field) on top of the Chebyshev error, and keeps fewer than r ranks
    rng = np.random.default_rng(10)
    W = rng.standard_normal((n ** dim, 2))
    plain = bbfmm.bbfmm_apply(dim, n, W, nc, None, "powexp", 1.0, ell, gamma)
    errs = []
    for eps in (1e-3, 1e-5, 1e-7):
        lr = bbfmm.bbfmm_apply(dim, n, W, nc, None, "powexp", 1.0, ell, gamma, svd_eps=eps)
        errs.append(_rel(lr, plain))
        assert errs[-1] < 20 * eps
    # a smaller threshold never keeps fewer ranks
    assert errs[0] >= errs[1] >= errs[2] and errs[0] > errs[2]


def test_lowrank_basis_rank_and_orthonormality():
    from oracle.kernels import kernel
    K = kernel("powexp", 1.0, 0.05, 2.0)
    xi = bbfmm.cheb_nodes(5)
    xv = xi[bbfmm._multi(5, 2)]
    s = 1.0 / 128                                        # level 7 of a unit square
    Ts = []
    for o in bbfmm.il_offsets(2):
        diff = s * (np.asarray(o)[None, None, :] + 0.5 * (xv[None, :, :] - xv[:, None, :]))
        Ts.append(K(np.sqrt((diff * diff).sum(-1))))
    U = bbfmm.lowrank_basis(Ts, 1e-5)
    assert U.shape[0] == 25 and 1 <= U.shape[1] < 25
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
    # each operator is reproduced to the threshold by its projection
    for T in Ts:
        assert np.linalg.norm(U @ (U.T @ T @ U) @ U.T - T) <= 1e-4 * np.linalg.norm(np.hstack(Ts))
