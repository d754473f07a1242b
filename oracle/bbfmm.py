"""FP64 black-box FMM for Q W on a uniform grid -- test infrastructure only.

Sec. 3.2 computes Q H^T with the fast multipole method, representing
well-separated kernel blocks by Chebyshev interpolation (the black-box FMM of
Fong & Darve 2009, which the paper cites for it).  This module follows those
steps in plain NumPy, in FP64, on the uniform tree of a cell-centred
N^dim grid (leaves of ``leaf`` cells per axis, levels 0..D with
N = leaf * 2^D):

1. Chebyshev nodes xi_k = cos((2k+1) pi / (2 n_c)), k = 0..n_c-1, mapped to
   every box; S(xi, x) = 1/n_c + (2/n_c) sum_{l=1}^{n_c-1} T_l(xi) T_l(x),
   tensor product over axes (box-normalised coordinates).
2. P2M   M_B[k]  = sum_{j in B} S(xi_k, x_j) w_j                  (leaves)
3. M2M   M_P[k]  = sum_children sum_k' S(xi_k, x_k'^child) M_c[k']
4. M2L   L_B[k] += sum_{A in IL(B)} sum_k' K(x_k^B, x_k'^A) M_A[k']
         IL(B) = children of the parent's neighbours that are not
         neighbours of B (levels 2..D)
5. L2L   L_c[k'] += sum_k S(xi_k, x_k'^c) L_P[k]          (transpose of 3)
6. L2P   f_i += sum_k S(xi_k, x_i) L_leaf[k]
7. P2P   f_i += sum_{A adjacent to leaf(i), incl. itself} sum_{j in A}
         K(x_i, x_j) w_j

Arrays are held coordinate-major: box arrays have shape
(2^l,)*dim + (r, p) with axis 0 = x; node and point multi-indices are
flattened in C order over (x, y[, z]), which is the order of ``numpy.kron``.
Every operator acts on the node (or point) axis of all boxes and all
right-hand sides at once: ``numpy.matmul(op, X)`` with X of shape
(..., nodes, p) gives out[..., a, c] = sum_b op[a, b] X[..., b, c].
"""

import itertools

import numpy as np
from numpy.polynomial import chebyshev as npcheb

from .kernels import kernel


def cheb_nodes(nc):
    k = np.arange(nc)
    return np.cos((2 * k + 1) * np.pi / (2 * nc))


def interp_matrix(nc, x):
    """S[k, j] = S_{n_c}(xi_k, x_j) for normalised coordinates x in [-1, 1]."""
    Txi = npcheb.chebvander(cheb_nodes(nc), nc - 1)
    Tx = npcheb.chebvander(np.asarray(x, np.float64), nc - 1)
    return (1.0 + 2.0 * Txi[:, 1:] @ Tx[:, 1:].T) / nc


def _kron_all(mats):
    out = mats[0]
    for a in mats[1:]:
        out = np.kron(out, a)
    return out


def _multi(nc, dim):
    """(nc^dim, dim) multi-indices in C order over (x, y[, z])."""
    return np.array(list(itertools.product(range(nc), repeat=dim)))


def tree_depth(n, leaf):
    nl = n // leaf
    if n % leaf or nl & (nl - 1):
        raise ValueError("N / leaf must be a power of two")
    return int(round(np.log2(nl)))


def padded_size(n, leaf):
    """Cells per axis of the tree for an N-cell axis: the smallest
    leaf * 2^D >= N (reading for grids that are not leaf * 2^D)."""
    npad = leaf
    while npad < n:
        npad *= 2
    return npad


def _to_leaves(W, dim, n, leaf):
    """Grid-order (m, p) -> (nl,)*dim + (leaf^dim, p), coordinate-major."""
    p = W.shape[1]
    nl = n // leaf
    a = W.reshape((n,) * dim + (p,))
    a = a.transpose(tuple(range(dim - 1, -1, -1)) + (dim,))      # x first
    a = a.reshape(sum(((nl, leaf) for _ in range(dim)), ()) + (p,))
    perm = tuple(2 * i for i in range(dim)) + tuple(2 * i + 1 for i in range(dim))
    a = a.transpose(perm + (2 * dim,))
    return a.reshape((nl,) * dim + (leaf ** dim, p))


def _from_leaves(F, dim, n, leaf):
    """Inverse of ``_to_leaves``."""
    p = F.shape[-1]
    nl = n // leaf
    a = F.reshape((nl,) * dim + (leaf,) * dim + (p,))
    perm = []
    for i in range(dim):
        perm += [i, dim + i]
    a = a.transpose(tuple(perm) + (2 * dim,))
    a = a.reshape((n,) * dim + (p,))
    a = a.transpose(tuple(range(dim - 1, -1, -1)) + (dim,))
    return a.reshape(n ** dim, p)


def _il_axis_targets(nb, o):
    """Target box indices along one axis for which offset o is in IL."""
    b = np.arange(nb)
    ok = (b + o >= 0) & (b + o < nb)
    even = (b % 2) == 0
    ok &= np.where(even, (o >= -2) & (o <= 3), (o >= -3) & (o <= 2))
    return b[ok]


def il_offsets(dim):
    return [o for o in itertools.product(range(-3, 4), repeat=dim)
            if max(abs(v) for v in o) >= 2]


def interaction_counts(dim, n, leaf):
    """(near pairs, interaction-list pairs) of the uniform (padded) tree."""
    D = tree_depth(padded_size(n, leaf), leaf)
    nl = 2 ** D
    near = 0
    for o in itertools.product((-1, 0, 1), repeat=dim):
        near += int(np.prod([nl - abs(v) for v in o]))
    far = 0
    for lev in range(2, D + 1):
        nb = 2 ** lev
        for o in il_offsets(dim):
            far += int(np.prod([len(_il_axis_targets(nb, v)) for v in o]))
    return near, far


def lowrank_basis(T_list, eps):
    """Common basis of a level's M2L operators (the SVD compression of the
    black-box FMM): the left singular vectors of [T_o1 T_o2 ...] whose
    singular values are at least eps times the largest.  The kernel is
    symmetric and the interaction list closed under o -> -o (T_-o = T_o^T),
    so the same basis serves the sources.  Returns U (r x k)."""
    fat = np.hstack(T_list)
    U, sv, _ = np.linalg.svd(fat, full_matrices=False)
    k = int((sv >= eps * sv[0]).sum()) if sv[0] > 0 else 1
    return U[:, :max(k, 1)]


def bbfmm_apply(dim, n, W, nc, leaf=None, family="powexp", theta=1.0,
                ell=1.0, gamma=1.0, svd_eps=None):
    """Approximate Q @ W (W is (m, p) in grid order) by the black-box FMM.

    An N that is not leaf * 2^D is handled by the padded-tree reading: the
    tree covers Npad = padded_size(N, leaf) cells per axis of the same size
    h = 1/N (root box [0, Npad h]^dim), the cells beyond N carry zero weight,
    and only the N^dim real rows are returned.

    svd_eps: if given, every level's M2L runs in the compressed form
    U (U^T T_o U) (U^T M) with the basis U of ``lowrank_basis`` at that
    relative singular-value threshold (the low-rank M2L of the black-box
    FMM; ranks follow the decay of the operators' singular values)."""
    if leaf is None:
        leaf = 8 if dim == 2 else 4
    W = np.asarray(W, np.float64)
    if W.ndim == 1:
        W = W[:, None]
    npad = padded_size(n, leaf)
    if npad != n:
        p = W.shape[1]
        Wp = np.zeros((npad,) * dim + (p,))
        Wp[(slice(0, n),) * dim] = W.reshape((n,) * dim + (p,))
        out = _bbfmm_tree(dim, npad, 1.0 / n, Wp.reshape(npad ** dim, p), nc, leaf,
                          family, theta, ell, gamma, svd_eps)
        return out.reshape((npad,) * dim + (p,))[(slice(0, n),) * dim].reshape(n ** dim, p)
    return _bbfmm_tree(dim, n, 1.0 / n, W, nc, leaf, family, theta, ell, gamma, svd_eps)


def _bbfmm_tree(dim, n, h, W, nc, leaf, family, theta, ell, gamma, svd_eps=None):
    """The FMM passes on a tree of n = leaf * 2^D cells per axis of side h
    (grid-order layout of ``W`` and of the result, the first axis fastest)."""
    K = kernel(family, theta, ell, gamma)
    D = tree_depth(n, leaf)
    xi = cheb_nodes(nc)
    kidx = _multi(nc, dim)
    lidx = _multi(leaf, dim)
    xi_vec = xi[kidx]                                    # (r, dim)

    # leaf interpolation and child transfer operators (steps 1-3)
    u = (np.arange(leaf) + 0.5 - leaf / 2.0) / (leaf / 2.0)
    S1 = interp_matrix(nc, u)
    S_leaf = _kron_all([S1] * dim)                       # (r, leaf^dim)
    S_half = [interp_matrix(nc, -0.5 + 0.5 * xi), interp_matrix(nc, 0.5 + 0.5 * xi)]

    Wl = _to_leaves(W, dim, n, leaf)
    F = np.zeros_like(Wl)

    # 7. P2P over adjacent leaves (including the leaf itself)
    nl = 2 ** D
    for o in itertools.product((-1, 0, 1), repeat=dim):
        diff = (np.asarray(o)[None, None, :] * leaf
                + lidx[None, :, :] - lidx[:, None, :]) * h
        Ko = K(np.sqrt((diff * diff).sum(-1)))           # (tgt, src)
        tsl = tuple(slice(max(0, -v), nl - max(0, v)) for v in o)
        ssl = tuple(slice(max(0, v), nl - max(0, -v)) for v in o)
        F[tsl] += np.matmul(Ko, Wl[ssl])

    if D >= 2:
        # 2. P2M
        M = {D: np.matmul(S_leaf, Wl)}
        # 3. M2M, levels D-1 .. 2
        for lev in range(D - 1, 1, -1):
            child = M[lev + 1]
            acc = np.zeros((2 ** lev,) * dim + child.shape[dim:])
            for c in itertools.product((0, 1), repeat=dim):
                Sc = _kron_all([S_half[v] for v in c])
                sl = tuple(slice(v, None, 2) for v in c)
                acc += np.matmul(Sc, child[sl])
            M[lev] = acc
        # 4. M2L, levels 2 .. D
        L = {}
        for lev in range(2, D + 1):
            nb = 2 ** lev
            s = n * h / nb                                # box side
            Ts = {}
            for o in il_offsets(dim):
                diff = s * (np.asarray(o)[None, None, :]
                            + 0.5 * (xi_vec[None, :, :] - xi_vec[:, None, :]))
                Ts[o] = K(np.sqrt((diff * diff).sum(-1)))    # (k tgt, k' src)
            Mlev = M[lev]
            if svd_eps is not None:
                U = lowrank_basis(list(Ts.values()), svd_eps)
                Ts = {o: U.T @ T @ U for o, T in Ts.items()}
                Mlev = np.matmul(U.T, Mlev)               # compressed multipoles
            acc = np.zeros(Mlev.shape)
            for o, T in Ts.items():
                tb = [_il_axis_targets(nb, v) for v in o]
                if any(len(t) == 0 for t in tb):
                    continue
                sb = [t + v for t, v in zip(tb, o)]
                src = Mlev[np.ix_(*sb)]
                acc[np.ix_(*tb)] += np.matmul(T, src)
            L[lev] = np.matmul(U, acc) if svd_eps is not None else acc
        # 5. L2L, levels 2 .. D-1 -> children
        for lev in range(2, D):
            for c in itertools.product((0, 1), repeat=dim):
                Sc = _kron_all([S_half[v] for v in c])
                sl = tuple(slice(v, None, 2) for v in c)
                L[lev + 1][sl] += np.matmul(Sc.T, L[lev])
        # 6. L2P
        F += np.matmul(S_leaf.T, L[D])

    return _from_leaves(F, dim, n, leaf)
