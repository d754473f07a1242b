"""Random-walk truths with covariance Q -- test infrastructure only.

Sec. 2.1: x_t = x_{t-1} + w_t (eq. ``equation_random_walk``), w_t ~ N(0, Q),
z_t = H x_t + v_t with v_t ~ N(0, R); the initial state has mean mu_0 and
covariance P_0.  Standard-normal draws come from ``synth.normal_draws`` in
the order x_0, then (w_k, v_k) for k = 1..steps.
"""

import numpy as np

from synth import normal_draws


def _sqrt_psd(A):
    """Symmetric square root of a PSD matrix (tiny negative eigenvalues,
    which rounding produces for smooth kernels, are clipped to zero)."""
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.sqrt(np.clip(w, 0.0, None))) @ V.T


def random_walk_stream(Q, H, r_var, steps, seed, P0=None, mu0=None):
    """Truth states and observations for a dense Q (small m).

    Returns (x_true (steps, m), y (steps, p)) with x_0 ~ N(mu0, P0)
    (P0 defaults to Q, mu0 to 0).
    """
    m = Q.shape[0]
    p = H.shape[0]
    P0 = Q if P0 is None else P0
    mu0 = np.zeros(m) if mu0 is None else mu0
    z = normal_draws(seed, m + steps * (m + p))
    sq, s0 = _sqrt_psd(Q), _sqrt_psd(P0)
    x = mu0 + s0 @ z[:m]
    xs, ys = [], []
    off = m
    for _ in range(steps):
        w = z[off:off + m]
        v = z[off + m:off + m + p]
        off += m + p
        x = x + sq @ w
        xs.append(x.copy())
        ys.append(H @ x + np.sqrt(r_var) * v)
    return np.array(xs), np.array(ys)

