"""FP64 reference of the IPFP sweep -- test infrastructure, never product code.

Notation follows the paper's Sec. 3: rows are candidates x (count N) with
margins n_x, columns are employers y (count M) with margins m_y, the entropy
scale is called ``sigma`` here (the paper's beta), and the scalings are
u_x = sqrt(mu_x0), v_y = sqrt(mu_0y) (Sec. 3.2, just before eq. 6). The
library returns them as ``a = u`` and ``b = v``.

Readings of the paper taken here (each one is listed in the design notes):

* Margin names: eq. 2 ties n to rows and m to columns. Alg. 1/2 and App. A
  swap the letters; eq. 2's convention is used throughout.
* The quadratic root of eq. 6 is evaluated in its rationalised form
  n / (s + sqrt(s^2 + n)), which is the same number as sqrt(n + s^2) - s but
  does not cancel when s >> sqrt(n).
* The kernel exp(Phi/2beta) means exp(Phi / (2 beta)), as eq. 4 requires.
* Update order (eq. 6, Alg. 1): v starts at 1; each sweep first updates every
  u from the current v, then every v from the new u.
* Convergence (the paper runs a fixed number of loops): after sweep i, when
  i is a multiple of ``check_every`` or i equals ``max_sweeps``, the row
  residual r = max_x |u_x^2 + u_x (K v)_x - n_x| / n_x of the current (u, v)
  is recorded; the solve stops when r < tol (tol = 0 never stops early).
  Column residuals vanish by construction right after the v update.

Parity status: ``ipfp_batch``, ``root``, ``row_residual`` and ``matching``
are pinned by the brute-force primal/dual solves in ``oracle.brute``, the
closed forms in ``oracle.closed`` and the invariants checked in the test
suite. ``ipfp_minibatch`` and ``half_step_rows`` are pinned against
``ipfp_batch`` (the paper states the mini-batch form is exact) and against the
closed forms. ``stable_factors`` is pinned against log(mu) of ``matching``.
``topk_matches`` is pinned against a selection loop that repeatedly takes the
largest remaining entry; ``welfare_gradient`` against central differences of
the optimal welfare computed by the IPFP-free primal Newton solve. The
converged ``ipfp_batch`` also reproduces the 60-digit equilibria of
``tests/golden/equilibria.json`` (Newton's method on eq. 5 in mpmath, written
without any code from this package).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

try:  # log-domain sums for surpluses whose kernel overflows FP64
    from scipy.special import logsumexp as _logsumexp
except Exception:  # pragma: no cover - scipy is present in this image
    _logsumexp = None


@dataclasses.dataclass
class IPFPResult:
    a: np.ndarray            # u = sqrt(mu_x0), length N
    b: np.ndarray            # v = sqrt(mu_0y), length M
    res_hist: list           # row residual at every check
    sweeps: int              # sweeps whose result is returned
    final_res: float


def surplus_from_factors(U, Q, V, P) -> np.ndarray:
    """Phi = U V^T + Q P^T in FP64 (eq. 8: p_xy = <f_x, g_y>, q_yx = <k_x, l_y>,
    phi = p + q from Sec. 3.1)."""
    U, Q, V, P = (np.asarray(t, dtype=np.float64) for t in (U, Q, V, P))
    return U @ V.T + Q @ P.T


def kernel_matrix(Phi, sigma: float) -> np.ndarray:
    """K = exp(Phi / (2 sigma)) (the matrix A of eq. 7 and Alg. 1)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    t = Phi / (2.0 * sigma)
    if t.size and np.max(np.abs(t)) >= 700.0:
        raise OverflowError("exp(Phi/2sigma) leaves FP64 range; use ipfp_logdomain")
    return np.exp(t)


def kernel_from_log2(T) -> np.ndarray:
    """K = 2^T for a surplus given in log2 units, T = Phi log2(e) / (2 sigma)
    (the same matrix as ``kernel_matrix``; 2^T = exp(Phi / 2 sigma))."""
    T = np.asarray(T, dtype=np.float64)
    if T.size and np.max(np.abs(T)) >= 1000.0:
        raise OverflowError("2^T leaves FP64 range")
    return np.exp2(T)


def root(marg, s):
    """Positive root w of w^2 + 2 s w - marg = 0, i.e. sqrt(marg + s^2) - s
    (eq. 6), evaluated as marg / (s + sqrt(s^2 + marg)). For s beyond 1e150 the
    square would overflow and marg / (2 s) is exact to FP64 rounding."""
    marg = np.asarray(marg, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    big = s > 1e150
    s_safe = np.where(big, 0.0, s)
    w = marg / (s_safe + np.sqrt(s_safe * s_safe + marg))
    return np.where(big, marg / (2.0 * np.where(big, s, 1.0)), w)


def row_residual(K, a, b, n) -> float:
    """max_x |u_x^2 + u_x (K v)_x - n_x| / n_x: the first margin equation of
    eq. 5 with u = sqrt(mu_x0), v = sqrt(mu_0y)."""
    Kv = K @ b
    return float(np.max(np.abs(a * a + a * Kv - n) / n))


def col_residual(K, a, b, m) -> float:
    """max_y |v_y^2 + v_y (K^T u)_y - m_y| / m_y (second equation of eq. 5)."""
    Ktu = K.T @ a
    return float(np.max(np.abs(b * b + b * Ktu - m) / m))


def _checks(i: int, max_sweeps: int, check_every: int) -> bool:
    return i % check_every == 0 or i == max_sweeps


def ipfp_batch(K, n, m, tol: float = 0.0, max_sweeps: int = 100,
               check_every: int = 1, b0=None) -> IPFPResult:
    """Batch IPFP (eq. 7, Alg. 1) on an explicit kernel matrix K (N x M).

    Every sweep computes s = K v / 2 and u = root(n, s), then s = K^T u / 2 and
    v = root(m, s). ``b0`` optionally replaces the initial v = 1 (a warm start;
    the initial u is never read)."""
    K = np.asarray(K, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N, M = K.shape
    v = np.ones(M) if b0 is None else np.array(b0, dtype=np.float64)
    u = np.ones(N)
    hist = []
    i = 0
    for i in range(1, max_sweeps + 1):
        u = root(n, 0.5 * (K @ v))
        v = root(m, 0.5 * (K.T @ u))
        if _checks(i, max_sweeps, check_every):
            r = row_residual(K, u, v, n)
            hist.append(r)
            if r < tol:
                break
    final = hist[-1] if hist else float("nan")
    return IPFPResult(u, v, hist, i, final)


def ipfp_logdomain(Phi, n, m, sigma: float, tol: float = 0.0,
                   max_sweeps: int = 100, check_every: int = 1,
                   b0=None) -> IPFPResult:
    """The same iteration as ``ipfp_batch`` with every kernel sum taken as a
    log-sum-exp, for surpluses where exp(Phi/2sigma) leaves FP64 range."""
    T = np.asarray(Phi, dtype=np.float64) / (2.0 * sigma)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N, M = T.shape
    v = np.ones(M) if b0 is None else np.array(b0, dtype=np.float64)
    u = np.ones(N)
    hist = []
    i = 0

    def row_sum(vv):   # (K v)_x = exp(LSE_y(T_xy + log v_y))
        return np.exp(_logsumexp(T + np.log(vv)[None, :], axis=1))

    for i in range(1, max_sweeps + 1):
        u = root(n, 0.5 * row_sum(v))
        v = root(m, 0.5 * np.exp(_logsumexp(T + np.log(u)[:, None], axis=0)))
        if _checks(i, max_sweeps, check_every):
            r = float(np.max(np.abs(u * u + u * row_sum(v) - n) / n))
            hist.append(r)
            if r < tol:
                break
    final = hist[-1] if hist else float("nan")
    return IPFPResult(u, v, hist, i, final)


def matching(K, a, b) -> np.ndarray:
    """mu_xy = K_xy u_x v_y (eq. 4 and the last step of Alg. 1)."""
    return np.asarray(K, dtype=np.float64) * np.outer(a, b)


# --- mini-batch form (Sec. 3.3) ----------------------------------------------

def half_step_rows(W_rows, Z, other, sigma: float) -> np.ndarray:
    """s_j = A_j w / 2 for one mini-batch of rows (eq. 9-10).

    ``W_rows`` are the batch's concatenated factors [f|k] (B x 2D), ``Z`` the
    other side's [g|l] (L x 2D), ``other`` the other side's current scaling.
    The slab A_j = exp(W_rows Z^T / 2 sigma) is formed and dropped here."""
    W_rows = np.asarray(W_rows, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    A = np.exp((W_rows @ Z.T) / (2.0 * sigma))
    return 0.5 * (A @ np.asarray(other, dtype=np.float64))


def ipfp_minibatch(U, Q, V, P, n, m, sigma: float, batch_x: int,
                   batch_y: int, tol: float = 0.0, max_sweeps: int = 100,
                   check_every: int = 1, b0=None) -> IPFPResult:
    """Mini-batch IPFP (eq. 9-10, Alg. 2): the kernel is never stored whole;
    each batch of B rows (then of B columns) forms its slab from the factors,
    takes its sum against the other side's current scaling and updates its own
    scalings. All u_j of one half-step read the same v, so the result equals
    batch IPFP's (Sec. 3.3)."""
    X = np.concatenate([np.asarray(U, np.float64), np.asarray(Q, np.float64)], 1)
    Y = np.concatenate([np.asarray(V, np.float64), np.asarray(P, np.float64)], 1)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N, M = X.shape[0], Y.shape[0]
    v = np.ones(M) if b0 is None else np.array(b0, dtype=np.float64)
    u = np.ones(N)
    hist = []
    i = 0

    def row_pass(vv):
        s = np.empty(N)
        for j in range(0, N, batch_x):
            s[j:j + batch_x] = half_step_rows(X[j:j + batch_x], Y, vv, sigma)
        return s

    for i in range(1, max_sweeps + 1):
        u = root(n, row_pass(v))
        s = np.empty(M)
        for j in range(0, M, batch_y):
            s[j:j + batch_y] = half_step_rows(Y[j:j + batch_y], X, u, sigma)
        v = root(m, s)
        if _checks(i, max_sweeps, check_every):
            r = float(np.max(np.abs(u * u + 2.0 * u * row_pass(v) - n) / n))
            hist.append(r)
            if r < tol:
                break
    final = hist[-1] if hist else float("nan")
    return IPFPResult(u, v, hist, i, final)


def stable_factors(U, Q, V, P, a, b, sigma: float):
    """Stable factors psi_x, xi_y with log mu_xy = <psi_x, xi_y> / (2 sigma)
    (eq. 11, Alg. 2's last two steps).

    Reading: the printed psi carries beta*log(u); with u = sqrt(mu_x0) that
    would give mu = K sqrt(u v), against eq. 4 and Alg. 1. The entries here are
    2 sigma log u = sigma log mu_x0 and 2 sigma log v, which reproduce eq. 4."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    N, M = len(a), len(b)
    psi = np.concatenate([np.asarray(U, np.float64), np.asarray(Q, np.float64),
                          (2.0 * sigma * np.log(a))[:, None], np.ones((N, 1))], 1)
    xi = np.concatenate([np.asarray(V, np.float64), np.asarray(P, np.float64),
                         np.ones((M, 1)), (2.0 * sigma * np.log(b))[:, None]], 1)
    return psi, xi


def welfare_gradient(K, a, b, X, Y):
    """Gradient of the optimal welfare with respect to the factors (the
    back-propagation into the recommender that Sec. 5 names as future work).

    At the optimum of eq. 2-3 the envelope theorem gives dW*/dPhi_xy = mu_xy
    (the entropy term does not depend on Phi), and Phi = X Y^T with X = [U|Q],
    Y = [V|P] (eq. 8), so dW*/dX = mu Y and dW*/dY = mu^T X, with
    mu = K_xy a_x b_y (eq. 4). Returns (G_X, G_Y) in FP64."""
    mu = matching(K, a, b)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    return mu @ Y, mu.T @ X


def topk_matches(logmu, k: int):
    """Recommendation lists from a matching (Sec. 4.1 ranks partners by the
    stable matching mu): for every row, the columns of the k largest log mu,
    best first, ties to the lower column; rows shorter than k are padded with
    index -1 and -inf. Returns (idx int64 rows x k, values rows x k)."""
    logmu = np.asarray(logmu, dtype=np.float64)
    R, C = logmu.shape
    order = np.argsort(-logmu, axis=1, kind="stable")[:, :k]
    vals = np.take_along_axis(logmu, order, axis=1)
    idx = np.full((R, k), -1, dtype=np.int64)
    out = np.full((R, k), -np.inf)
    idx[:, :order.shape[1]] = order
    out[:, :order.shape[1]] = vals
    return idx, out


def pair_evals(N: int, M: int, sweeps: int) -> int:
    """Work unit used for throughput: every sweep consumes each K_xy twice."""
    return 2 * N * M * sweeps

