"""Closed forms and exact replays of the IPFP iteration -- test infrastructure.

* Uniform market (constant surplus c, equal margins n on every row and m on
  every column): by symmetry mu_xy = mu for all pairs, and eq. 4 with the
  margin constraints of eq. 2 gives mu = k sqrt((n - M mu)(m - N mu)),
  k = exp(c / 2 beta). Squaring, mu solves
      (1 - k^2 N M) mu^2 + k^2 (n N + m M) mu - k^2 n m = 0
  on (0, min(n/M, m/N)); then u^2 = mu_x0 = n - M mu and v^2 = m - N mu.
  The 1x1 market is N = M = 1; with k = 1 it gives mu = n m / (n + m).
* Separable surplus phi_xy = alpha_x + gamma_y: the kernel factorises as
  K = k l^T (k_x = exp(alpha_x / 2 beta), l_y = exp(gamma_y / 2 beta)), so the
  row sums of eq. 6 are s_x = k_x (l . v) / 2 and the column sums
  s_y = l_y (k . u) / 2. ``separable_replay`` runs the exact Gauss-Seidel
  sequence of eq. 6 in O(N + M) per sweep, which makes sweep-by-sweep parity
  possible at sizes where no N x M matrix can be formed.

Parity status: the closed forms are pinned by the brute-force solvers of
``oracle.brute``; ``separable_replay`` against ``oracle.ipfp.ipfp_batch``
on small separable markets.
"""
from __future__ import annotations

import math

import numpy as np

from .ipfp import IPFPResult, root


def _quad_root_in(a2: float, a1: float, a0: float, hi: float) -> float:
    """The root of a2 x^2 + a1 x + a0 = 0 lying in (0, hi), computed without
    cancellation (a0 < 0 < a1 here)."""
    if a2 == 0.0:
        return -a0 / a1
    disc = math.sqrt(a1 * a1 - 4.0 * a2 * a0)
    # roots: q = -(a1 + disc)/2 ; x1 = q / a2, x2 = a0 / q
    q = -0.5 * (a1 + disc)
    cands = [q / a2, a0 / q]
    good = [x for x in cands if 0.0 < x < hi]
    if not good:
        raise ValueError("no root in range")
    return min(good)


def uniform_market(c: float, n: float, m: float, N: int, M: int, beta: float):
    """(mu, u, v) of the uniform market at the optimum."""
    k2 = math.exp(c / beta)  # k^2 with k = exp(c / 2 beta)
    mu = _quad_root_in(1.0 - k2 * N * M, k2 * (n * N + m * M), -k2 * n * m,
                       min(n / M, m / N))
    return mu, math.sqrt(n - M * mu), math.sqrt(m - N * mu)


def separable_replay(alpha, gamma, n, m, beta: float, tol: float = 0.0,
                     max_sweeps: int = 100, check_every: int = 1,
                     b0=None) -> IPFPResult:
    """Exact IPFP iterate sequence (eq. 6) for phi_xy = alpha_x + gamma_y, with
    the same sweep order, residual and stopping rule as ``ipfp_batch``."""
    alpha = np.asarray(alpha, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    k = np.exp(alpha / (2.0 * beta))
    l = np.exp(gamma / (2.0 * beta))
    v = np.ones(len(gamma)) if b0 is None else np.array(b0, dtype=np.float64)
    u = np.ones(len(alpha))
    hist = []
    i = 0
    for i in range(1, max_sweeps + 1):
        u = root(n, 0.5 * k * float(l @ v))
        v = root(m, 0.5 * l * float(k @ u))
        if i % check_every == 0 or i == max_sweeps:
            r = float(np.max(np.abs(u * u + u * k * float(l @ v) - n) / n))
            hist.append(r)
            if r < tol:
                break
    return IPFPResult(u, v, hist, i, hist[-1] if hist else float("nan"))
