"""IPFP-free solutions of the matching program -- test infrastructure only.

These routines never run the IPFP update. They solve the paper's welfare
program directly, so that agreement with ``oracle.ipfp`` is evidence about
the iteration, not a restatement of it.

Primal (eq. 2-3): maximise
    W(mu) = sum_xy mu_xy phi_xy + beta E(mu),
    E(mu) = - sum_{x, y in Y0} mu_xy log(mu_xy / n_x)
            - sum_{y, x in X0} mu_xy log(mu_xy / m_y),
over mu_xy > 0 with the unmatched masses eliminated through the margin
constraints, mu_x0 = n_x - sum_y mu_xy and mu_0y = m_y - sum_x mu_xy.
Matched pairs appear in both entropy sums, the unmatched masses in one each.
Its gradient is phi_xy - beta log(mu_xy^2 / (mu_x0 mu_0y)); setting it to
zero gives eq. 4, so the optimum is the IPFP fixed point.

Dual (Lagrange multipliers alpha_x, gamma_y for the two constraint families):
    G(alpha, gamma) = sum n_x alpha_x + sum m_y gamma_y
                      + beta (sum mu_x0 + sum mu_0y + 2 sum mu_xy)
with mu_x0 = n_x exp(-1 - alpha_x/beta), mu_0y = m_y exp(-1 - gamma_y/beta),
mu_xy = sqrt(n_x m_y) exp((phi_xy - alpha_x - gamma_y)/(2 beta) - 1).
G is convex and min G = max W. IPFP is exact block minimisation of G over
alpha then gamma, so G never increases along the iteration.

Both problems are solved here by damped Newton with a backtracking line search
(interior for the primal), in FP64, for markets of up to a few dozen pairs.

Parity status: pinned against each other (strong duality, identical mu) and
against the closed forms of ``oracle.closed``.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class BruteResult:
    mu: np.ndarray      # N x M matched masses
    mu_x0: np.ndarray   # N unmatched row masses
    mu_0y: np.ndarray   # M unmatched column masses
    value: float        # optimal W (primal) or G (dual)
    iters: int
    grad_norm: float


def welfare(Phi, n, m, beta: float, mu) -> float:
    """W(mu) of eq. 2 with E of eq. 3 (unmatched masses from the margins)."""
    Phi, n, m, mu = (np.asarray(t, dtype=np.float64) for t in (Phi, n, m, mu))
    mx0 = n - mu.sum(1)
    m0y = m - mu.sum(0)
    e_rows = -np.sum(mu * np.log(mu / n[:, None])) - np.sum(mx0 * np.log(mx0 / n))
    e_cols = -np.sum(mu * np.log(mu / m[None, :])) - np.sum(m0y * np.log(m0y / m))
    return float(np.sum(mu * Phi) + beta * (e_rows + e_cols))


def primal_newton(Phi, n, m, beta: float, max_iter: int = 200,
                  gtol: float = 1e-14) -> BruteResult:
    """Maximise W over mu_xy > 0 by damped Newton.

    Gradient: g_xy = phi_xy - beta (2 log mu_xy - log mu_x0 - log mu_0y).
    Hessian:  H = -beta (2 diag(1/mu) + [x=x'] / mu_x0 + [y=y'] / mu_0y)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N, M = Phi.shape
    mu = 0.5 * np.minimum(n[:, None] / M, m[None, :] / N) * np.ones((N, M))
    same_row = np.kron(np.eye(N), np.ones((M, M)))
    same_col = np.kron(np.ones((N, N)), np.eye(M))
    it = 0
    gnorm = np.inf
    for it in range(1, max_iter + 1):
        mx0 = n - mu.sum(1)
        m0y = m - mu.sum(0)
        g = Phi - beta * (2 * np.log(mu) - np.log(mx0)[:, None] - np.log(m0y)[None, :])
        gnorm = float(np.max(np.abs(g)))
        if gnorm < gtol:
            break
        row_w = np.repeat(1.0 / mx0, M)           # per flattened (x, y)
        col_w = np.tile(1.0 / m0y, N)
        H = -beta * (np.diag(2.0 / mu.ravel()) + same_row * row_w[:, None]
                     + same_col * col_w[:, None])
        step = np.linalg.solve(H, -g.ravel()).reshape(N, M)
        w0 = welfare(Phi, n, m, beta, mu)
        slope = float(np.sum(g * step))
        t = 1.0
        while True:
            cand = mu + t * step
            ok = (np.all(cand > 0) and np.all(n - cand.sum(1) > 0)
                  and np.all(m - cand.sum(0) > 0))
            # the last term admits rounding noise once the ascent is below FP64 resolution
            if ok and welfare(Phi, n, m, beta, cand) >= w0 + 1e-4 * t * slope - 4e-16 * abs(w0):
                break
            t *= 0.5
            if t < 1e-30:
                break
        if t < 1e-30:
            break
        mu = cand
    mx0 = n - mu.sum(1)
    m0y = m - mu.sum(0)
    return BruteResult(mu, mx0, m0y, welfare(Phi, n, m, beta, mu), it, gnorm)


def _dual_masses(Phi, n, m, beta, al, ga):
    mx0 = n * np.exp(-1.0 - al / beta)
    m0y = m * np.exp(-1.0 - ga / beta)
    mu = np.sqrt(np.outer(n, m)) * np.exp(
        (Phi - al[:, None] - ga[None, :]) / (2.0 * beta) - 1.0)
    return mu, mx0, m0y


def dual_value(Phi, n, m, beta: float, al, ga) -> float:
    """G(alpha, gamma) as defined in the module docstring."""
    Phi, n, m, al, ga = (np.asarray(t, dtype=np.float64) for t in (Phi, n, m, al, ga))
    mu, mx0, m0y = _dual_masses(Phi, n, m, beta, al, ga)
    return float(n @ al + m @ ga + beta * (mx0.sum() + m0y.sum() + 2.0 * mu.sum()))


def multipliers_from_scalings(a, b, n, m, beta: float):
    """alpha, gamma that give mu_x0 = a^2 and mu_0y = b^2 (inverting the dual
    masses): alpha_x = -beta (1 + log(a_x^2 / n_x)), likewise gamma_y."""
    a, b, n, m = (np.asarray(t, dtype=np.float64) for t in (a, b, n, m))
    return -beta * (1.0 + np.log(a * a / n)), -beta * (1.0 + np.log(b * b / m))


def dual_newton(Phi, n, m, beta: float, max_iter: int = 200,
                gtol: float = 1e-14) -> BruteResult:
    """Minimise G by damped Newton over the N + M multipliers.

    dG/dalpha_x = n_x - mu_x0 - sum_y mu_xy, dG/dgamma_y = m_y - mu_0y - sum_x mu_xy;
    d2G/dalpha_x^2 = mu_x0/beta + sum_y mu_xy/(2 beta),
    d2G/dalpha_x dgamma_y = mu_xy/(2 beta), and symmetrically for gamma."""
    Phi = np.asarray(Phi, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N, M = Phi.shape
    # start where every exponent (phi - alpha - gamma) / 2 beta is <= 0
    c = max(0.0, float(Phi.max()))
    al = np.full(N, c / 2)
    ga = np.full(M, c / 2)
    it = 0
    gnorm = np.inf
    for it in range(1, max_iter + 1):
        mu, mx0, m0y = _dual_masses(Phi, n, m, beta, al, ga)
        g = np.concatenate([n - mx0 - mu.sum(1), m - m0y - mu.sum(0)])
        gnorm = float(np.max(np.abs(g)))
        if gnorm < gtol:
            break
        H = np.zeros((N + M, N + M))
        H[:N, :N] = np.diag(mx0 / beta + mu.sum(1) / (2 * beta))
        H[N:, N:] = np.diag(m0y / beta + mu.sum(0) / (2 * beta))
        H[:N, N:] = mu / (2 * beta)
        H[N:, :N] = mu.T / (2 * beta)
        step = np.linalg.solve(H, -g)
        g0 = dual_value(Phi, n, m, beta, al, ga)
        slope = float(g @ step)
        t = 1.0
        while t > 1e-30:
            if dual_value(Phi, n, m, beta, al + t * step[:N], ga + t * step[N:]) \
                    <= g0 + 1e-4 * t * slope + 4e-16 * abs(g0):
                break
            t *= 0.5
        al = al + t * step[:N]
        ga = ga + t * step[N:]
    mu, mx0, m0y = _dual_masses(Phi, n, m, beta, al, ga)
    return BruteResult(mu, mx0, m0y, dual_value(Phi, n, m, beta, al, ga), it, gnorm)
