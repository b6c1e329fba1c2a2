"""Writes equilibria.json: high-precision equilibria of small TU matching
markets, computed here with mpmath alone (no code from ``oracle/``), so that
the oracle can be checked against values it did not produce.

    python tests/golden/make_golden.py

For each market the unknowns are the scalings a_x = sqrt(mu_x0) and
b_y = sqrt(mu_0y). Substituting eq. 4 (mu_xy = exp(phi_xy / 2 beta) a_x b_y)
into the margin constraints of eq. 2 gives the square system of eq. 5:

    a_x^2 + a_x sum_y K_xy b_y = n_x,    b_y^2 + b_y sum_x K_xy a_x = m_y,

with K_xy = exp(phi_xy / 2 beta). It is solved by Newton's method at 60
significant digits. The starting point comes from a few alternating exact
solves of each equation for its own unknown (a positive root of a quadratic),
then Newton runs until the update is below 10^-55. The welfare W of eq. 2 at
the solution, sum mu phi + beta E(mu) with the entropy E of eq. 3, is stored
as well. Every value is written with 40 significant digits.
"""
import json
import os

import mpmath as mp

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))

# (name, phi rows, n, m, beta): decimal strings, so the inputs are exact
MARKETS = [
    ("one_by_one", [["0.7"]], ["1"], ["2"], "1"),
    ("two_by_three", [["0.5", "-1.25", "2"], ["1.5", "0.25", "-0.75"]],
     ["1", "2"], ["0.5", "1.5", "1"], "0.8"),
    ("four_by_three", [["0.125", "0.875", "-0.5"], ["1", "-1", "0.25"],
                       ["-0.375", "0.625", "1.5"], ["2", "0", "-2"]],
     ["1", "1", "3", "0.25"], ["2", "0.5", "1"], "0.5"),
    ("large_surplus", [["30", "12", "-4"], ["25", "28", "3"]],
     ["1", "4"], ["2", "1", "3"], "0.75"),
]


def solve(phi, n, m, beta):
    N, M = len(n), len(m)
    K = [[mp.exp(phi[x][y] / (2 * beta)) for y in range(M)] for x in range(N)]

    def pos_root(marg, s):       # t^2 + 2 s t = marg, t > 0
        return marg / (s + mp.sqrt(s * s + marg))

    a = [mp.mpf(1)] * N
    b = [mp.mpf(1)] * M
    for _ in range(200):
        a = [pos_root(n[x], sum(K[x][y] * b[y] for y in range(M)) / 2) for x in range(N)]
        b = [pos_root(m[y], sum(K[x][y] * a[x] for x in range(N)) / 2) for y in range(M)]

    def F(z):
        aa, bb = z[:N], z[N:]
        out = [aa[x] ** 2 + aa[x] * sum(K[x][y] * bb[y] for y in range(M)) - n[x]
               for x in range(N)]
        out += [bb[y] ** 2 + bb[y] * sum(K[x][y] * aa[x] for x in range(N)) - m[y]
                for y in range(M)]
        return out

    def J(z):
        aa, bb = z[:N], z[N:]
        Jm = mp.matrix(N + M, N + M)
        for x in range(N):
            Jm[x, x] = 2 * aa[x] + sum(K[x][y] * bb[y] for y in range(M))
            for y in range(M):
                Jm[x, N + y] = aa[x] * K[x][y]
        for y in range(M):
            Jm[N + y, N + y] = 2 * bb[y] + sum(K[x][y] * aa[x] for x in range(N))
            for x in range(N):
                Jm[N + y, x] = bb[y] * K[x][y]
        return Jm

    z = mp.matrix(a + b)
    for _ in range(100):
        step = mp.lu_solve(J(z), mp.matrix(F(z)))
        z = z - step
        if mp.norm(step) < mp.mpf(10) ** -55:
            break
    else:
        raise RuntimeError("Newton did not converge")
    a = [z[i] for i in range(N)]
    b = [z[N + i] for i in range(M)]
    mu = [[K[x][y] * a[x] * b[y] for y in range(M)] for x in range(N)]
    ent = mp.mpf(0)
    for x in range(N):
        for y in range(M):
            ent -= mu[x][y] * mp.log(mu[x][y] / n[x]) + mu[x][y] * mp.log(mu[x][y] / m[y])
        ent -= a[x] ** 2 * mp.log(a[x] ** 2 / n[x])
    for y in range(M):
        ent -= b[y] ** 2 * mp.log(b[y] ** 2 / m[y])
    W = sum(mu[x][y] * phi[x][y] for x in range(N) for y in range(M)) + beta * ent
    resid = max(abs(v) for v in F(z))
    return a, b, mu, W, resid


def s40(v):
    return mp.nstr(v, 40, min_fixed=-mp.inf, max_fixed=mp.inf)


def main(path=None):
    out = {"source": "eq. 2-5 (Sec. 3.1-3.2), solved by Newton's method in mpmath at 60 digits "
                     "by tests/golden/make_golden.py",
           "markets": []}
    for name, phi_s, n_s, m_s, beta_s in MARKETS:
        phi = [[mp.mpf(v) for v in row] for row in phi_s]
        n = [mp.mpf(v) for v in n_s]
        m = [mp.mpf(v) for v in m_s]
        beta = mp.mpf(beta_s)
        a, b, mu, W, resid = solve(phi, n, m, beta)
        assert resid < mp.mpf(10) ** -50, (name, resid)
        out["markets"].append({
            "name": name, "phi": phi_s, "n": n_s, "m": m_s, "beta": beta_s,
            "a": [s40(v) for v in a], "b": [s40(v) for v in b],
            "mu": [[s40(v) for v in row] for row in mu], "welfare": s40(W)})
    with open(path or os.path.join(HERE, "equilibria.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
