"""Seeded synthetic inputs for the IPFP matching market (random draws only).

This module holds the input recipes shared by the tests, the benchmark and the
smoke check. It draws factor matrices and margins and nothing else: no part of
the matching computation lives here, so both the CPU oracle and the HIP path
can be fed from it without sharing any of the method's arithmetic.

Workload shapes follow the configurations the implementation is measured on:

* ``C1``  500 x 400 markets, d = 16 per side, factors N(0, 1/16), sigma = 1,
  unit margins (plain path, FP64).
* ``C2``  20,000 x 20,000, d = 32, N(0, 1/32), sigma = 0.5, n_x = 1,
  m_y uniform on {1..5} (plain FP32 vs fused BF16 on the same market).
* ``C3``  1,000,000 x 1,000,000, d = 64, N(0, 1/64), sigma = 1, n_x = 1,
  m_y uniform on {1..10} (fused BF16 mini-batch path).
* ``C4``  serving mix: market sizes log-uniform in [1e3, 2e5] per side,
  d = 32, sigma in {0.5, 1}, unit margins, Poisson(200/s) arrivals.
* ``C5``  2,000,000 x 200,000, d = 128, N(0, 1/128), sigma in {0.1, 1},
  n_x = 1, m_y = min(Zipf(1.5), 1000) (precision stress).

The paper's own timing study (Sec. 4.2) draws factors from U[0, 1/sqrt(D)]
with D = 50 and equal capacities; ``paper_uniform`` reproduces that recipe.

All draws come from ``numpy.random.Generator(PCG64(seed))`` with
``seed = 19214 + 1000 * c`` for configuration ``c`` unless a seed is given.
The draw order is U, Q, V, P, then the column margins m (row margins are
constant in every configuration). Factors are drawn in float32: those float32
values ARE the factor values of the market (both sides read the same bytes).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 19214


@dataclasses.dataclass
class Market:
    """One synthetic market: factors (float32, row-major) and margins (float64)."""

    U: np.ndarray  # N x d
    Q: np.ndarray  # N x d
    V: np.ndarray  # M x d
    P: np.ndarray  # M x d
    n: np.ndarray  # N, row (candidate) margins
    m: np.ndarray  # M, column (employer) margins
    sigma: float
    name: str = ""

    @property
    def N(self) -> int:
        return self.U.shape[0]

    @property
    def M(self) -> int:
        return self.V.shape[0]

    @property
    def d(self) -> int:
        return self.U.shape[1]


def config_seed(c: int) -> int:
    return BASE_SEED + 1000 * c


def _normal(rng: np.random.Generator, rows: int, d: int, var: float) -> np.ndarray:
    out = rng.standard_normal((rows, d), dtype=np.float32)
    out *= np.float32(math.sqrt(var))
    return out


def _col_margins(rng: np.random.Generator, M: int, kind: str) -> np.ndarray:
    if kind == "unit":
        return np.ones(M, dtype=np.float64)
    if kind.startswith("uint"):  # "uint1-5": uniform integers in [lo, hi]
        lo, hi = (int(t) for t in kind[4:].split("-"))
        return rng.integers(lo, hi + 1, size=M).astype(np.float64)
    if kind.startswith("zipf"):  # "zipf1.5cap1000"
        a, cap = kind[4:].split("cap")
        return np.minimum(rng.zipf(float(a), size=M), int(cap)).astype(np.float64)
    raise ValueError(kind)


def factor_market(N: int, M: int, d: int, var: float, sigma: float,
                  col_margin: str = "unit", seed: int = BASE_SEED,
                  name: str = "") -> Market:
    """Gaussian factor market: U,Q ~ N(0,var)^{N x d}, V,P ~ N(0,var)^{M x d}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = _normal(rng, N, d, var)
    Q = _normal(rng, N, d, var)
    V = _normal(rng, M, d, var)
    P = _normal(rng, M, d, var)
    m = _col_margins(rng, M, col_margin)
    n = np.ones(N, dtype=np.float64)
    return Market(U, Q, V, P, n, m, float(sigma), name)


# --- the five configurations (full size) and reduced-size variants that keep
# --- each configuration's distribution.

CONFIGS = {
    1: dict(N=500, M=400, d=16, var=1 / 16, sigma=1.0, col_margin="unit",
            max_sweeps=2000, tol=1e-10),
    2: dict(N=20000, M=20000, d=32, var=1 / 32, sigma=0.5, col_margin="uint1-5",
            max_sweeps=500, tol=1e-6),
    3: dict(N=1_000_000, M=1_000_000, d=64, var=1 / 64, sigma=1.0,
            col_margin="uint1-10", max_sweeps=100, tol=0.0, row_batch=65536),
    5: dict(N=2_000_000, M=200_000, d=128, var=1 / 128, sigma=1.0,
            col_margin="zipf1.5cap1000", max_sweeps=200, tol=0.0),
}


def config_market(c: int, N: int | None = None, M: int | None = None,
                  sigma: float | None = None, seed: int | None = None) -> Market:
    """Market of configuration ``c``; N, M (and sigma) may be overridden to get
    a reduced-size market with the same factor and margin distributions."""
    cfg = CONFIGS[c]
    return factor_market(
        N if N is not None else cfg["N"], M if M is not None else cfg["M"],
        cfg["d"], cfg["var"], cfg["sigma"] if sigma is None else sigma,
        cfg["col_margin"], config_seed(c) if seed is None else seed,
        name=f"C{c}")


def paper_uniform(N: int, M: int, D: int = 50, seed: int = BASE_SEED) -> Market:
    """The timing study's recipe: factors U[0, 1/sqrt(D)], n_x = 1 (C = N),
    m_y = N / M, beta = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hi = np.float32(1.0 / math.sqrt(D))
    U, Q = (rng.random((N, D), dtype=np.float32) * hi for _ in range(2))
    V, P = (rng.random((M, D), dtype=np.float32) * hi for _ in range(2))
    return Market(U, Q, V, P, np.ones(N), np.full(M, N / M), 1.0, "paper")


def random_phi(N: int, M: int, scale: float, seed: int) -> np.ndarray:
    """A dense surplus matrix with i.i.d. N(0, scale^2) entries (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((N, M)) * scale


def random_margins(K: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=K)


# --- serving mix ---------------------------------------------------------

@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    N: int
    M: int
    d: int
    sigma: float
    seed: int


def serving_requests(count: int = 512, rate_hz: float = 200.0,
                     lo: float = 1e3, hi: float = 2e5, d: int = 32,
                     seed: int = BASE_SEED + 4000) -> list[Request]:
    """Arrival times and per-request market shapes of the serving mix.

    Arrival gaps are Exp(1/rate) from the parent stream; each request's sizes,
    sigma and factor seed come from its own spawned stream."""
    ss = np.random.SeedSequence(seed)
    parent = np.random.Generator(np.random.PCG64(ss))
    gaps = parent.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i, child in enumerate(ss.spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        N = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        M = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        sigma = float(rng.choice([0.5, 1.0]))
        fseed = int(rng.integers(0, 2**31 - 1))
        out.append(Request(i, float(t[i]), N, M, d, sigma, fseed))
    return out


def request_market(r: Request) -> Market:
    return factor_market(r.N, r.M, r.d, 1.0 / r.d, r.sigma, "unit", r.seed,
                         name=f"req{r.index}")


def device_request_factors(torch, r: Request, device="cuda"):
    """(U, Q, V, P, n, m) of a serving request drawn directly on the device:
    the distribution of ``request_market`` (i.i.d. N(0, 1/d) float32 factors,
    unit margins) from torch's device generator seeded with the request's
    seed, so a large request mix never passes through host memory. The
    numbers differ from ``request_market``'s (another generator)."""
    g = torch.Generator(device=device)
    g.manual_seed(r.seed)
    sd = math.sqrt(1.0 / r.d)
    U, Q = (torch.randn(r.N, r.d, generator=g, device=device) * sd for _ in range(2))
    V, P = (torch.randn(r.M, r.d, generator=g, device=device) * sd for _ in range(2))
    n = torch.ones(r.N, dtype=torch.float64, device=device)
    m = torch.ones(r.M, dtype=torch.float64, device=device)
    return U, Q, V, P, n, m
