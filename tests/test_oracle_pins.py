"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test ties ``oracle.ipfp`` to something fixed by the paper's model or by
mathematics: an IPFP-free solve of the welfare program (eq. 2-3) and of its
dual, closed forms, invariants of eq. 4-6, and brute-force searches. The
mutation tests at the end plant plausible mistakes in the oracle's arithmetic
(on the CPU) and check that a pin fails.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import brute, closed, ipfp, quant
import workloads


def small_market(N, M, seed, beta=1.0, scale=1.0):
    rng = np.random.default_rng(seed)
    Phi = rng.normal(0.0, scale, size=(N, M))
    n = rng.uniform(0.5, 2.0, size=N)
    m = rng.uniform(0.5, 2.0, size=M)
    return Phi, n, m, beta


SHAPES = [(3, 3), (3, 5), (4, 4), (5, 3), (6, 6), (6, 4)]


def converged(Phi, n, m, beta):
    K = ipfp.kernel_matrix(Phi, beta)
    return K, ipfp.ipfp_batch(K, n, m, tol=1e-15, max_sweeps=20000)


# --- independent solves of the welfare program ------------------------------

@pytest.mark.parametrize("N,M", SHAPES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_primal_and_dual_newton_agree(N, M, beta):
    Phi, n, m, _ = small_market(N, M, seed=N * 10 + M, beta=beta)
    p = brute.primal_newton(Phi, n, m, beta)
    d = brute.dual_newton(Phi, n, m, beta)
    assert p.grad_norm < 1e-10 and d.grad_norm < 1e-10
    assert abs(p.value - d.value) <= 1e-12 * max(1.0, abs(p.value))   # strong duality
    np.testing.assert_allclose(p.mu, d.mu, rtol=1e-10, atol=0)
    np.testing.assert_allclose(p.mu_x0, d.mu_x0, rtol=1e-10)


@pytest.mark.parametrize("N,M", SHAPES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_ipfp_fixed_point_is_welfare_optimum(N, M, beta):
    Phi, n, m, _ = small_market(N, M, seed=100 + N * 10 + M, beta=beta)
    K, r = converged(Phi, n, m, beta)
    mu = ipfp.matching(K, r.a, r.b)
    p = brute.primal_newton(Phi, n, m, beta)
    np.testing.assert_allclose(mu, p.mu, rtol=1e-10)
    np.testing.assert_allclose(r.a ** 2, p.mu_x0, rtol=1e-10)   # mu_x0 = u^2
    np.testing.assert_allclose(r.b ** 2, p.mu_0y, rtol=1e-10)   # mu_0y = v^2
    w = brute.welfare(Phi, n, m, beta, mu)
    assert abs(w - p.value) <= 1e-11 * max(1.0, abs(p.value))


@pytest.mark.parametrize("seed", range(4))
def test_ipfp_dual_never_increases(seed):
    """IPFP is exact block minimisation of the dual: every half-step lowers G."""
    Phi, n, m, beta = small_market(5, 4, seed=200 + seed, beta=0.7, scale=2.0)
    K = ipfp.kernel_matrix(Phi, beta)
    v = np.ones(4)
    u = np.ones(5)
    prev = np.inf
    for _ in range(60):
        u = ipfp.root(n, 0.5 * K @ v)
        g1 = brute.dual_value(Phi, n, m, beta, *brute.multipliers_from_scalings(u, v, n, m, beta))
        v = ipfp.root(m, 0.5 * K.T @ u)
        g2 = brute.dual_value(Phi, n, m, beta, *brute.multipliers_from_scalings(u, v, n, m, beta))
        assert g1 <= prev + 1e-12 * abs(prev if np.isfinite(prev) else 1.0)
        assert g2 <= g1 + 1e-12 * abs(g1)
        prev = g2
    d = brute.dual_newton(Phi, n, m, beta)
    assert abs(prev - d.value) < 1e-9 * abs(d.value)


# --- closed forms -------------------------------------------------------------

@pytest.mark.parametrize("N,M,c,n,m,beta", [
    (1, 1, 0.0, 1.0, 1.0, 1.0), (1, 1, 0.3, 2.0, 0.5, 0.7), (3, 4, -0.5, 1.0, 2.0, 1.0),
    (5, 2, 1.2, 0.3, 3.0, 0.5)])
def test_uniform_closed_form_matches_brute_force(N, M, c, n, m, beta):
    mu, u, v = closed.uniform_market(c, n, m, N, M, beta)
    Phi = np.full((N, M), c)
    p = brute.primal_newton(Phi, np.full(N, n), np.full(M, m), beta)
    np.testing.assert_allclose(p.mu, mu, rtol=1e-11)
    np.testing.assert_allclose(p.mu_x0, u * u, rtol=1e-11)


def test_one_by_one_unit_kernel():
    for n, m in [(1.0, 1.0), (2.0, 3.0), (0.25, 7.0)]:
        mu, _, _ = closed.uniform_market(0.0, n, m, 1, 1, 1.0)
        assert mu == pytest.approx(n * m / (n + m), rel=1e-15)


@pytest.mark.parametrize("N,M", [(1, 1), (7, 13), (50, 20)])
def test_ipfp_reaches_uniform_closed_form(N, M):
    c, n, m, beta = 0.4, 1.0, 2.0, 1.0
    mu, u, v = closed.uniform_market(c, n, m, N, M, beta)
    K, r = converged(np.full((N, M), c), np.full(N, n), np.full(M, m), beta)
    # v^2 = m - N mu cancels when most column mass is matched (50x20: ~400x
    # amplification), so the closed form itself is good to ~1e-13 there
    np.testing.assert_allclose(r.a, u, rtol=1e-12)
    np.testing.assert_allclose(r.b, v, rtol=1e-12)
    np.testing.assert_allclose(ipfp.matching(K, r.a, r.b), mu, rtol=1e-13)


def test_separable_replay_equals_batch():
    rng = np.random.default_rng(5)
    al, ga = rng.normal(size=9), rng.normal(size=7)
    n, m = rng.uniform(0.5, 2, 9), rng.uniform(0.5, 2, 7)
    K = ipfp.kernel_matrix(al[:, None] + ga[None, :], 0.8)
    a = ipfp.ipfp_batch(K, n, m, tol=0, max_sweeps=37, check_every=5)
    b = closed.separable_replay(al, ga, n, m, 0.8, tol=0, max_sweeps=37, check_every=5)
    np.testing.assert_allclose(a.a, b.a, rtol=1e-13)
    np.testing.assert_allclose(a.b, b.b, rtol=1e-13)
    np.testing.assert_allclose(a.res_hist, b.res_hist, rtol=1e-6, atol=1e-15)
    assert a.sweeps == b.sweeps == 37


# --- invariants ---------------------------------------------------------------

def test_column_margins_hold_after_every_sweep():
    Phi, n, m, beta = small_market(30, 20, seed=7, scale=1.5)
    K = ipfp.kernel_matrix(Phi, beta)
    for sweeps in (1, 2, 5, 17):
        r = ipfp.ipfp_batch(K, n, m, max_sweeps=sweeps)
        assert ipfp.col_residual(K, r.a, r.b, m) < 1e-14
        mu = ipfp.matching(K, r.a, r.b)
        assert np.all(mu >= 0)
        assert np.all(r.a ** 2 <= n) and np.all(r.b ** 2 <= m)


def test_residual_history_decreases_to_zero():
    m_ = workloads.config_market(1, N=60, M=40)
    Phi = ipfp.surplus_from_factors(m_.U, m_.Q, m_.V, m_.P)
    K = ipfp.kernel_matrix(Phi, m_.sigma)
    r = ipfp.ipfp_batch(K, m_.n, m_.m, tol=1e-12, max_sweeps=2000)
    assert r.final_res < 1e-12 and r.sweeps < 2000
    assert r.res_hist[-1] < r.res_hist[0]


def test_homogeneity_in_margins():
    Phi, n, m, beta = small_market(8, 6, seed=9)
    K = ipfp.kernel_matrix(Phi, beta)
    c = 3.7
    r1 = ipfp.ipfp_batch(K, n, m, max_sweeps=25)
    r2 = ipfp.ipfp_batch(K, c * n, c * m, max_sweeps=25, b0=np.full(6, math.sqrt(c)))
    np.testing.assert_allclose(r2.a, math.sqrt(c) * r1.a, rtol=1e-13)
    np.testing.assert_allclose(r2.b, math.sqrt(c) * r1.b, rtol=1e-13)


def test_transpose_symmetry_at_convergence():
    Phi, n, m, beta = small_market(6, 9, seed=11)
    _, r = converged(Phi, n, m, beta)
    _, t = converged(Phi.T.copy(), m, n, beta)
    np.testing.assert_allclose(t.a, r.b, rtol=1e-12)
    np.testing.assert_allclose(t.b, r.a, rtol=1e-12)


def test_warm_start_resume_is_exact():
    Phi, n, m, beta = small_market(12, 10, seed=12)
    K = ipfp.kernel_matrix(Phi, beta)
    full = ipfp.ipfp_batch(K, n, m, max_sweeps=100)
    half = ipfp.ipfp_batch(K, n, m, max_sweeps=50)
    rest = ipfp.ipfp_batch(K, n, m, max_sweeps=50, b0=half.b)
    assert np.array_equal(full.a, rest.a) and np.array_equal(full.b, rest.b)


@pytest.mark.parametrize("bx,by", [(1, 1), (3, 7), (64, 5), (1000, 1000)])
def test_minibatch_equals_batch(bx, by):
    """Sec. 3.3: the mini-batch form makes no approximation."""
    mk = workloads.config_market(2, N=70, M=45)
    Phi = ipfp.surplus_from_factors(mk.U, mk.Q, mk.V, mk.P)
    K = ipfp.kernel_matrix(Phi, mk.sigma)
    a = ipfp.ipfp_batch(K, mk.n, mk.m, max_sweeps=12, check_every=4)
    b = ipfp.ipfp_minibatch(mk.U, mk.Q, mk.V, mk.P, mk.n, mk.m, mk.sigma, bx, by,
                            max_sweeps=12, check_every=4)
    np.testing.assert_allclose(b.a, a.a, rtol=1e-12)
    np.testing.assert_allclose(b.b, a.b, rtol=1e-12)
    np.testing.assert_allclose(b.res_hist, a.res_hist, rtol=1e-8, atol=1e-15)


def test_logdomain_equals_batch():
    Phi, n, m, beta = small_market(10, 8, seed=13, scale=3.0)
    K = ipfp.kernel_matrix(Phi, beta)
    a = ipfp.ipfp_batch(K, n, m, max_sweeps=30)
    b = ipfp.ipfp_logdomain(Phi, n, m, beta, max_sweeps=30)
    np.testing.assert_allclose(b.a, a.a, rtol=1e-12)
    np.testing.assert_allclose(b.b, a.b, rtol=1e-12)


def test_logdomain_on_large_surplus_matches_dual_newton():
    """A constant shift of Phi scales K by exp(c/2beta); at Phi + 30 (beta 0.5)
    nearly all of the smaller side is matched and the log-domain sums must still
    reach the optimum."""
    Phi, n, m, beta = small_market(4, 3, seed=14, beta=0.5)
    Phi = Phi + 30.0
    r = ipfp.ipfp_logdomain(Phi, n, m, beta, tol=1e-15, max_sweeps=5000)
    d = brute.dual_newton(Phi, n, m, beta)
    np.testing.assert_allclose(r.a ** 2, d.mu_x0, rtol=1e-7)
    np.testing.assert_allclose(r.b ** 2, d.mu_0y, rtol=1e-7)
    with pytest.raises(OverflowError):
        ipfp.kernel_matrix(Phi + 1200.0, beta)


def test_stable_factors_reproduce_log_mu():
    mk = workloads.config_market(1, N=9, M=7)
    Phi = ipfp.surplus_from_factors(mk.U, mk.Q, mk.V, mk.P)
    K = ipfp.kernel_matrix(Phi, mk.sigma)
    r = ipfp.ipfp_batch(K, mk.n, mk.m, max_sweeps=40)
    psi, xi = ipfp.stable_factors(mk.U, mk.Q, mk.V, mk.P, r.a, r.b, mk.sigma)
    assert psi.shape == (9, 2 * mk.d + 2) and xi.shape == (7, 2 * mk.d + 2)
    np.testing.assert_allclose(psi @ xi.T / (2 * mk.sigma),
                               np.log(ipfp.matching(K, r.a, r.b)), rtol=1e-12, atol=1e-12)


# --- the quadratic root ------------------------------------------------------

def test_root_is_accurate_where_literal_form_cancels():
    mpmath.mp.dps = 700   # enough digits that the literal form does not cancel up to s = 1e300
    rng = np.random.default_rng(15)
    s = np.concatenate([10.0 ** rng.uniform(-8, 200, 300), [0.0, 1e-300, 1e151, 1e300]])
    marg = rng.uniform(0.1, 10.0, len(s))
    w = ipfp.root(marg, s)
    for wi, si, ni in zip(w, s, marg):
        exact = mpmath.sqrt(mpmath.mpf(ni) + mpmath.mpf(si) ** 2) - mpmath.mpf(si)
        assert abs(wi - float(exact)) <= 4e-16 * float(exact)


# --- quantisers vs brute-force nearest-value search ---------------------------

def test_bf16_round_is_nearest_even():
    rng = np.random.default_rng(16)
    x = np.concatenate([rng.normal(0, 1, 4000).astype(np.float32),
                        (rng.normal(0, 1, 1000) * 1e-3).astype(np.float32)])
    # include exact ties: bf16 value plus half an ulp
    base = quant.bf16_round(rng.normal(0, 1, 200).astype(np.float32))
    ties = (base.view(np.uint32) + np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties])
    allv = (np.arange(65536, dtype=np.uint32) << np.uint32(16)).view(np.float32)
    finite = allv[np.isfinite(allv)]
    got = quant.bf16_round(x)
    for xi, gi in zip(x.astype(np.float64), got.astype(np.float64)):
        d = np.abs(finite.astype(np.float64) - xi)
        best = finite[d == d.min()]
        if len(best) == 1:
            assert gi == best[0]
        else:   # tie: the code with an even last bit
            codes = best.view(np.uint32) >> 16
            assert gi == best[(codes & 1) == 0][0]


def test_e4m3_round_is_nearest_even_saturating():
    table = quant.e4m3_value_table()
    finite = table[np.isfinite(table)]
    rng = np.random.default_rng(17)
    x = np.concatenate([rng.normal(0, 100, 3000), rng.normal(0, 0.01, 1000),
                        [500.0, -1e6, 448.0, 464.0, 0.0]])
    # exact midpoints between neighbours are ties
    pos = np.unique(finite[finite >= 0])
    x = np.concatenate([x, (pos[1:] + pos[:-1]) / 2])
    got = quant.e4m3_round(x)
    codes_of = {float(v): c for c, v in enumerate(table) if np.isfinite(v)}
    for xi, gi in zip(x, got):
        xc = min(max(xi, -448.0), 448.0)
        d = np.abs(finite - xc)
        best = np.unique(finite[d == d.min()])
        if len(best) == 1:
            assert gi == best[0]
        else:
            even = [b for b in best if codes_of[float(b)] % 2 == 0]
            assert gi == even[0]
    assert np.array_equal(quant.e4m3_value_table()[quant.e4m3_codes(got)], got)


def test_pow2_row_scale_is_smallest_fitting_power():
    rng = np.random.default_rng(18)
    rows = rng.normal(0, 1, (200, 16)) * 10.0 ** rng.uniform(-5, 5, (200, 1))
    rows[0] = 0.0
    rows[1, :] = 448.0
    s = quant.pow2_row_scale(rows)
    amax = np.abs(rows).max(1)
    assert s[0] == 1.0 and s[1] == 1.0
    nz = amax > 0
    assert np.all(amax[nz] <= 448.0 * s[nz])
    assert np.all(amax[nz] > 448.0 * s[nz] / 2)
    assert np.all(np.log2(s) == np.round(np.log2(s)))


# --- planted mistakes must fail a pin ------------------------------------------

def _pin_fails(solve):
    """True when ``solve`` (Phi, n, m, beta) -> (mu, mu_x0) disagrees with the
    brute-force optimum on a 4x5 market."""
    Phi, n, m, beta = small_market(4, 5, seed=19, beta=0.8)
    p = brute.primal_newton(Phi, n, m, beta)
    mu, mx0 = solve(Phi, n, m, beta)
    return not (np.allclose(mu, p.mu, rtol=1e-8) and np.allclose(mx0, p.mu_x0, rtol=1e-8))


def _ipfp_with(K_fn, root_fn, swap_margins=False):
    def solve(Phi, n, m, beta):
        K = K_fn(Phi, beta)
        v = np.ones(K.shape[1])
        rows, cols = (m[: K.shape[0]], n[: K.shape[1]]) if swap_margins else (n, m)
        for _ in range(5000):
            u = root_fn(rows, 0.5 * K @ v)
            v = root_fn(cols, 0.5 * K.T @ u)
        return K * np.outer(u, v), u * u
    return solve


def test_mutations_are_caught():
    good = _ipfp_with(ipfp.kernel_matrix, ipfp.root)
    assert not _pin_fails(good)
    # kernel scale exp(Phi/beta) instead of exp(Phi/2beta)
    assert _pin_fails(_ipfp_with(lambda P, b: np.exp(P / b), ipfp.root))
    # dropped factor 1/2 in s
    assert _pin_fails(_ipfp_with(ipfp.kernel_matrix, lambda mg, s: ipfp.root(mg, 2 * s)))
    # wrong sign in the root
    assert _pin_fails(_ipfp_with(ipfp.kernel_matrix,
                                 lambda mg, s: np.sqrt(mg + s * s) + s))
    # margin dropped from the root (u = sqrt(s^2 + 1) - s)
    assert _pin_fails(_ipfp_with(ipfp.kernel_matrix,
                                 lambda mg, s: ipfp.root(np.ones_like(mg), s)))
    # n and m exchanged (the letter swap of Alg. 1), on a square market
    def swapped(Phi, n, m, beta):
        return _ipfp_with(ipfp.kernel_matrix, ipfp.root, swap_margins=True)(
            Phi[:, :4], n, m, beta)
    Phi, n, m, beta = small_market(4, 5, seed=19, beta=0.8)
    p4 = brute.primal_newton(Phi[:, :4], n, m[:4], beta)
    mu_s, _ = swapped(Phi, n, m, beta)
    assert not np.allclose(mu_s, p4.mu, rtol=1e-8)
    # transposed kernel in the row pass (on the square part)
    def transposed(Phi, n, m, beta):
        K = ipfp.kernel_matrix(Phi[:, :4], beta)
        v = np.ones(4)
        for _ in range(3000):
            u = ipfp.root(n, 0.5 * K.T @ v)
            v = ipfp.root(m[:4], 0.5 * K @ u)
        return K * np.outer(u, v), u * u
    Phi, n, m, beta = small_market(4, 5, seed=19, beta=0.8)
    p = brute.primal_newton(Phi[:, :4], n, m[:4], beta)
    mu, mx0 = transposed(Phi, n, m, beta)
    assert not np.allclose(mu, p.mu, rtol=1e-8)


def test_packed_rows_reduce_to_plain_rounding_and_log2_kernel():
    """With unit prescale packed_rows is exactly the BF16 / e4m3 rounding, and
    2^(X Y^T) with the prescaled operands approximates exp(Phi / 2 sigma) to
    the operand rounding (each of the 2d products carries <= 2^-8 relative)."""
    rng = np.random.default_rng(21)
    X = rng.normal(0, 0.2, (30, 16)).astype(np.float32)
    Y = rng.normal(0, 0.2, (20, 16)).astype(np.float32)
    assert np.array_equal(quant.packed_rows(X, 0.0, "bf16"), quant.bf16_round(X).astype(np.float64))
    assert np.array_equal(quant.packed_rows(X, 0.0, "fp8"), quant.e4m3_quantize_rows(X)[0])
    assert quant.prescale(np.log2(np.e) / 2) == np.float32(1.0)
    for sigma in (0.3, 1.0):
        Xq = quant.packed_rows(X, sigma, "bf16")
        Yq = quant.packed_rows(Y, sigma, "bf16")
        K2 = ipfp.kernel_from_log2(Xq @ Yq.T)
        K = ipfp.kernel_matrix(X.astype(np.float64) @ Y.astype(np.float64).T, sigma)
        bound = np.abs(X.astype(np.float64)) @ np.abs(Y.astype(np.float64)).T / (2 * sigma)
        assert np.all(np.abs(np.log(K2 / K)) <= 2 * 2.0 ** -8 * bound + 1e-12)


def test_packed_rows_f32_is_one_rounding_of_the_exact_product():
    """FP32 operands: the product p x of two FP32 numbers is exact in FP64
    (48 significant bits), so rounding that FP64 product once to FP32 is the
    correctly rounded FP32 product the packer forms; with unit prescale the
    operands are the FP32 inputs themselves, and the log2 kernel of the FP32
    operands matches exp(Phi / 2 sigma) to FP32 rounding."""
    rng = np.random.default_rng(23)
    X = (rng.normal(0, 0.2, (40, 24)) * np.exp(rng.normal(0, 3, (40, 24)))).astype(np.float32)
    X[0, :3] = (0.0, 1e-42, -3e38)       # zero, a subnormal, a huge value
    unit = np.log2(np.e) / 2
    assert np.array_equal(quant.packed_rows(X, unit, "f32"), X.astype(np.float64))
    for sigma in (0.1, 0.37, 1.0, 5.0):
        p = float(quant.prescale(sigma))
        want = np.array([float(np.float32(float(x) * p)) for x in X.ravel()]).reshape(X.shape)
        got = quant.packed_rows(X, sigma, "f32")
        assert np.array_equal(got, want)
    Y = rng.normal(0, 0.2, (20, 24)).astype(np.float32)
    Xs = rng.normal(0, 0.2, (30, 24)).astype(np.float32)
    for sigma in (0.1, 1.0):
        K2 = ipfp.kernel_from_log2(quant.packed_rows(Xs, sigma, "f32") @
                                   quant.packed_rows(Y, sigma, "f32").T)
        K = ipfp.kernel_matrix(Xs.astype(np.float64) @ Y.astype(np.float64).T, sigma)
        bound = np.abs(Xs.astype(np.float64)) @ np.abs(Y.astype(np.float64)).T / (2 * sigma)
        # p = sqrt(c)(1 + e), |e| <= 2^-24, and each operand carries one more
        # rounding: every product is c x y (1 + 4 u) at worst
        assert np.all(np.abs(np.log(K2 / K)) <= 4 * 2.0 ** -24 * bound + 1e-12)
        assert not np.array_equal(K2, K)


def test_topk_matches_is_repeated_selection():
    """Sec. 4.1: recommendation = the partners of largest mu. Pinned against a
    plain selection loop (take the largest remaining, lowest index on ties)."""
    rng = np.random.default_rng(7)
    L = rng.integers(0, 4, size=(6, 9)).astype(float)   # many exact ties
    L[2, :] = -np.inf
    for k in (1, 3, 9, 12):
        idx, val = ipfp.topk_matches(L, k)
        for r in range(L.shape[0]):
            left = list(range(L.shape[1]))
            for j in range(k):
                if j >= L.shape[1]:
                    assert idx[r, j] == -1 and val[r, j] == -np.inf
                    continue
                best = max(left, key=lambda c: (L[r, c], -c))
                left.remove(best)
                assert idx[r, j] == best and val[r, j] == L[r, best]


def test_welfare_gradient_is_derivative_of_optimal_welfare():
    """Envelope theorem, checked without IPFP: central differences of the
    primal optimum W*(X, Y) (damped Newton on eq. 2-3) against mu Y, mu^T X."""
    rng = np.random.default_rng(11)
    N, M, d, beta = 3, 4, 2, 0.7
    U, Q = rng.normal(0, 0.6, (N, d)), rng.normal(0, 0.6, (N, d))
    V, P = rng.normal(0, 0.6, (M, d)), rng.normal(0, 0.6, (M, d))
    n, m = rng.uniform(0.5, 2.0, N), rng.uniform(0.5, 2.0, M)
    X, Y = np.concatenate([U, Q], 1), np.concatenate([V, P], 1)

    def wstar(X_, Y_):
        return brute.primal_newton(X_ @ Y_.T, n, m, beta).value

    K = ipfp.kernel_matrix(X @ Y.T, beta)
    r = ipfp.ipfp_batch(K, n, m, tol=1e-15, max_sweeps=5000)
    GX, GY = ipfp.welfare_gradient(K, r.a, r.b, X, Y)
    eps = 1e-5
    for (i, j) in [(0, 0), (1, 3), (2, 1)]:
        E = np.zeros_like(X)
        E[i, j] = eps
        fd = (wstar(X + E, Y) - wstar(X - E, Y)) / (2 * eps)
        assert abs(fd - GX[i, j]) < 1e-6 * max(1.0, abs(fd)), (i, j, fd, GX[i, j])
    for (i, j) in [(0, 2), (3, 0)]:
        E = np.zeros_like(Y)
        E[i, j] = eps
        fd = (wstar(X, Y + E) - wstar(X, Y - E)) / (2 * eps)
        assert abs(fd - GY[i, j]) < 1e-6 * max(1.0, abs(fd)), (i, j, fd, GY[i, j])


def test_workload_generators_are_seeded_and_shaped():
    """The seeded inputs both sides share: same seed -> same bytes; the
    configurations' shapes, dtypes and margin distributions."""
    a = workloads.config_market(2, N=300, M=200)
    b = workloads.config_market(2, N=300, M=200)
    for x, y in zip((a.U, a.Q, a.V, a.P, a.n, a.m), (b.U, b.Q, b.V, b.P, b.n, b.m)):
        assert np.array_equal(x, y)
    assert a.U.dtype == np.float32 and a.U.shape == (300, 32) and a.V.shape == (200, 32)
    assert np.all(a.n == 1.0) and set(np.unique(a.m)) <= {1.0, 2.0, 3.0, 4.0, 5.0}
    c5 = workloads.config_market(5, N=1000, M=5000)
    assert c5.m.min() >= 1 and c5.m.max() <= 1000 and c5.U.shape == (1000, 128)
    reqs = workloads.serving_requests(count=64)
    assert len(reqs) == 64 and reqs[0].arrival_s == 0.0
    assert all(1000 <= r.N <= 200_000 and 1000 <= r.M <= 200_000 for r in reqs)
    assert all(r.sigma in (0.5, 1.0) and r.d == 32 for r in reqs)
    assert all(reqs[i].arrival_s <= reqs[i + 1].arrival_s for i in range(63))
    assert workloads.serving_requests(count=64)[5] == reqs[5]


def test_jacobi_sweeps_interleave_two_gauss_seidel_chains():
    """The symmetric single-pass variant (both half-steps from the previous
    sweep's scalings, one kernel evaluation per sweep) is two independent
    copies of the eq. 6 iteration run on alternate sweeps: its u after sweep
    2k - 1 and its v after sweep 2k are exactly the Gauss-Seidel iterate of
    sweep k. So it spends as many kernel evaluations as the paper's order for
    the same iterate, and cannot converge in fewer of them."""
    Phi, n, m, beta = small_market(40, 30, seed=5)
    K = ipfp.kernel_matrix(Phi, beta)
    sweeps = 6
    gs = [ipfp.ipfp_batch(K, n, m, max_sweeps=k) for k in range(1, sweeps + 1)]
    u, v = np.ones(40), np.ones(30)
    ju, jv = [], []
    for _ in range(2 * sweeps):
        u, v = ipfp.root(n, 0.5 * (K @ v)), ipfp.root(m, 0.5 * (K.T @ u))
        ju.append(u)
        jv.append(v)
    for k in range(1, sweeps + 1):
        np.testing.assert_array_equal(ju[2 * k - 2], gs[k - 1].a)
        np.testing.assert_array_equal(jv[2 * k - 1], gs[k - 1].b)


def test_golden_equilibria_computed_in_mpmath():
    """Small markets solved to 60 digits by Newton's method on eq. 5 in mpmath
    (``tests/golden/equilibria.json``, written by
    ``tests/golden/make_golden.py``, which uses no oracle code): the oracle's
    converged IPFP reproduces a, b and mu (eq. 4), and the IPFP-free primal
    Newton solve reproduces mu and the welfare of eq. 2."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "equilibria.json")
    with open(path) as f:
        data = json.load(f)
    assert len(data["markets"]) >= 4
    for mk in data["markets"]:
        Phi = np.array(mk["phi"], dtype=np.float64)
        n = np.array(mk["n"], dtype=np.float64)
        m = np.array(mk["m"], dtype=np.float64)
        beta = float(mk["beta"])
        a = np.array(mk["a"], dtype=np.float64)
        b = np.array(mk["b"], dtype=np.float64)
        mu = np.array(mk["mu"], dtype=np.float64)
        K = ipfp.kernel_matrix(Phi, beta)
        r = ipfp.ipfp_batch(K, n, m, tol=1e-15, max_sweeps=200000)
        np.testing.assert_allclose(r.a, a, rtol=1e-12, err_msg=mk["name"])
        np.testing.assert_allclose(r.b, b, rtol=1e-12, err_msg=mk["name"])
        np.testing.assert_allclose(ipfp.matching(K, r.a, r.b), mu, rtol=1e-12,
                                   err_msg=mk["name"])
        br = brute.primal_newton(Phi, n, m, beta)
        np.testing.assert_allclose(br.mu, mu, rtol=1e-9, err_msg=mk["name"])
        assert abs(br.value - float(mk["welfare"])) <= 1e-10 * abs(float(mk["welfare"]))


def test_golden_file_is_what_its_script_writes(tmp_path):
    """``tests/golden/equilibria.json`` is exactly the output of its committed
    generator (mpmath only), so no stored value comes from anywhere else."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(here, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = tmp_path / "equilibria.json"
    mod.main(str(out))
    with open(os.path.join(here, "equilibria.json")) as f:
        assert out.read_text() == f.read()
