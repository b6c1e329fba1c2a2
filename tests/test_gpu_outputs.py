"""GPU tests of the solve's outputs beyond (a, b): the stable factors of
eq. 11, the top-k recommendation lists ranked by the stable matching, and the
gradient of the optimal welfare with respect to the factors.

Top-k is an integer decision taken from floating-point scores, and near-ties
may order differently in the kernel's FP32 and the oracle's FP64. The oracle
scores the same quantised operands, and the test checks what is unique: every
returned index is valid and distinct, its score matches the oracle's log mu
there, the list is sorted, and it holds every entry that beats the k-th best by
more than the score tolerance, and nothing below it by more than that."""
import numpy as np
import pytest

import workloads
from helpers import banner, market_tensors, require_gpu
from oracle import ipfp as O, quant

pytestmark = pytest.mark.gpu

# |T| stays below ~30 here; FP32 accumulation of a 128-term product and the
# FP32 sum with log2 b are good to ~1e-5 in log2 units
SCORE_TOL = 2e-4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


def test_stable_factors_reproduce_matching(torch, lib):
    banner("stable factors")
    mk = workloads.config_market(1)
    t = market_tensors(torch, mk, torch.float64)
    a, b, _ = lib.solve_market(*t, mk.sigma, tol=1e-12, max_sweeps=500, path="plain",
                               compute="f64")
    psi, xi = lib.stable_factors(t[0], t[1], t[2], t[3], mk.sigma, a, b)
    psi_r, xi_r = O.stable_factors(mk.U, mk.Q, mk.V, mk.P, a.cpu().numpy(), b.cpu().numpy(),
                                   mk.sigma)
    np.testing.assert_allclose(psi.cpu().numpy(), psi_r, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(xi.cpu().numpy(), xi_r, rtol=1e-15, atol=1e-15)
    # log mu_xy = <psi_x, xi_y> / 2 sigma against the library's own mu output
    xs = torch.arange(0, mk.N, 7, device="cuda")
    ys = torch.arange(0, mk.N, 7, device="cuda") % mk.M
    mu = lib.mu_pairs(*t[:4], mk.sigma, a, b, xs, ys).cpu().numpy()
    lm = (psi[xs] * xi[ys]).sum(1).cpu().numpy() / (2 * mk.sigma)
    np.testing.assert_allclose(lm, np.log(mu), rtol=0, atol=1e-12)


@pytest.mark.parametrize("in_dtype", ["f64", "f32", "fp8"])
def test_margin_residuals_match_oracle(torch, lib, in_dtype):
    """eq. 5's margin residuals of a solve's (a, b) against the surplus of the
    factors as given, FP64 on both sides: a plain FP64 solve stopped early
    (residuals of order 1e-3) and a fused BF16 one (its margins hold for the
    rounded operands, so the true residuals show the operand rounding)."""
    banner(f"margin residuals, {in_dtype} factors")
    mk = workloads.config_market(2, N=1500, M=1100)
    sx = sy = None
    if in_dtype == "fp8":
        tens, scales = [], []
        for A, B in ((mk.U, mk.Q), (mk.V, mk.P)):
            vals, s = quant.e4m3_quantize_rows(np.concatenate([A, B], 1).astype(np.float64))
            codes = quant.e4m3_codes(vals / s[:, None])
            d = A.shape[1]
            tens.append([codes[:, :d], codes[:, d:]])
            scales.append(s.astype(np.float32))
            A[...], B[...] = vals[:, :d], vals[:, d:]
        t = [torch.from_numpy(np.ascontiguousarray(c)).cuda().view(torch.float8_e4m3fn)
             for c in (tens[0][0], tens[0][1], tens[1][0], tens[1][1])]
        t += [torch.from_numpy(mk.n).cuda(), torch.from_numpy(mk.m).cuda()]
        sx, sy = (torch.from_numpy(s).cuda() for s in scales)
    else:
        t = market_tensors(torch, mk, torch.float64 if in_dtype == "f64" else torch.float32)
    K = O.kernel_matrix(O.surplus_from_factors(mk.U, mk.Q, mk.V, mk.P), mk.sigma)
    for path, compute, sweeps in (("plain", "f64", 4), ("fused", "bf16", 30)):
        a, b, _ = lib.solve_market(*t, mk.sigma, max_sweeps=sweeps, path=path, compute=compute,
                                   scale_x=sx, scale_y=sy)
        rr, cr, mr, mc = lib.margin_residuals(*t, mk.sigma, a, b, scale_x=sx, scale_y=sy)
        an, bn = a.cpu().numpy(), b.cpu().numpy()
        want_r = np.abs(an * an + an * (K @ bn) - mk.n) / mk.n
        want_c = np.abs(bn * bn + bn * (K.T @ an) - mk.m) / mk.m
        print(f"margin residuals {in_dtype} {path}/{compute}: max row {mr:.3e} col {mc:.3e}",
              flush=True)
        np.testing.assert_allclose(rr.cpu().numpy(), want_r, rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(cr.cpu().numpy(), want_c, rtol=1e-9, atol=1e-13)
        assert mr == float(rr.max()) and mc == float(cr.max())
        assert mr == pytest.approx(O.row_residual(K, an, bn, mk.n), rel=1e-9, abs=1e-13)
        assert mc == pytest.approx(O.col_residual(K, an, bn, mk.m), rel=1e-9, abs=1e-13)


def check_lists(idx, score, ref_logmu, k):
    R, C = ref_logmu.shape
    ref_idx, ref_val = O.topk_matches(ref_logmu, k)
    for r in range(R):
        got = idx[r]
        valid = got[got >= 0]
        assert len(valid) == min(k, C), (r, got)
        assert len(set(valid.tolist())) == len(valid)
        assert np.all(got[len(valid):] == -1) and np.all(np.isneginf(score[r, len(valid):]))
        s = score[r, :len(valid)].astype(np.float64)
        assert np.all(np.diff(s) <= 1e-6), (r, s)
        np.testing.assert_allclose(s, ref_logmu[r, valid], rtol=0, atol=SCORE_TOL)
        kth = ref_val[r, len(valid) - 1]
        must = np.nonzero(ref_logmu[r] > kth + SCORE_TOL)[0]
        assert set(must.tolist()) <= set(valid.tolist()), (r, must, valid)
        assert np.all(ref_logmu[r, valid] >= kth - SCORE_TOL)


@pytest.mark.parametrize("N,M,d,compute,k", [
    (1000, 700, 32, "bf16", 10), (700, 1000, 32, "bf16", 16), (333, 2050, 64, "bf16", 32),
    (900, 600, 64, "fp8", 8), (50, 5, 16, "bf16", 8), (3, 1, 8, "bf16", 4),
    (700, 900, 128, "fp8", 10), (800, 500, 96, "bf16", 12), (600, 650, 128, "bf16", 32),
    (700, 900, 64, "bf16", 10), (513, 777, 48, "bf16", 16),
    (600, 500, 64, "f32", 10), (300, 400, 128, "f32", 16), (70, 40, 16, "f32", 32)])
def test_topk_lists_match_oracle(torch, lib, N, M, d, compute, k):
    banner(f"topk {N}x{M} d={d} {compute} k={k}")
    mk = workloads.factor_market(N, M, d, 1.0 / d, 0.5, "uint1-5", seed=N + M + k,
                                 name="topk")
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, tol=1e-8, max_sweeps=200, compute=compute) as h:
        while not h.run(16):
            pass
        a, b, _ = h.read()
        lists = [h.topk(k, side) for side in (0, 1)]
    a, b = a.cpu().numpy(), b.cpu().numpy()
    X = quant.packed_rows(np.concatenate([mk.U, mk.Q], 1), mk.sigma, compute)
    Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, compute)
    T = X @ Y.T
    logmu = np.log(2.0) * (T + np.log2(a)[:, None] + np.log2(b)[None, :])
    for side, (idx, score) in enumerate(lists):
        ref = logmu if side == 0 else logmu.T
        check_lists(idx.cpu().numpy(), score.cpu().numpy(), ref, k)


@pytest.mark.parametrize("compute,k,ties,d", [("bf16", 10, False, 32), ("fp8", 32, False, 32),
                                              ("bf16", 12, True, 32), ("bf16", 10, False, 64),
                                              ("bf16", 16, True, 48)])
def test_topk_long_rows_match_oracle(torch, lib, compute, k, ties, d):
    """256 rows over a reduced side of 70,000 rows (about 550 stages per
    workgroup, so the lists fill early and then take rare insertions), every
    row against the oracle as in the small cases; with `ties` the reduced
    rows repeat 50 distinct factor rows, so exact ties sit at the k-th
    position. d = 48 and 64 with k <= 16 take the pass that interleaves two
    subtiles' score chains."""
    import dataclasses
    banner(f"topk 256x70000 d={d} {compute} k={k} ties={ties}")
    N, M = 256, 70_000
    mk = workloads.factor_market(N, M, d, 1.0 / d, 0.5, "uint1-5", seed=7000 + k, name="seed")
    if ties:
        pool = np.random.default_rng(5).integers(0, 50, M)
        mk = dataclasses.replace(mk, V=np.ascontiguousarray(mk.V[pool]),
                                 P=np.ascontiguousarray(mk.P[pool]))
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, tol=1e-6, max_sweeps=60, compute=compute) as h:
        while not h.run(20):
            pass
        a, b, _ = h.read()
        idx, score = h.topk(k, 0)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    X = quant.packed_rows(np.concatenate([mk.U, mk.Q], 1), mk.sigma, compute)
    Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, compute)
    logmu = np.log(2.0) * (X @ Y.T + np.log2(a)[:, None] + np.log2(b)[None, :])
    check_lists(idx.cpu().numpy(), score.cpu().numpy(), logmu, k)


def test_topk_full_width_sampled(torch, lib):
    """N = M = 200,000 (grid of many splits): sampled rows against the oracle."""
    banner("topk 200k sampled rows")
    mk = workloads.config_market(3, N=200_000, M=200_000)
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, max_sweeps=3) as h:
        h.run(10)
        a, b, _ = h.read()
        idx, score = h.topk(10, 0)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    rows = np.random.default_rng(3).choice(mk.N, 48, replace=False)
    X = quant.packed_rows(np.concatenate([mk.U[rows], mk.Q[rows]], 1), mk.sigma, "bf16")
    Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, "bf16")
    logmu = np.log(2.0) * (X @ Y.T + np.log2(a[rows])[:, None] + np.log2(b)[None, :])
    check_lists(idx.cpu().numpy()[rows], score.cpu().numpy()[rows], logmu, 10)


@pytest.mark.parametrize("N,M,d", [(1000, 700, 32), (333, 2050, 64), (257, 20000, 32),
                                   (130, 90, 50), (64, 70, 100), (100, 41, 128),
                                   (300, 500, 16), (200, 333, 48), (150, 260, 80),
                                   (170, 129, 96)])
def test_gradient_matches_oracle(torch, lib, N, M, d):
    """G = mu [V|P] and mu^T [U|Q] (envelope theorem) against the oracle on
    the same packed operands. Bound per component, from the arithmetic: P in
    two BF16 parts (relative 2^-18); each FP32 accumulator takes 16 MFMA
    additions per 128-row stage and is folded into FP64 every 8 stages
    (128 x 2^-24), so |G - G_ref| <= 1.2e-5 sum_y mu_xy |Y_y| < 2e-5.
    The widths cover every column-group layout: 2d = 32, 64, 96 (one group of
    1-3 blocks), 128 and 256 (full groups of 4), and 160, 200, 192 (a full
    group and a narrower second one of 1, 3 and 2 blocks)."""
    banner(f"gradient {N}x{M} d={d}")
    mk = workloads.factor_market(N, M, d, 1.0 / d, 0.7, "uint1-5", seed=N * 7 + M + d,
                                 name="grad")
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, tol=1e-9, max_sweeps=300) as h:
        while not h.run(16):
            pass
        a, b, _ = h.read()
        gx = h.gradient(0).cpu().numpy()
        gy = h.gradient(1).cpu().numpy()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    p = float(quant.prescale(mk.sigma))
    X = quant.packed_rows(np.concatenate([mk.U, mk.Q], 1), mk.sigma, "bf16")
    Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, "bf16")
    K = O.kernel_from_log2(X @ Y.T)
    GX, GY = O.welfare_gradient(K, a, b, X / p, Y / p)
    mu = O.matching(K, a, b)
    bx = mu @ np.abs(Y / p)
    by = mu.T @ np.abs(X / p)
    ex = np.max(np.abs(gx - GX) / bx)
    ey = np.max(np.abs(gy - GY) / by)
    print(f"gradient {N}x{M} d={d}: max |err| / sum mu|Y| = {ex:.2e} (rows), {ey:.2e} (cols)",
          flush=True)
    assert gx.shape == (N, 2 * d) and gy.shape == (M, 2 * d)
    assert ex < 2e-5 and ey < 2e-5


def test_gradient_full_width_sampled(torch, lib):
    """N = M = 200,000, d = 64 (C3 distribution; many splits, both column
    groups of the launch): sampled rows and columns against the oracle on the
    same packed operands, with the bound of the small-size test."""
    banner("gradient 200k sampled rows and columns")
    mk = workloads.config_market(3, N=200_000, M=200_000)
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, max_sweeps=4) as h:
        h.run(3)
        a, b, _ = h.read()
        gx = h.gradient(0).cpu().numpy()
        gy = h.gradient(1).cpu().numpy()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    p = float(quant.prescale(mk.sigma))
    X = quant.packed_rows(np.concatenate([mk.U, mk.Q], 1), mk.sigma, "bf16")
    Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, "bf16")
    rng = np.random.default_rng(64)
    for side, G, A, B, wa, wb in ((0, gx, X, Y, a, b), (1, gy, Y, X, b, a)):
        rows = rng.choice(A.shape[0], 24, replace=False)
        mu = O.kernel_from_log2(A[rows] @ B.T) * wa[rows][:, None] * wb[None, :]
        ref = mu @ (B / p)
        bound = mu @ np.abs(B / p)
        err = np.max(np.abs(G[rows] - ref) / bound)
        print(f"gradient 200k side {side}: max |err| / sum mu|Y| = {err:.2e}", flush=True)
        assert err < 2e-5


def test_output_errors(torch, lib):
    """Invalid requests for the outputs are refused with IPFP_EINVAL: k outside
    1..32, a side other than 0 or 1, the gradient of FP8 operands, and top-k or
    gradient of a plain (materialised-K) market."""
    banner("output error paths")
    mk = workloads.factor_market(300, 200, 16, 1.0 / 16, 1.0, "unit", seed=5, name="err")
    t = market_tensors(torch, mk)
    with lib.Market(*t, mk.sigma, max_sweeps=3) as h:
        h.run(2)
        for call in (lambda: h.topk(0, 0), lambda: h.topk(33, 0), lambda: h.topk(4, 2),
                     lambda: h.gradient(2)):
            with pytest.raises(lib.IPFPError) as e:
                call()
            assert e.value.code == -1
        idx, _ = h.topk(4, 1)          # still usable after refused calls
        assert idx.shape == (200, 4)
    with lib.Market(*t, mk.sigma, max_sweeps=3, compute="fp8") as h:
        h.run(1)
        with pytest.raises(lib.IPFPError) as e:
            h.gradient(0)
        assert e.value.code == -1
    with lib.Market(*t, mk.sigma, max_sweeps=3, path="plain", compute="f32") as h:
        h.run(1)
        for call in (lambda: h.topk(4, 0), lambda: h.gradient(0)):
            with pytest.raises(lib.IPFPError) as e:
                call()
            assert e.value.code == -1
