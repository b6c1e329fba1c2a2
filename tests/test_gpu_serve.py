"""GPU tests of the serving layer: grouped launches over many resident markets
must give every request exactly the result of solving it alone (the grouped
kernels run the single-market arithmetic per market), small requests must
match the FP64 oracle, and admission, cancellation and error reporting must
behave as documented."""
import numpy as np
import pytest

import workloads
from helpers import banner, market_tensors, rel_err, require_gpu, to_dev
from oracle import ipfp as O, quant

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


# (N, M, d, sigma, tol, max_sweeps, check_every): sizes across all three lanes,
# ragged against every tile, two kpads (d = 32 -> 64, d = 40 -> 96)
MIX = [
    (700, 1300, 32, 1.0, 1e-6, 60, 1),
    (1500, 900, 32, 0.5, 1e-6, 60, 1),
    (3100, 2900, 32, 1.0, 0.0, 9, 3),
    (5000, 7001, 40, 0.5, 1e-6, 60, 2),
    (9000, 12000, 32, 1.0, 1e-6, 60, 1),
    (12345, 9876, 40, 1.0, 1e-6, 60, 1),
    (30000, 20000, 32, 0.5, 1e-6, 40, 4),
    (70000, 60000, 32, 1.0, 1e-6, 30, 1),
]


def mix_market(i, N, M, d, sigma):
    return workloads.factor_market(N, M, d, 1.0 / d, sigma, col_margin="uint1-5",
                                   seed=19214 + 7000 + i, name=f"mix{i}")


def alone(torch, lib, t, spec, compute):
    N, M, d, sigma, tol, ms, ce = spec
    return lib.solve_market(*t, sigma, tol=tol, max_sweeps=ms, check_every=ce,
                            compute=compute)


@pytest.mark.parametrize("compute,widths", [
    ("bf16", dict(chunk=3, lanes=3)), ("fp8", dict(chunk=3, lanes=3)),
    ("bf16", dict(chunk=1, lanes=4, lane_blocks=512)),
    ("bf16", dict(chunk=8, lanes=2, lane_blocks=4096))])
def test_mix_equals_alone_bitwise(torch, lib, compute, widths):
    banner(f"serve mix vs alone {compute} {widths}")
    mks = [mix_market(i, *s[:4]) for i, s in enumerate(MIX)]
    tens = [market_tensors(torch, mk) for mk in mks]
    with lib.Server(compute=compute, **widths) as srv:
        reqs = []
        # half now, the rest while the first half runs
        for i, (t, s) in enumerate(zip(tens, MIX)):
            N, M, d, sigma, tol, ms, ce = s
            reqs.append(srv.submit(*t, sigma, tol=tol, max_sweeps=ms, check_every=ce))
            if i == len(MIX) // 2:
                srv.wait(reqs[0])
        for r in reqs:
            srv.wait(r, timeout_ms=60_000)
        lanes = {r.lane for r in reqs}
        st = srv.stats()
    assert all(r.finished for r in reqs)
    # the mix's sizes fall in three size classes whatever the lane count
    assert len(lanes) == min(widths["lanes"], 3), lanes
    assert st["finished"] == len(MIX) and st["arena_used"] == 0
    for t, s, r in zip(tens, MIX, reqs):
        a, b, info = alone(torch, lib, t, s, compute)
        assert r.status == info.status, (s, r.status, info.status)
        assert r.info.sweeps == info.sweeps and r.info.residuals == info.residuals, s
        assert torch.equal(r.a, a) and torch.equal(r.b, b), s
        assert r.t_submit <= r.t_admit <= r.t_done


# wide FP8 rows: packed widths 192 and 256, which run two output tiles per
# wave in the grouped pass as in the single-market one
WIDE = [(700, 1300, 128, 1.0, 1e-6, 40, 1), (1500, 900, 96, 0.5, 1e-6, 40, 1),
        (3100, 2900, 128, 1.0, 0.0, 9, 3), (20000, 9000, 80, 1.0, 1e-6, 30, 2)]


def test_wide_fp8_mix_equals_alone_bitwise(torch, lib):
    banner("serve wide fp8 mix vs alone")
    mks = [mix_market(100 + i, *s[:4]) for i, s in enumerate(WIDE)]
    tens = [market_tensors(torch, mk) for mk in mks]
    with lib.Server(compute="fp8", chunk=3, lanes=2) as srv:
        reqs = [srv.submit(*t, s[3], tol=s[4], max_sweeps=s[5], check_every=s[6])
                for t, s in zip(tens, WIDE)]
        for r in reqs:
            srv.wait(r, timeout_ms=60_000)
    for t, s, r in zip(tens, WIDE, reqs):
        a, b, info = alone(torch, lib, t, s, "fp8")
        assert r.status == info.status, (s, r.status, info.status)
        assert r.info.sweeps == info.sweeps and r.info.residuals == info.residuals, s
        assert torch.equal(r.a, a) and torch.equal(r.b, b), s


def test_serving_tuner_choice_keeps_results(torch, lib, tmp_path):
    """The serving-width tuner runs a small mix over its candidates and caches
    a choice; a server with those widths still returns every request's
    alone-solve result bit for bit."""
    from paper_2411_19214_amd import tune
    banner("serving tuner on a small mix")
    specs = MIX[:5]
    mks = [mix_market(i, *s[:4]) for i, s in enumerate(specs)]
    tens = [market_tensors(torch, mk) for mk in mks]
    path = str(tmp_path / "tune.json")
    out = tune.tune_serving(tens, [0.0, 0.001, 0.002, 0.003, 0.004], [s[3] for s in specs],
                            repeats=1, arena_bytes=1 << 30, path=path, max_sweeps=40)
    choice = out["choice"]
    assert len(out["trials"]) == 7
    assert set(choice) == {"chunk", "lane_blocks", "lanes"}
    assert tune._load(path)
    with lib.Server(compute="bf16", **choice) as srv:
        reqs = [srv.submit(*t, s[3], tol=1e-6, max_sweeps=40) for t, s in zip(tens, specs)]
        for r in reqs:
            srv.wait(r, timeout_ms=60_000)
    for t, s, r in zip(tens, specs, reqs):
        a, b, info = lib.solve_market(*t, s[3], tol=1e-6, max_sweeps=40)
        assert r.status == info.status and torch.equal(r.a, a) and torch.equal(r.b, b)


def test_unconverged_mix_shapes_follow_the_oracle(torch, lib):
    """The serving mix's requests that stop at the 200-sweep cap are nearly
    balanced (N within 4 % of M, unit margins, sigma = 1): IPFP's slowest mode,
    the balance between the two sides' unmatched masses, contracts slowly
    there. On the very factors the benchmark draws on the device, the served
    solve (identical to solving alone) follows the FP64 oracle fed the same
    BF16 operands check by check, and the oracle on the unquantised factors
    is just as slow: the cap, not a precision floor, stops them."""
    reqs = [r for r in workloads.serving_requests()
            if r.sigma == 1.0 and max(r.N, r.M) <= 8000 and abs(r.N - r.M) <= 0.04 * r.N]
    assert len(reqs) >= 3
    for r in reqs[:4]:
        banner(f"served shape {r.N}x{r.M} sigma={r.sigma} (request {r.index}), 200 sweeps")
        t = workloads.device_request_factors(torch, r)
        a, b, info = lib.solve_market(*t, r.sigma, tol=1e-6, max_sweeps=200, check_every=1)
        U, Q, V, P = (x.cpu().numpy() for x in t[:4])
        n, m = np.ones(r.N), np.ones(r.M)
        X = quant.packed_rows(np.concatenate([U, Q], 1), r.sigma, "bf16")
        Y = quant.packed_rows(np.concatenate([V, P], 1), r.sigma, "bf16")
        ref = O.ipfp_batch(O.kernel_from_log2(X @ Y.T), n, m, tol=1e-6, max_sweeps=200)
        ex = O.ipfp_batch(O.kernel_matrix(O.surplus_from_factors(U, Q, V, P), r.sigma), n, m,
                          tol=1e-6, max_sweeps=200)
        h = info.residuals
        print(f"request {r.index} {r.N}x{r.M}: GPU {info.sweeps} sweeps, residual "
              f"{h[-1]:.3e}; oracle (same operands) {ref.sweeps} sweeps {ref.res_hist[-1]:.3e}; "
              f"oracle (FP64 factors) {ex.sweeps} sweeps {ex.res_hist[-1]:.3e}", flush=True)
        np.testing.assert_allclose(h, ref.res_hist, rtol=5e-3, atol=3e-7)
        assert info.sweeps == ref.sweeps
        assert rel_err(a.cpu().numpy(), ref.a) < 2e-5 and rel_err(b.cpu().numpy(), ref.b) < 2e-5
        # the exact market is as slow: the same stop (or within a few sweeps of it)
        assert abs(ex.sweeps - ref.sweeps) <= max(5, ref.sweeps // 20)


def test_small_requests_match_oracle(torch, lib):
    banner("serve small requests vs oracle")
    specs = MIX[:2]
    mks = [mix_market(i, *s[:4]) for i, s in enumerate(specs)]
    with lib.Server() as srv:
        reqs = [srv.submit(*market_tensors(torch, mk), s[3], tol=s[4], max_sweeps=s[5],
                           check_every=s[6]) for mk, s in zip(mks, specs)]
        for r in reqs:
            srv.wait(r)
    for mk, s, r in zip(mks, specs, reqs):
        X = quant.packed_rows(np.concatenate([mk.U, mk.Q], 1), mk.sigma, "bf16")
        Y = quant.packed_rows(np.concatenate([mk.V, mk.P], 1), mk.sigma, "bf16")
        ref = O.ipfp_batch(O.kernel_from_log2(X @ Y.T), mk.n, mk.m, tol=s[4],
                           max_sweeps=s[5], check_every=s[6])
        assert r.info.sweeps == ref.sweeps
        assert rel_err(r.a.cpu().numpy(), ref.a) < 2e-5
        assert rel_err(r.b.cpu().numpy(), ref.b) < 2e-5


def test_admission_by_footprint(torch, lib):
    banner("serve admission under a small arena")
    specs = [MIX[4], MIX[5], MIX[4], MIX[5]]
    foot = max(lib.footprint(s[0], s[1], s[2]) for s in specs)
    mks = [mix_market(10 + i, *s[:4]) for i, s in enumerate(specs)]
    tens = [market_tensors(torch, mk) for mk in mks]
    with lib.Server(arena_bytes=int(foot * 2.2)) as srv:
        reqs = [srv.submit(*t, s[3], tol=s[4], max_sweeps=s[5], check_every=s[6])
                for t, s in zip(tens, specs)]
        for r in reqs:
            srv.wait(r)
        st = srv.stats()
        # a market that can never fit is refused at once
        big = workloads.factor_market(200_000, 200_000, 32, 1 / 32, 1.0, seed=5, name="big")
        with pytest.raises(lib.IPFPError) as e:
            srv.submit(*market_tensors(torch, big), 1.0)
        assert e.value.code == -2
    assert st["arena_peak"] <= st["arena_bytes"]
    # not all four fit at once, so someone waited for a slot
    assert max(r.t_admit for r in reqs) >= min(r.t_done for r in reqs)
    for t, s, r in zip(tens, specs, reqs):
        a, b, info = alone(torch, lib, t, s, "bf16")
        assert torch.equal(r.a, a) and torch.equal(r.b, b)


def test_cancel_and_errors(torch, lib):
    banner("serve cancel, invalid margin, compute mismatch")
    s = MIX[6]
    mk = mix_market(20, *s[:4])
    t = market_tensors(torch, mk)
    bad = mix_market(21, 900, 800, 32, 1.0)
    U, Q, V, P, n, m = market_tensors(torch, bad)
    m[5] = 0.0
    with lib.Server(max_active=1) as srv:
        long = srv.submit(*t, s[3], tol=0.0, max_sweeps=100_000)
        queued = srv.submit(*t, s[3], tol=0.0, max_sweeps=10)
        broken = srv.submit(U, Q, V, P, n, m, 1.0, tol=1e-6)
        srv.cancel(queued)
        srv.wait(queued)
        assert queued.status == -5 and queued.t_admit == 0.0
        srv.cancel(long)
        srv.wait(long, timeout_ms=60_000)
        assert long.status == -5
        srv.wait(broken, timeout_ms=60_000)
        assert broken.status == -1
        # a request whose compute differs from the server's is refused
        import ctypes
        from paper_2411_19214_amd import _lib
        mk_s = lib._market_struct(*t, s[3])
        opt = lib._options("fused", "fp8", 1e-6, 10, 1, 0, 0, None, False, False)
        res = _lib.Result()
        res.a, res.b = long.a.data_ptr(), long.b.data_ptr()
        tk = ctypes.c_uint64()
        rc = lib.library().ipfp_submit(srv.handle, ctypes.byref(mk_s), ctypes.byref(opt),
                                       ctypes.byref(res), ctypes.byref(tk), None)
        assert rc == -1
