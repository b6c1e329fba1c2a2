"""GPU parity of the plain (materialised-K) path against the FP64 oracle."""
import numpy as np
import pytest

import workloads
from helpers import banner, market_tensors, rel_err, require_gpu, to_dev
from oracle import ipfp as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


def oracle_factor(mk, sweeps, tol=0.0, check_every=1):
    Phi = O.surplus_from_factors(mk.U, mk.Q, mk.V, mk.P)
    K = O.kernel_matrix(Phi, mk.sigma)
    return K, O.ipfp_batch(K, mk.n, mk.m, tol=tol, max_sweeps=sweeps,
                           check_every=check_every)


def test_c1_fp64_converges_like_oracle(torch, lib):
    """Config C1 (500 x 400, d = 16, FP64): parity to 1e-12 at tol 1e-10."""
    banner("C1 plain f64")
    mk = workloads.config_market(1)
    U, Q, V, P, n, m = market_tensors(torch, mk, torch.float64)
    a, b, info = lib.solve_market(U, Q, V, P, n, m, mk.sigma, tol=1e-10,
                                  max_sweeps=2000, path="plain", compute="f64")
    K, r = oracle_factor(mk, 2000, tol=1e-10)
    assert info.status == 0 and info.sweeps == r.sweeps
    assert rel_err(a.cpu().numpy(), r.a) < 1e-12
    assert rel_err(b.cpu().numpy(), r.b) < 1e-12
    np.testing.assert_allclose(info.residuals, r.res_hist, rtol=1e-6, atol=1e-15)
    assert info.final_res < 1e-10


@pytest.mark.parametrize("N,M", [(1, 1), (2, 31), (33, 2), (255, 257), (257, 1000),
                                 (1000, 33)])
def test_explicit_phi_ragged_f64_and_f32(torch, lib, N, M):
    banner(f"phi ragged {N}x{M}")
    Phi = workloads.random_phi(N, M, 0.7, seed=N * 7919 + M)
    n = workloads.random_margins(N, 0.5, 2.0, seed=N + 1)
    m = workloads.random_margins(M, 0.5, 3.0, seed=M + 2)
    K = O.kernel_matrix(Phi, 0.8)
    r = O.ipfp_batch(K, n, m, max_sweeps=25, check_every=5)
    for compute, tol in (("f64", 1e-13), ("f32", 2e-6)):
        a, b, info = lib.solve_market_phi(to_dev(torch, Phi), to_dev(torch, n),
                                          to_dev(torch, m), 0.8, max_sweeps=25,
                                          check_every=5, compute=compute)
        assert info.sweeps == 25 and len(info.residuals) == 5
        assert rel_err(a.cpu().numpy(), r.a) < tol, compute
        assert rel_err(b.cpu().numpy(), r.b) < tol, compute
        np.testing.assert_allclose(info.residuals, r.res_hist, rtol=1e-4 if compute == "f32" else 1e-9,
                                   atol=1e-12)


def test_explicit_phi_fp32_input(torch, lib):
    banner("phi f32 input")
    Phi = workloads.random_phi(300, 200, 1.0, seed=3).astype(np.float32)
    n = np.ones(300)
    m = workloads.random_margins(200, 1, 4, seed=4)
    r = O.ipfp_batch(O.kernel_matrix(Phi.astype(np.float64), 0.5), n, m, max_sweeps=40)
    a, b, info = lib.solve_market_phi(to_dev(torch, Phi), to_dev(torch, n), to_dev(torch, m),
                                      0.5, max_sweeps=40, compute="f64")
    assert rel_err(a.cpu().numpy(), r.a) < 1e-12


def test_c2_shape_fp32_mu_within_1e5(torch, lib):
    """C2 distribution at 4000 x 4000: plain FP32 K, mu relative error <= 1e-5
    against the FP64 oracle at the same sweep count."""
    banner("C2-shape plain f32 4000")
    mk = workloads.config_market(2, N=4000, M=4000)
    U, Q, V, P, n, m = market_tensors(torch, mk)
    a, b, info = lib.solve_market(U, Q, V, P, n, m, mk.sigma, max_sweeps=60,
                                  check_every=10, path="plain", compute="f32")
    K, r = oracle_factor(mk, 60, check_every=10)
    ag, bg = a.cpu().numpy(), b.cpu().numpy()
    assert rel_err(ag, r.a) < 1e-5 and rel_err(bg, r.b) < 1e-5
    rng = np.random.default_rng(0)
    xs, ys = rng.integers(0, 4000, 20000), rng.integers(0, 4000, 20000)
    mu_g = K[xs, ys] * ag[xs] * bg[ys]
    mu_o = K[xs, ys] * r.a[xs] * r.b[ys]
    assert rel_err(mu_g, mu_o) < 1e-5


def test_warm_start_resume_is_bitwise(torch, lib):
    banner("plain warm start")
    mk = workloads.config_market(1, N=300, M=200)
    U, Q, V, P, n, m = market_tensors(torch, mk, torch.float64)
    kw = dict(path="plain", compute="f64")
    a_full, b_full, _ = lib.solve_market(U, Q, V, P, n, m, mk.sigma, max_sweeps=30, **kw)
    _, b_half, _ = lib.solve_market(U, Q, V, P, n, m, mk.sigma, max_sweeps=15, **kw)
    a2, b2, _ = lib.solve_market(U, Q, V, P, n, m, mk.sigma, max_sweeps=15, b0=b_half, **kw)
    assert torch.equal(a_full, a2) and torch.equal(b_full, b2)


def test_graph_replay_matches_eager(torch, lib):
    banner("plain graph vs eager")
    mk = workloads.config_market(1, N=500, M=400)
    U, Q, V, P, n, m = market_tensors(torch, mk)
    outs = []
    for g in (False, True):
        outs.append(lib.solve_market(U, Q, V, P, n, m, mk.sigma, tol=1e-9, max_sweeps=500,
                                     check_every=4, path="plain", use_graph=g))
    (a0, b0, i0), (a1, b1, i1) = outs
    assert torch.equal(a0, a1) and torch.equal(b0, b1) and i0.sweeps == i1.sweeps


def test_invalid_margin_and_nonfinite(torch, lib):
    banner("plain error paths")
    Phi = to_dev(torch, workloads.random_phi(10, 8, 1.0, seed=5))
    n = to_dev(torch, np.ones(10))
    m = to_dev(torch, np.ones(8))
    bad = n.clone()
    bad[3] = 0.0
    with pytest.raises(lib.IPFPError) as e:
        lib.solve_market_phi(Phi, bad, m, 1.0, max_sweeps=3)
    assert e.value.code == -1
    Pn = Phi.clone()
    Pn[2, 2] = float("nan")
    with pytest.raises(lib.IPFPError) as e:
        lib.solve_market_phi(Pn, n, m, 1.0, max_sweeps=3)
    assert e.value.code == -4
    with pytest.raises(lib.IPFPError) as e:
        lib.solve_market_phi(Phi, n, m, -1.0, max_sweeps=3)
    assert e.value.code == -1


def test_not_converged_status(torch, lib):
    mk = workloads.config_market(1, N=200, M=150)
    U, Q, V, P, n, m = market_tensors(torch, mk, torch.float64)
    a, b, info = lib.solve_market(U, Q, V, P, n, m, mk.sigma, tol=1e-14, max_sweeps=3,
                                  path="plain", compute="f64")
    assert info.status == 1 and info.sweeps == 3 and len(info.residuals) == 3


def test_golden_equilibria_fp64(torch, lib):
    """The plain FP64 path on the markets solved to 60 digits in mpmath
    (eq. 5; ``tests/golden/equilibria.json``): a, b within 1e-12 relative."""
    import json
    import os
    banner("golden equilibria plain f64")
    path = os.path.join(os.path.dirname(__file__), "golden", "equilibria.json")
    with open(path) as f:
        markets = json.load(f)["markets"]
    for mk in markets:
        Phi = np.array(mk["phi"], dtype=np.float64)
        n = np.array(mk["n"], dtype=np.float64)
        m = np.array(mk["m"], dtype=np.float64)
        a, b, info = lib.solve_market_phi(to_dev(torch, Phi), to_dev(torch, n),
                                          to_dev(torch, m), float(mk["beta"]), tol=1e-15,
                                          max_sweeps=4000, check_every=10, compute="f64")
        print(f"golden {mk['name']}: {info.sweeps} sweeps, residual {info.final_res:.1e}",
              flush=True)
        assert rel_err(a.cpu().numpy(), np.array(mk["a"], dtype=np.float64)) < 1e-12
        assert rel_err(b.cpu().numpy(), np.array(mk["b"], dtype=np.float64)) < 1e-12
