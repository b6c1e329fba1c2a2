"""End-to-end precision of each compute type against the FP64 oracle on the
unquantised factors, at reduced sizes that keep each configuration's
distribution (factor variance, sigma, margins).

Both sides run the same fixed number of sweeps. Two matchings are measured
over every pair, each against the oracle's mu:
* mu as the library returns it (``ipfp_mu_pairs``): K in FP64 from the factors
  as given, times the GPU's scalings a_x b_y (eq. 4);
* mu implied by the solve itself: K of the rounded operands the kernels used
  (2^T with T from the same quantised values, formed by the oracle), times
  the GPU's a_x b_y -- the matching whose margins the solve satisfies.
Bars:
* the plain FP32 path and the fused FP32 path: within 1e-5 relative on every
  mu_xy as returned;
* the fused BF16 path: mu as returned within 1e-3 relative on every pair
  (max, every case, sigma = 0.1 included). That is the matching the library
  hands out, so the 1e-3 target applies to it. The solve's own matching (K of
  the BF16 operands) is bounded by its measured RMS and max with a margin of
  1.5, to catch regressions; at sigma = 0.1 its RMS is 1.5e-3, above 1e-3,
  because the operand rounding moves every exponent by about
  2^-9 |terms| sqrt(2d) / (2 sigma);
* FP8 is reported (its operand rounding, not the kernels, sets its error;
  the parity tests bound the kernels' own error).
"""
import numpy as np
import pytest

import workloads
from helpers import banner, market_tensors, require_gpu
from oracle import ipfp as O, quant

pytestmark = pytest.mark.gpu

SWEEPS = 150


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


def mu_errors(K, a, b, ref):
    mu = O.matching(K, a, b)
    mu_ref = O.matching(ref.K, ref.a, ref.b)
    rel = np.abs(mu - mu_ref) / mu_ref
    return float(np.sqrt(np.mean(rel ** 2))), float(rel.max())


CASES = [
    # (config, N, M, sigma, paths, bounds on the BF16 solve's matching: RMS, max)
    (2, 4000, 4000, None, ("plain", "f32", "bf16", "fp8"), (9e-4, 7.2e-3)),
    (3, 4000, 4000, None, ("plain", "f32", "bf16", "fp8"), (3.2e-4, 2.3e-3)),
    (5, 8000, 800, 1.0, ("plain", "f32", "bf16", "fp8"), (2.3e-4, 1.2e-3)),
    (5, 8000, 800, 0.1, ("plain", "f32", "bf16", "fp8"), (2.3e-3, 1.3e-2)),
]


@pytest.mark.parametrize("cfg,N,M,sigma,paths,solve_bound", CASES)
def test_precision_against_fp64_factors(torch, lib, cfg, N, M, sigma, paths, solve_bound):
    banner(f"precision C{cfg} {N}x{M} sigma={sigma}")
    mk = workloads.config_market(cfg, N=N, M=M, sigma=sigma)
    K = O.kernel_matrix(O.surplus_from_factors(mk.U, mk.Q, mk.V, mk.P), mk.sigma)
    ref = O.ipfp_batch(K, mk.n, mk.m, max_sweeps=SWEEPS)
    ref.K = K
    t = market_tensors(torch, mk)
    A = np.concatenate([mk.U, mk.Q], 1)
    B = np.concatenate([mk.V, mk.P], 1)
    for p in paths:
        if p == "plain":
            a, b, _ = lib.solve_market(*t, mk.sigma, max_sweeps=SWEEPS, path="plain",
                                       compute="f32")
            Ks = K
        elif p == "f32":
            a, b, _ = lib.solve_market(*t, mk.sigma, max_sweeps=SWEEPS, compute="f32")
            Ks = O.kernel_from_log2(quant.packed_rows(A, mk.sigma, p) @
                                    quant.packed_rows(B, mk.sigma, p).T)
        else:
            a, b, _ = lib.solve_market(*t, mk.sigma, max_sweeps=SWEEPS, compute=p)
            Ks = O.kernel_from_log2(quant.packed_rows(A, mk.sigma, p) @
                                    quant.packed_rows(B, mk.sigma, p).T)
        a, b = a.cpu().numpy(), b.cpu().numpy()
        out_rms, out_max = mu_errors(K, a, b, ref)
        sol_rms, sol_max = mu_errors(Ks, a, b, ref)
        eab = max(np.max(np.abs(a - ref.a) / ref.a), np.max(np.abs(b - ref.b) / ref.b))
        print(f"precision C{cfg} N={N} M={M} d={mk.d} sigma={mk.sigma} {p}: "
              f"mu returned RMS {out_rms:.2e} max {out_max:.2e}; "
              f"mu of the solve RMS {sol_rms:.2e} max {sol_max:.2e}; "
              f"a,b max rel {eab:.2e}", flush=True)
        if p in ("plain", "f32"):
            assert out_max < 1e-5
        elif p == "bf16":
            assert out_max < 1e-3
            assert sol_rms < solve_bound[0] and sol_max < solve_bound[1]
