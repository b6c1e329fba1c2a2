"""The allocation-free solve (``ipfp_solve_market_noalloc``) against the
allocating one (``ipfp_solve_market``), through the C ABI.

Both run the same set-up and sweep kernels with the same split counts, so
their (a, b), residual histories and sweep counts must agree bit for bit --
stricter than the parity bar of the kernels against the oracle, which the
allocating solve already meets. Two calls in a row on the per-device scratch
array, the second with a smaller market, show that what the first call leaves
behind does not leak into the second."""
import numpy as np
import pytest

import workloads
from helpers import banner, market_tensors, require_gpu
from paper_2411_19214_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


def same(x, y):
    return np.array_equal(x.cpu().numpy().view(np.uint64), y.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("compute", ["bf16", "fp8"])
def test_noalloc_equals_solve_two_calls(torch, lib, compute):
    big = workloads.config_market(3, N=3001, M=2477)
    small = workloads.config_market(2, N=1203, M=911)
    tb, ts = market_tensors(torch, big), market_tensors(torch, small)
    kw = dict(max_sweeps=9, check_every=2, compute=compute)
    banner(f"noalloc {compute}: {big.N}x{big.M} d={big.d}, then {small.N}x{small.M} d={small.d}")
    # two allocation-free calls in a row, the second smaller
    nb = lib.solve_market(*tb, big.sigma, no_alloc=True, **kw)
    ns = lib.solve_market(*ts, small.sigma, no_alloc=True, **kw)
    rb = lib.solve_market(*tb, big.sigma, **kw)
    rs = lib.solve_market(*ts, small.sigma, **kw)
    for (na, nbv, ni), (ra, rbv, ri) in ((nb, rb), (ns, rs)):
        assert ni.status == ri.status == _lib.OK
        assert ni.sweeps == ri.sweeps == 9
        assert same(na, ra) and same(nbv, rbv)
        assert ni.residuals == ri.residuals
        assert ni.fixups == ri.fixups


def test_noalloc_converged_and_plain(torch, lib):
    # a tolerance stop (the returned state is the converged sweep's) on the
    # fused path, then the plain FP64 path (K carved from the same array)
    mk = workloads.config_market(3, N=2500, M=2100)
    t = market_tensors(torch, mk)
    banner("noalloc fused tol 1e-7, then plain f64 C1")
    n = lib.solve_market(*t, mk.sigma, tol=1e-7, max_sweeps=200, no_alloc=True)
    r = lib.solve_market(*t, mk.sigma, tol=1e-7, max_sweeps=200)
    assert n[2].status == r[2].status == _lib.OK and n[2].sweeps == r[2].sweeps
    assert same(n[0], r[0]) and same(n[1], r[1]) and n[2].residuals == r[2].residuals
    c1 = workloads.config_market(1)
    t1 = market_tensors(torch, c1, dtype=torch.float64)
    kw = dict(path="plain", compute="f64", tol=1e-10, max_sweeps=2000)
    n = lib.solve_market(*t1, c1.sigma, no_alloc=True, **kw)
    r = lib.solve_market(*t1, c1.sigma, **kw)
    assert n[2].status == r[2].status == _lib.OK and n[2].sweeps == r[2].sweeps
    assert same(n[0], r[0]) and same(n[1], r[1]) and n[2].residuals == r[2].residuals


def test_noalloc_refuses_a_market_beyond_the_array(torch, lib):
    # plain FP32 K of 3000 x 6000 needs 72 MB > 64 MiB: refused before any launch
    mk = workloads.config_market(2, N=3000, M=6000)
    t = market_tensors(torch, mk)
    assert lib.footprint(3000, 6000, mk.d, path="plain") > _lib.NOALLOC_BYTES
    banner("noalloc refusal")
    with pytest.raises(lib.IPFPError) as e:
        lib.solve_market(*t, mk.sigma, path="plain", compute="f32", max_sweeps=3,
                         no_alloc=True)
    assert e.value.code == _lib.EBUDGET
    # the array still works afterwards
    small = workloads.config_market(2, N=700, M=500)
    ts = market_tensors(torch, small)
    n = lib.solve_market(*ts, small.sigma, max_sweeps=5, no_alloc=True)
    r = lib.solve_market(*ts, small.sigma, max_sweeps=5)
    assert same(n[0], r[0]) and same(n[1], r[1])
