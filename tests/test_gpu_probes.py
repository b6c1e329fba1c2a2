"""GPU tests of the roofline probes (ipfp_probe): every kind runs and returns a
rate that is physically possible on one MI355X (no MFMA probe above its
published dense peak, the read probe below the HBM peak), the mixed probes
sit below the bare matrix stream, and malformed requests are refused."""
import ctypes

import pytest

from helpers import banner, require_gpu

pytestmark = pytest.mark.gpu

# published dense peaks (flop/s) and HBM bandwidth (B/s), with 5 % slack for
# timer granularity
PEAK = {"mfma_bf16": 2.5e15, "mfma_fp8": 5.0e15, "mfma_f32": 157.3e12,
        "mfma_bf16_2w": 2.5e15, "mfma_bf16_epi": 2.5e15, "mfma_fp8_epi": 5.0e15,
        "hbm_read": 8.0e12}
# small work sizes: each launch lasts a few milliseconds
WORK = {"exp2": 20000, "mfma_bf16": 4000, "mfma_fp8": 2000, "mfma_f32": 1000,
        "hbm_read": 1 << 30, "mfma_bf16_2w": 30000, "mfma_bf16_epi": 30000,
        "mfma_fp8_epi": 15000}


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib():
    import paper_2411_19214_amd as L
    return L


def test_every_probe_returns_a_possible_rate(torch, lib):
    banner("probes")
    rates = {}
    for kind, work in WORK.items():
        rate, ms = lib.probe(kind, work)
        print(f"probe {kind}: {rate:.4g} in {ms:.2f} ms", flush=True)
        assert ms > 0 and rate > 0
        if kind in PEAK:
            assert rate < 1.05 * PEAK[kind], kind
        rates[kind] = rate
    # the epilogue beside the matrix stream can only slow it down
    assert rates["mfma_bf16_epi"] < 1.02 * rates["mfma_bf16_2w"]
    assert rates["mfma_fp8_epi"] < 1.02 * rates["mfma_fp8"]


def test_probe_refuses_bad_requests(torch, lib):
    from paper_2411_19214_amd import _lib
    L = lib.library()
    ctx = lib.Context.default(0)
    rate, ms = ctypes.c_double(), ctypes.c_double()
    for kind, work in ((-1, 100), (8, 100), (_lib.PROBE_EXP2, 0),
                       (_lib.PROBE_HBM_READ, (1 << 30) + 16)):
        assert L.ipfp_probe(ctx.handle, kind, work, ctypes.byref(rate), ctypes.byref(ms),
                            None) == _lib.EINVAL, (kind, work)
