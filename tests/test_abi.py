"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and its host-side logic (defaults, validation, footprint
sizes, error strings) behaves as documented. No device work is launched."""
import ctypes
import os
import re

import pytest

import paper_2411_19214_amd as L
from paper_2411_19214_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipfp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = set(re.findall(r"\b(ipfp_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return L.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ipfp_create", "ipfp_solve_market", "ipfp_solve_market_phi",
                 "ipfp_mu_pairs", "ipfp_footprint", "ipfp_submit", "ipfp_poll",
                 "ipfp_cancel", "ipfp_market_open", "ipfp_pack_side"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_error_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert lib.ipfp_strerror(code).decode()
    assert lib.ipfp_strerror(-99).decode() == "unknown error code"
    assert lib.ipfp_abi_version() == 2


def test_default_options(lib):
    o = _lib.Options()
    lib.ipfp_default_options(ctypes.byref(o))
    assert (o.path, o.compute, o.max_sweeps, o.check_every) == (_lib.PATH_FUSED, _lib.BF16,
                                                                100, 1)
    s = _lib.ServerOptions()
    lib.ipfp_default_server_options(ctypes.byref(s))
    assert (s.max_active, s.lanes, s.chunk, s.compute) == (256, 3, 4, _lib.BF16)
    assert (s.lane_blocks, s.aging_ms) == (2048, 4000.0)
    assert s.arena_bytes == 1 << 30


def _market(N=1000, M=800, d=32):
    mk = _lib.Market()
    mk.N, mk.M, mk.d = N, M, d
    mk.in_dtype = _lib.F32
    mk.U = mk.Q = mk.V = mk.P = 1
    mk.ld_x = mk.ld_y = d
    mk.n = mk.m = 1
    mk.sigma = 1.0
    return mk


def _opts(lib, **kw):
    o = _lib.Options()
    lib.ipfp_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _footprint(lib, mk, o):
    out = ctypes.c_size_t()
    rc = lib.ipfp_footprint(ctypes.byref(mk), ctypes.byref(o), ctypes.byref(out))
    return rc, out.value


def test_footprint_sizes(lib):
    # fused BF16, d = 32: packed operands (2d = 64 codes of 2 B per row) dominate
    rc, b16 = _footprint(lib, _market(100_000, 50_000, 32), _opts(lib))
    assert rc == 0
    packed = (100_000 + 50_000) * 64 * 2
    assert packed < b16 < 4 * packed
    # FP8 halves the operand bytes; the rest (partial sums, shifts) is shared
    rc8, b8 = _footprint(lib, _market(100_000, 50_000, 32), _opts(lib, compute=_lib.FP8E4M3))
    assert rc8 == 0 and b8 < b16 and b16 - b8 >= packed // 2
    # plain FP32 stores K: N x (M rounded up to 64) x 4 B
    rc, b = _footprint(lib, _market(1000, 1000, 8), _opts(lib, path=_lib.PATH_PLAIN,
                                                          compute=_lib.F32))
    assert rc == 0 and b >= 1000 * 1024 * 4


@pytest.mark.parametrize("field,value", [
    ("N", 0), ("M", 0), ("d", 0), ("d", 129), ("sigma", 0.0), ("sigma", float("inf")),
    ("sigma", float("nan")), ("ld_x", 16)])
def test_invalid_markets_are_rejected(lib, field, value):
    mk = _market()
    setattr(mk, field, value)
    rc, _ = _footprint(lib, mk, _opts(lib))
    assert rc == _lib.EINVAL


@pytest.mark.parametrize("field,value", [
    ("max_sweeps", 0), ("check_every", 0), ("tol", -1.0), ("splits", 300),
    ("tile_rows", 384), ("compute", _lib.F64), ("path", 7)])
def test_invalid_options_are_rejected(lib, field, value):
    rc, _ = _footprint(lib, _market(), _opts(lib, **{field: value}))
    assert rc == _lib.EINVAL


def test_plain_path_accepts_wide_factors_fused_does_not(lib):
    mk = _market(d=200)
    assert _footprint(lib, mk, _opts(lib))[0] == _lib.EINVAL
    assert _footprint(lib, mk, _opts(lib, path=_lib.PATH_PLAIN, compute=_lib.F32))[0] == 0


def test_null_arguments(lib):
    assert lib.ipfp_create(None, 0, 0) == _lib.EINVAL
    assert lib.ipfp_solve_market(None, None, None, None, None) == _lib.EINVAL
    assert lib.ipfp_server_create(None, None, None) == _lib.EINVAL
    assert lib.ipfp_poll(None, 1, None) == _lib.EINVAL
    assert lib.ipfp_cancel(None, 1) == _lib.EINVAL
    assert lib.ipfp_footprint(None, None, None) == _lib.EINVAL
    # outputs of a resident market: a null handle is refused before any device call
    assert lib.ipfp_market_topk(None, 0, 10, None, None, None) == _lib.EINVAL
    assert lib.ipfp_market_gradient(None, 0, None, 128, None) == _lib.EINVAL
    assert lib.ipfp_market_run(None, 1, None, None) == _lib.EINVAL
    assert lib.ipfp_stable_factors(None, None, None, None, None, 0, None, 0, None) == _lib.EINVAL
    assert lib.ipfp_tune(None, None, None, None, None, None) == _lib.EINVAL
    assert lib.ipfp_margin_residuals(None, None, None, None, None, None, None, None,
                                     None) == _lib.EINVAL
    assert lib.ipfp_probe(None, 0, 1, None, None, None) == _lib.EINVAL


def test_plan_reports_the_layout(lib):
    # without a device the split rule assumes 256 compute units and one resident
    # workgroup per unit; the plan must agree with the footprint either way
    o = _opts(lib)
    mk = _market(200_000, 50_000, 32)
    p = _lib.Plan()
    assert lib.ipfp_plan_market(ctypes.byref(mk), ctypes.byref(o), ctypes.byref(p)) == 0
    assert p.kpad == 64 and p.rows_per_workgroup in (256, 512)
    assert (p.splits_row, p.splits_col) == (p.auto_splits_row, p.auto_splits_col)
    assert p.blocks_row == -(-200_000 // p.rows_per_workgroup) * p.splits_row
    assert p.footprint_bytes == _footprint(lib, mk, o)[1]
    o2 = _opts(lib, splits=3, splits_col=5)
    assert lib.ipfp_plan_market(ctypes.byref(mk), ctypes.byref(o2), ctypes.byref(p)) == 0
    assert (p.splits_row, p.splits_col) == (3, 5)
    o3 = _opts(lib, splits=3)
    assert lib.ipfp_plan_market(ctypes.byref(mk), ctypes.byref(o3), ctypes.byref(p)) == 0
    assert (p.splits_row, p.splits_col) == (3, 3)
    assert lib.ipfp_plan_market(ctypes.byref(mk), ctypes.byref(_opts(lib, splits_col=-1)),
                                ctypes.byref(p)) == _lib.EINVAL


def test_noalloc_capacity_matches_the_header(lib):
    text = open(HEADER).read()
    m = re.search(r"#define IPFP_NOALLOC_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_BYTES
    assert lib.ipfp_solve_market_noalloc(None, None, None, None, None) == _lib.EINVAL


def test_clock_is_monotonic_ms(lib):
    import time
    a = lib.ipfp_clock_ms()
    t = time.monotonic() * 1e3
    b = lib.ipfp_clock_ms()
    assert a <= t + 1.0 and t <= b + 1.0 and b >= a


def test_tune_cache_keys_and_roundtrip(tmp_path):
    from paper_2411_19214_amd import tune
    k1 = tune.shape_key("gfx950", "bf16", 64, 1_000_000, 1_000_000)
    assert k1 == "gfx950|bf16|k128|N1048576|M1048576"
    assert tune.shape_key("gfx950", "fp8", 32, 700, 1500) == "gfx950|fp8|k64|N512|M2048"
    assert tune.shape_key("gfx950", "bf16", 40, 3, 1) == "gfx950|bf16|k96|N4|M1"
    path = str(tmp_path / "sub" / "tune.json")
    assert tune._load(path) == {}
    tune._store(path, {k1: {"options": {"tile_rows": 512, "splits": 0}}})
    assert tune._load(path)[k1]["options"] == {"tile_rows": 512, "splits": 0}


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before anything imports torch still leaves a single
    HIP runtime mapped (the one torch ships), so torch's device pointers and
    streams are valid on both sides of the boundary."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2411_19214_amd import _lib\n"
            "_lib.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
