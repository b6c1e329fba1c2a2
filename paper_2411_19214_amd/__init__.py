"""MI355X-native IPFP for Choo-Siow transferable-utility matching markets.

Thin Python binding over libipfp.so (include/ipfp.h). Torch tensors are used
for device memory and streams only; every step of the sweep runs in the
library's HIP kernels. Names follow the paper: rows x are candidates with
margins n, columns y are employers with margins m, sigma is the entropy scale
(the paper's beta), and the returned scalings are a = sqrt(mu_x0),
b = sqrt(mu_0y) (Sec. 3.2).

    a, b, info = solve_market(U, Q, V, P, n, m, sigma, tol=1e-6)

solves the market with surplus Phi = U V^T + Q P^T (eq. 8) by the fused
mini-batch path (Sec. 3.3); ``path="plain"`` materialises K = exp(Phi/2sigma)
instead (batch IPFP, eq. 7), and ``solve_market_phi`` takes a dense Phi.
"""
from __future__ import annotations

import ctypes
import dataclasses

from . import _lib

__all__ = ["IPFPError", "Context", "SolveInfo", "solve_market", "solve_market_phi",
           "Market", "mu_pairs", "pack_side", "footprint", "library", "Server", "Request",
           "clock_ms", "stable_factors", "margin_residuals", "probe", "plan"]

_DT = {"f64": _lib.F64, "f32": _lib.F32, "bf16": _lib.BF16, "fp8": _lib.FP8E4M3,
       "fp8e4m3": _lib.FP8E4M3}
_PATH = {"fused": _lib.PATH_FUSED, "plain": _lib.PATH_PLAIN}


def library():
    return _lib.load()


class IPFPError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = library().ipfp_strerror(code).decode()
        super().__init__(f"{what}: {msg} (code {code})" if what else msg)
        self.code = code


def _check(code: int, what: str) -> int:
    if code < 0:
        raise IPFPError(code, what)
    return code


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return _lib.F64
    if t.dtype == torch.float32:
        return _lib.F32
    if t.dtype == torch.bfloat16:
        return _lib.BF16
    if t.dtype == torch.float8_e4m3fn:
        return _lib.FP8E4M3
    raise TypeError(f"unsupported factor dtype {t.dtype}")


def _row_scales(scale, rows, name):
    """Device FP32 per-row scales of FP8 factors (checked here for shape and
    type; the library checks that each is a power of two)."""
    torch = _torch()
    if scale is None:
        raise ValueError(f"FP8 factors need {name} (FP32 per-row power-of-two scales)")
    _dev(scale, name)
    if scale.dtype != torch.float32 or scale.shape != (rows,) or not scale.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 vector of length {rows}")
    return scale.data_ptr()


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return t


class Context:
    """One library context per device (scratch budget accounting)."""

    _default = {}

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(library().ipfp_create(ctypes.byref(h), device, budget_bytes), "ipfp_create")
        self.handle = h
        self.device = device

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib._LIB is not None:
                _lib._LIB.ipfp_destroy(self.handle)
                self.handle = None
        except Exception:  # interpreter shutdown
            pass

    @classmethod
    def default(cls, device: int = 0) -> "Context":
        if device not in cls._default:
            cls._default[device] = cls(device)
        return cls._default[device]


@dataclasses.dataclass
class SolveInfo:
    status: int
    sweeps: int
    final_res: float
    residuals: list
    setup_ms: float
    loop_ms: float
    pass_ms: float
    pass_launches: int
    fixups: int

    @property
    def converged(self) -> bool:
        return self.status == _lib.OK


def _market_struct(U, Q, V, P, n, m, sigma, scale_x=None, scale_y=None):
    for t, nm in ((U, "U"), (Q, "Q"), (V, "V"), (P, "P"), (n, "n"), (m, "m")):
        _dev(t, nm)
    torch = _torch()
    if n.dtype != torch.float64 or m.dtype != torch.float64:
        raise TypeError("margins must be float64")
    if not (n.is_contiguous() and m.is_contiguous()):
        raise ValueError("margins must be contiguous")
    N, d = U.shape
    M = V.shape[0]
    if Q.shape != (N, d) or V.shape != (M, d) or P.shape != (M, d):
        raise ValueError("factor shapes must be U,Q: N x d and V,P: M x d")
    if n.shape != (N,) or m.shape != (M,):
        raise ValueError("margin lengths must be N and M")
    dt = _dtype_code(U)
    if any(_dtype_code(t) != dt for t in (Q, V, P)):
        raise TypeError("all factors must share one dtype")
    for t, nm in ((U, "U"), (Q, "Q"), (V, "V"), (P, "P")):
        if t.stride(1) != 1:
            raise ValueError(f"{nm} rows must be contiguous")
    if U.stride(0) != Q.stride(0) or V.stride(0) != P.stride(0):
        raise ValueError("U/Q and V/P must share a row stride")
    mk = _lib.Market()
    mk.N, mk.M, mk.d = N, M, d
    mk.in_dtype = dt
    mk.U, mk.Q, mk.V, mk.P = U.data_ptr(), Q.data_ptr(), V.data_ptr(), P.data_ptr()
    mk.ld_x, mk.ld_y = U.stride(0), V.stride(0)
    mk.n, mk.m = n.data_ptr(), m.data_ptr()
    mk.sigma = float(sigma)
    if dt == _lib.FP8E4M3:
        mk.scale_x = _row_scales(scale_x, N, "scale_x")
        mk.scale_y = _row_scales(scale_y, M, "scale_y")
    return mk


def _options(path, compute, tol, max_sweeps, check_every, splits, tile_rows, b0,
             use_graph, time_passes, splits_col=0):
    o = _lib.Options()
    library().ipfp_default_options(ctypes.byref(o))
    o.path = _PATH[path]
    o.compute = _DT[compute]
    o.tol = float(tol)
    o.max_sweeps = int(max_sweeps)
    o.check_every = int(check_every)
    o.splits = int(splits)
    o.splits_col = int(splits_col)
    o.tile_rows = int(tile_rows)
    o.b0 = b0.data_ptr() if b0 is not None else None
    o.use_graph = int(bool(use_graph))
    o.time_passes = int(bool(time_passes))
    return o


def _info(code, r, hist):
    n = min(r.n_res, len(hist))
    return SolveInfo(code, r.sweeps, r.final_res, [hist[i] for i in range(n)],
                     r.setup_ms, r.loop_ms, r.pass_ms, r.pass_launches, r.fixups)


def solve_market(U, Q, V, P, n, m, sigma, tol=0.0, max_sweeps=100, check_every=1,
                 path="fused", compute=None, splits=0, tile_rows=0, b0=None,
                 use_graph=False, time_passes=False, stream=None, ctx=None, no_alloc=False,
                 scale_x=None, scale_y=None, splits_col=0):
    """IPFP on the factor market Phi = U V^T + Q P^T; returns (a, b, info).
    ``compute`` is "bf16", "fp8" or "f32" on the fused path, "f32" or "f64"
    (storage of K) on the plain path. FP8 factors (torch.float8_e4m3fn codes)
    take per-row power-of-two scales ``scale_x`` (N) and ``scale_y`` (M).
    ``no_alloc=True`` calls ``ipfp_solve_market_noalloc`` (scratch from the
    library's fixed per-device array; only the outputs a, b are allocated
    here, by torch)."""
    torch = _torch()
    if compute is None:
        compute = "bf16" if path == "fused" else "f32"
    mk = _market_struct(U, Q, V, P, n, m, sigma, scale_x, scale_y)
    if b0 is not None:
        _dev(b0, "b0")
        if b0.dtype != torch.float64 or b0.shape != (mk.M,):
            raise ValueError("b0 must be float64 of length M")
    opt = _options(path, compute, tol, max_sweeps, check_every, splits, tile_rows, b0,
                   use_graph, time_passes, splits_col)
    a = torch.empty(mk.N, dtype=torch.float64, device=U.device)
    b = torch.empty(mk.M, dtype=torch.float64, device=U.device)
    hist = (ctypes.c_double * 4096)()
    r = _lib.Result()
    r.a, r.b = a.data_ptr(), b.data_ptr()
    r.res_hist = hist
    r.res_cap = 4096
    ctx = ctx or Context.default(U.device.index or 0)
    fn = library().ipfp_solve_market_noalloc if no_alloc else library().ipfp_solve_market
    code = _check(fn(ctx.handle, ctypes.byref(mk), ctypes.byref(opt), ctypes.byref(r),
                     _stream_ptr(stream)),
                  "ipfp_solve_market_noalloc" if no_alloc else "ipfp_solve_market")
    return a, b, _info(code, r, hist)


def solve_market_phi(Phi, n, m, sigma, tol=0.0, max_sweeps=100, check_every=1,
                     compute="f32", b0=None, use_graph=False, time_passes=False,
                     stream=None, ctx=None):
    """Batch IPFP on a dense surplus Phi (N x M, float32 or float64)."""
    torch = _torch()
    _dev(Phi, "Phi")
    _dev(n, "n")
    _dev(m, "m")
    N, M = Phi.shape
    if Phi.stride(1) != 1:
        raise ValueError("Phi rows must be contiguous")
    if n.dtype != torch.float64 or m.dtype != torch.float64 or n.shape != (N,) or m.shape != (M,):
        raise ValueError("margins must be float64 of lengths N and M")
    opt = _options("plain", compute, tol, max_sweeps, check_every, 0, 0, b0, use_graph,
                   time_passes)
    a = torch.empty(N, dtype=torch.float64, device=Phi.device)
    b = torch.empty(M, dtype=torch.float64, device=Phi.device)
    hist = (ctypes.c_double * 4096)()
    r = _lib.Result()
    r.a, r.b = a.data_ptr(), b.data_ptr()
    r.res_hist = hist
    r.res_cap = 4096
    ctx = ctx or Context.default(Phi.device.index or 0)
    code = _check(library().ipfp_solve_market_phi(
        ctx.handle, N, M, _dtype_code(Phi), Phi.data_ptr(), Phi.stride(0), n.data_ptr(),
        m.data_ptr(), float(sigma), ctypes.byref(opt), ctypes.byref(r),
        _stream_ptr(stream)), "ipfp_solve_market_phi")
    return a, b, _info(code, r, hist)


class Market:
    """A market kept resident on the device: open once, run sweeps in batches,
    read the scalings at any point (``ipfp_market_*``)."""

    def __init__(self, U, Q, V, P, n, m, sigma, tol=0.0, max_sweeps=100,
                 check_every=1, path="fused", compute=None, splits=0, tile_rows=0,
                 b0=None, use_graph=False, time_passes=False, stream=None, ctx=None,
                 scale_x=None, scale_y=None, splits_col=0):
        if compute is None:
            compute = "bf16" if path == "fused" else "f32"
        # the library reads these buffers until close()
        self._keep = (U, Q, V, P, n, m, b0, scale_x, scale_y)
        self._mk = _market_struct(U, Q, V, P, n, m, sigma, scale_x, scale_y)
        self._opt = _options(path, compute, tol, max_sweeps, check_every, splits,
                             tile_rows, b0, use_graph, time_passes, splits_col)
        self.ctx = ctx or Context.default(U.device.index or 0)
        self.device = U.device
        self.stream = stream
        h = ctypes.c_void_p()
        _check(library().ipfp_market_open(self.ctx.handle, ctypes.byref(self._mk),
                                          ctypes.byref(self._opt), ctypes.byref(h),
                                          _stream_ptr(stream)), "ipfp_market_open")
        self.handle = h
        self.done = False

    def run(self, sweeps: int) -> bool:
        done = ctypes.c_int(0)
        _check(library().ipfp_market_run(self.handle, int(sweeps), ctypes.byref(done),
                                         _stream_ptr(self.stream)), "ipfp_market_run")
        self.done = bool(done.value)
        return self.done

    def read(self):
        torch = _torch()
        a = torch.empty(self._mk.N, dtype=torch.float64, device=self.device)
        b = torch.empty(self._mk.M, dtype=torch.float64, device=self.device)
        hist = (ctypes.c_double * 4096)()
        r = _lib.Result()
        r.res_hist = hist
        r.res_cap = 4096
        code = _check(library().ipfp_market_read(self.handle, a.data_ptr(), b.data_ptr(),
                                                 ctypes.byref(r), _stream_ptr(self.stream)),
                      "ipfp_market_read")
        return a, b, _info(code, r, hist)

    def topk(self, k: int, side: int = 0):
        """Recommendation lists at the current state (``ipfp_market_topk``):
        (indices int32 rows x k, log mu float32 rows x k), best first; side 0
        ranks employers for every candidate, side 1 candidates for every
        employer."""
        torch = _torch()
        rows = self._mk.N if side == 0 else self._mk.M
        idx = torch.empty((rows, k), dtype=torch.int32, device=self.device)
        score = torch.empty((rows, k), dtype=torch.float32, device=self.device)
        _check(library().ipfp_market_topk(self.handle, int(side), int(k), idx.data_ptr(),
                                          score.data_ptr(), _stream_ptr(self.stream)),
               "ipfp_market_topk")
        return idx, score

    def gradient(self, side: int = 0):
        """dW/d[U|Q] (side 0, N x 2d) or dW/d[V|P] (side 1, M x 2d) at the
        current state, FP64 (``ipfp_market_gradient``)."""
        torch = _torch()
        rows = self._mk.N if side == 0 else self._mk.M
        w = 2 * self._mk.d
        g = torch.empty((rows, w), dtype=torch.float64, device=self.device)
        _check(library().ipfp_market_gradient(self.handle, int(side), g.data_ptr(), w,
                                              _stream_ptr(self.stream)),
               "ipfp_market_gradient")
        return g

    def close(self):
        if getattr(self, "handle", None):
            library().ipfp_market_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def mu_pairs(U, Q, V, P, sigma, a, b, xs, ys, stream=None, ctx=None, scale_x=None,
             scale_y=None):
    """mu at requested (x, y) pairs: exp(Phi_xy / 2 sigma) a_x b_y (eq. 4)."""
    torch = _torch()
    n_dummy = torch.ones(U.shape[0], dtype=torch.float64, device=U.device)
    m_dummy = torch.ones(V.shape[0], dtype=torch.float64, device=U.device)
    mk = _market_struct(U, Q, V, P, n_dummy, m_dummy, sigma, scale_x, scale_y)
    xs = xs.to(device=U.device, dtype=torch.int64).contiguous()
    ys = ys.to(device=U.device, dtype=torch.int64).contiguous()
    out = torch.empty(xs.numel(), dtype=torch.float64, device=U.device)
    ctx = ctx or Context.default(U.device.index or 0)
    _check(library().ipfp_mu_pairs(ctx.handle, ctypes.byref(mk), a.data_ptr(),
                                   b.data_ptr(), xs.data_ptr(), ys.data_ptr(), xs.numel(),
                                   out.data_ptr(), _stream_ptr(stream)), "ipfp_mu_pairs")
    return out


def margin_residuals(U, Q, V, P, n, m, sigma, a, b, stream=None, ctx=None, scale_x=None,
                     scale_y=None):
    """Residuals of eq. 5's margin equations for scalings (a, b) against the
    surplus formed in FP64 from the factors as given (``ipfp_margin_residuals``):
    (row_res (N), col_res (M), max row, max column)."""
    torch = _torch()
    mk = _market_struct(U, Q, V, P, n, m, sigma, scale_x, scale_y)
    rr = torch.empty(mk.N, dtype=torch.float64, device=U.device)
    cr = torch.empty(mk.M, dtype=torch.float64, device=U.device)
    mr, mc = ctypes.c_double(), ctypes.c_double()
    ctx = ctx or Context.default(U.device.index or 0)
    _check(library().ipfp_margin_residuals(ctx.handle, ctypes.byref(mk), a.data_ptr(),
                                           b.data_ptr(), rr.data_ptr(), cr.data_ptr(),
                                           ctypes.byref(mr), ctypes.byref(mc),
                                           _stream_ptr(stream)), "ipfp_margin_residuals")
    return rr, cr, mr.value, mc.value


def stable_factors(U, Q, V, P, sigma, a, b, stream=None, ctx=None, scale_x=None,
                   scale_y=None):
    """(psi, xi) of eq. 11: log mu_xy = <psi_x, xi_y> / (2 sigma), FP64."""
    torch = _torch()
    n_dummy = torch.ones(U.shape[0], dtype=torch.float64, device=U.device)
    m_dummy = torch.ones(V.shape[0], dtype=torch.float64, device=U.device)
    mk = _market_struct(U, Q, V, P, n_dummy, m_dummy, sigma, scale_x, scale_y)
    w = 2 * mk.d + 2
    psi = torch.empty((mk.N, w), dtype=torch.float64, device=U.device)
    xi = torch.empty((mk.M, w), dtype=torch.float64, device=U.device)
    ctx = ctx or Context.default(U.device.index or 0)
    _check(library().ipfp_stable_factors(ctx.handle, ctypes.byref(mk), a.data_ptr(),
                                         b.data_ptr(), psi.data_ptr(), w, xi.data_ptr(), w,
                                         _stream_ptr(stream)), "ipfp_stable_factors")
    return psi, xi


def pack_side(A, B, compute="bf16", sigma=0.0, stream=None, ctx=None, in_scale=None):
    """The fused path's packed operand of one side: (codes, scales or None),
    prescaled by sqrt(log2(e) / (2 sigma)) as the solver does (no prescale for
    sigma = 0). BF16 codes come back as int16 (bit patterns), FP8 codes as
    uint8, FP32 values as float32. FP8 input (float8_e4m3fn codes) takes its
    per-row scales from ``in_scale``."""
    torch = _torch()
    rows, d = A.shape
    kpad = ctypes.c_int64()
    ctx = ctx or Context.default(A.device.index or 0)
    lib = library()
    dt = _dtype_code(A)
    isc = _row_scales(in_scale, rows, "in_scale") if dt == _lib.FP8E4M3 else None
    _check(lib.ipfp_pack_side(ctx.handle, rows, d, dt, None, None, None, A.stride(0),
                              _DT[compute], float(sigma), None, None, ctypes.byref(kpad),
                              None),
           "ipfp_pack_side")
    scale = None
    if compute == "bf16":
        out = torch.empty((rows, kpad.value), dtype=torch.int16, device=A.device)
    elif compute == "f32":
        out = torch.empty((rows, kpad.value), dtype=torch.float32, device=A.device)
    else:
        out = torch.empty((rows, kpad.value), dtype=torch.uint8, device=A.device)
        scale = torch.empty(rows, dtype=torch.float32, device=A.device)
    _check(lib.ipfp_pack_side(ctx.handle, rows, d, dt, A.data_ptr(), B.data_ptr(), isc,
                              A.stride(0), _DT[compute], float(sigma), out.data_ptr(),
                              scale.data_ptr() if scale is not None else None,
                              ctypes.byref(kpad), _stream_ptr(stream)), "ipfp_pack_side")
    return out, scale


def plan(N, M, d, compute="bf16", splits=0, tile_rows=0, splits_col=0) -> dict:
    """The fused path's layout of an N x M market on the current device
    (``ipfp_plan_market``): packed width, workgroup height, automatic and
    chosen split counts and grid sizes of both half-sweeps, footprint."""
    mk = _lib.Market()
    mk.N, mk.M, mk.d = N, M, d
    mk.in_dtype = _lib.F32
    mk.U = mk.Q = mk.V = mk.P = 1
    mk.ld_x = mk.ld_y = d
    mk.n = mk.m = 1
    mk.sigma = 1.0
    opt = _options("fused", compute, 0.0, 1, 1, splits, tile_rows, None, False, False,
                   splits_col)
    out = _lib.Plan()
    _check(library().ipfp_plan_market(ctypes.byref(mk), ctypes.byref(opt), ctypes.byref(out)),
           "ipfp_plan_market")
    return {k: getattr(out, k) for k, _ in _lib.Plan._fields_}


def footprint(N, M, d, path="fused", compute=None, splits=0, tile_rows=0) -> int:
    """Scratch bytes a solve of an N x M market with d factors per side needs."""
    if compute is None:
        compute = "bf16" if path == "fused" else "f32"
    mk = _lib.Market()
    mk.N, mk.M, mk.d = N, M, d
    mk.in_dtype = _lib.F32
    mk.U = mk.Q = mk.V = mk.P = 1
    mk.ld_x = mk.ld_y = d
    mk.n = mk.m = 1
    mk.sigma = 1.0
    opt = _options(path, compute, 0.0, 1, 1, splits, tile_rows, None, False, False)
    out = ctypes.c_size_t()
    _check(library().ipfp_footprint(ctypes.byref(mk), ctypes.byref(opt), ctypes.byref(out)),
           "ipfp_footprint")
    return out.value


_PROBES = {"exp2": (_lib.PROBE_EXP2, 200000), "mfma_bf16": (_lib.PROBE_MFMA_BF16, 40000),
           "mfma_fp8": (_lib.PROBE_MFMA_FP8, 20000), "mfma_f32": (_lib.PROBE_MFMA_F32, 10000),
           "hbm_read": (_lib.PROBE_HBM_READ, 16 << 30),
           "mfma_bf16_2w": (_lib.PROBE_MFMA_BF16_2W, 1500000),
           "mfma_bf16_epi": (_lib.PROBE_MFMA_BF16_EPI, 1000000),
           "mfma_fp8_epi": (_lib.PROBE_MFMA_FP8_EPI, 500000)}


def probe(kind: str, work: int = 0, stream=None, ctx=None):
    """A roofline probe (``ipfp_probe``): (rate, ms). kind: "exp2" (results/s),
    "mfma_bf16" / "mfma_fp8" / "mfma_f32" (flop/s), "hbm_read" (bytes/s), and
    the matrix stream at the passes' occupancy, bare ("mfma_bf16_2w") or with
    the sum pass's exp2/FMA epilogue beside it ("mfma_bf16_epi",
    "mfma_fp8_epi"), in MFMA flop/s."""
    code, default = _PROBES[kind]
    rate, ms = ctypes.c_double(), ctypes.c_double()
    ctx = ctx or Context.default(0)
    _check(library().ipfp_probe(ctx.handle, code, int(work or default), ctypes.byref(rate),
                                ctypes.byref(ms), _stream_ptr(stream)), "ipfp_probe")
    return rate.value, ms.value


def clock_ms() -> float:
    """The host clock (CLOCK_MONOTONIC, ms) that request times are taken on."""
    return library().ipfp_clock_ms()


@dataclasses.dataclass
class Request:
    """A submitted market: its outputs (filled once finished) and times."""
    ticket: int
    a: object
    b: object
    N: int
    M: int
    status: int = _lib.EBUSY
    state: int = _lib.REQ_QUEUED
    lane: int = -1
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    info: SolveInfo = None

    @property
    def finished(self) -> bool:
        return self.state == _lib.REQ_FINISHED


class Server:
    """Continuous-batching server (``ipfp_server_*``): submit markets, poll or
    wait for them; the library's scheduler thread packs, groups and sweeps
    them on the device."""

    def __init__(self, arena_bytes=1 << 30, max_active=256, lanes=3, chunk=4,
                 compute="bf16", tile_rows=0, lane_pairs=(0.0, 0.0, 0.0), lane_blocks=0,
                 aging_ms=0.0, ctx=None, device=0):
        o = _lib.ServerOptions()
        library().ipfp_default_server_options(ctypes.byref(o))
        o.arena_bytes = int(arena_bytes)
        o.max_active = int(max_active)
        o.lanes = int(lanes)
        o.chunk = int(chunk)
        o.compute = _DT[compute]
        o.tile_rows = int(tile_rows)
        for k, v in enumerate(lane_pairs):
            o.lane_pairs[k] = float(v)
        o.lane_blocks = int(lane_blocks)
        o.aging_ms = float(aging_ms)
        self.compute = compute
        self.ctx = ctx or Context.default(device)
        h = ctypes.c_void_p()
        _check(library().ipfp_server_create(self.ctx.handle, ctypes.byref(o),
                                            ctypes.byref(h)), "ipfp_server_create")
        self.handle = h
        self._live = {}     # ticket -> (request, buffers the library uses)

    def submit(self, U, Q, V, P, n, m, sigma, tol=1e-6, max_sweeps=100, check_every=1,
               splits=0, b0=None, stream=None, scale_x=None, scale_y=None) -> Request:
        torch = _torch()
        mk = _market_struct(U, Q, V, P, n, m, sigma, scale_x, scale_y)
        opt = _options("fused", self.compute, tol, max_sweeps, check_every, splits, 0, b0,
                       False, False)
        a = torch.empty(mk.N, dtype=torch.float64, device=U.device)
        b = torch.empty(mk.M, dtype=torch.float64, device=U.device)
        hist = (ctypes.c_double * 4096)()
        r = _lib.Result()
        r.a, r.b = a.data_ptr(), b.data_ptr()
        r.res_hist = hist
        r.res_cap = 4096
        t = ctypes.c_uint64()
        _check(library().ipfp_submit(self.handle, ctypes.byref(mk), ctypes.byref(opt),
                                     ctypes.byref(r), ctypes.byref(t), _stream_ptr(stream)),
               "ipfp_submit")
        req = Request(t.value, a, b, mk.N, mk.M)
        self._live[t.value] = (req, (U, Q, V, P, n, m, b0, mk, opt, r, hist, scale_x,
                                     scale_y))
        return req

    def _update(self, req, code, info):
        req.state = info.state
        req.lane = info.lane
        req.t_submit, req.t_admit, req.t_done = info.t_submit, info.t_admit, info.t_done
        if info.state == _lib.REQ_FINISHED:
            _, keep = self._live.pop(req.ticket)
            req.status = code
            req.info = _info(code, keep[9], keep[10])

    def poll(self, req: Request) -> bool:
        if req.finished:
            return True
        info = _lib.RequestInfo()
        code = library().ipfp_poll(self.handle, req.ticket, ctypes.byref(info))
        if code == _lib.ENOTFOUND:
            raise IPFPError(code, "ipfp_poll")
        self._update(req, code, info)
        return req.finished

    def wait(self, req: Request, timeout_ms: float = -1.0) -> Request:
        if req.finished:
            return req
        info = _lib.RequestInfo()
        code = library().ipfp_wait(self.handle, req.ticket, float(timeout_ms),
                                   ctypes.byref(info))
        if code == _lib.ENOTFOUND:
            raise IPFPError(code, "ipfp_wait")
        self._update(req, code, info)
        return req

    def cancel(self, req: Request) -> None:
        if not req.finished:
            code = library().ipfp_cancel(self.handle, req.ticket)
            if code not in (_lib.OK, _lib.EINVAL):
                raise IPFPError(code, "ipfp_cancel")

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _check(library().ipfp_server_get_stats(self.handle, ctypes.byref(st)),
               "ipfp_server_get_stats")
        return {k: getattr(st, k) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            library().ipfp_server_destroy(self.handle)
            self.handle = None
            for req, _ in list(self._live.values()):
                req.state = _lib.REQ_FINISHED
                req.status = _lib.ECANCELLED
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
