"""Tile and split choice for the fused path, cached per market shape.

``ipfp_tune`` (the C ABI) times whole sweeps of a market for each candidate
workgroup height and reduction-split count and returns the fastest. This
module keeps the winners in a JSON file keyed by device architecture, compute
type, packed width and the power-of-two buckets of N and M, so that a shape is
tuned once per machine:

    opts = tuned(U, Q, V, P, n, m, sigma, compute="bf16")
    a, b, info = solve_market(U, Q, V, P, n, m, sigma, **opts)

The split counts are cached as multiples of the library's automatic counts
(``plan``), so they carry over to other shapes of the same bucket.

The cache file is ``$IPFP_TUNE_CACHE`` or ``~/.cache/ipfp/tune.json``.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

from . import _lib


def cache_path() -> str:
    return os.environ.get("IPFP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ipfp", "tune.json"))


def _bucket(x: int) -> int:
    return 1 << max(0, round(math.log2(max(1, x))))


def shape_key(arch: str, compute: str, d: int, N: int, M: int) -> str:
    kpad = (2 * d + 63) // 64 * 64 if compute == "fp8" else (2 * d + 31) // 32 * 32
    return f"{arch}|{compute}|k{kpad}|N{_bucket(N)}|M{_bucket(M)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _apply(choice: dict, N: int, M: int, d: int, compute: str) -> dict:
    """Solve options for a market of this shape from a cached choice: the
    split counts are stored as multiples of the automatic counts, so a shape
    that shares the bucket gets its own automatic count times the multiple."""
    from . import plan
    auto = plan(N, M, d, compute=compute, tile_rows=choice["tile_rows"])
    return {"tile_rows": choice["tile_rows"],
            "splits": max(1, min(256, round(choice["row_split_mult"] * auto["auto_splits_row"]))),
            "splits_col": max(1, min(256, round(choice["col_split_mult"] *
                                                auto["auto_splits_col"])))}


def tuned(U, Q, V, P, n, m, sigma, compute="bf16", path=None, refresh=False,
          stream=None, ctx=None) -> dict:
    """{"tile_rows", "splits", "splits_col"} for this market, from the cache or
    measured on the device (``ipfp_tune``) and then cached (as multiples of
    the automatic split counts)."""
    from . import Context, _check, _market_struct, _options, _stream_ptr, library, plan
    import torch
    path = path or cache_path()
    arch = torch.cuda.get_device_properties(U.device).gcnArchName.split(":")[0]
    N, d, M = U.shape[0], U.shape[1], V.shape[0]
    key = shape_key(arch, compute, d, N, M)
    table = _load(path)
    if not refresh and key in table:
        return _apply(table[key]["choice"], N, M, d, compute)
    mk = _market_struct(U, Q, V, P, n, m, sigma)
    opt = _options("fused", compute, 0.0, 4, 4, 0, 0, None, False, False)
    best = _lib.Options()
    ms = ctypes.c_double()
    ctx = ctx or Context.default(U.device.index or 0)
    _check(library().ipfp_tune(ctx.handle, ctypes.byref(mk), ctypes.byref(opt),
                               ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)),
           "ipfp_tune")
    auto = plan(N, M, d, compute=compute, tile_rows=best.tile_rows)
    choice = {"tile_rows": best.tile_rows,
              "row_split_mult": best.splits / auto["auto_splits_row"],
              "col_split_mult": best.splits_col / auto["auto_splits_col"]}
    table = _load(path)
    table[key] = {"choice": choice, "sweep_ms": ms.value,
                  "tuned_shape": [N, M, d], "splits": [best.splits, best.splits_col]}
    _store(path, table)
    return _apply(choice, N, M, d, compute)


# --- serving widths ----------------------------------------------------------

SERVING_CANDIDATES = {"chunk": (2, 4, 8), "lane_blocks": (1024, 2048, 4096), "lanes": (2, 3, 4)}


def serving_key(arch: str, compute: str) -> str:
    return f"serving|{arch}|{compute}"


def _run_mix(markets, arrivals, sigmas, compute, tol, max_sweeps, **server_opts):
    """One pass of a request mix through a fresh server; (p50, p99) of the
    sojourn time (ms) and the makespan (ms)."""
    import time

    import numpy as np

    from . import Server, clock_ms
    with Server(compute=compute, **server_opts) as srv:
        reqs = []
        t0 = clock_ms()
        for t, at, sg in zip(markets, arrivals, sigmas):
            due = t0 + 1e3 * at
            while clock_ms() < due:
                time.sleep(min(0.002, max(0.0, (due - clock_ms()) / 1e3)))
            reqs.append(srv.submit(*t, sg, tol=tol, max_sweeps=max_sweeps))
        for r in reqs:
            srv.wait(r)
    soj = np.array([r.t_done - r.t_submit for r in reqs])
    return (float(np.percentile(soj, 50)), float(np.percentile(soj, 99)),
            max(r.t_done for r in reqs) - t0)


def tune_serving(markets, arrivals, sigmas, compute="bf16", tol=1e-6, max_sweeps=200,
                 repeats=3, arena_bytes=16 << 30, path=None, log=None) -> dict:
    """Serving widths for a request mix: coordinate search over the server's
    sweeps per round (chunk), lane fill target (lane_blocks) and number of
    lanes, each candidate run `repeats` times on the same mix (markets: list of
    (U, Q, V, P, n, m) device tensors; arrivals in seconds from the first;
    sigmas). The score is the median over repeats of the p99 sojourn time.
    The winner is cached in the tuning JSON under the device's serving key."""
    import statistics

    import torch
    best = {"chunk": 4, "lane_blocks": 2048, "lanes": 3}
    trials = []

    def score(opts):
        runs = [_run_mix(markets, arrivals, sigmas, compute, tol, max_sweeps,
                         arena_bytes=arena_bytes, **opts) for _ in range(repeats)]
        p99 = statistics.median(r[1] for r in runs)
        trials.append({"options": dict(opts), "p50_ms": [r[0] for r in runs],
                       "p99_ms": [r[1] for r in runs], "makespan_ms": [r[2] for r in runs]})
        if log:
            log(f"serving tune {opts}: p99 {p99:.1f} ms")
        return p99

    best_s = score(best)
    for knob, values in SERVING_CANDIDATES.items():
        start = best[knob]
        for v in values:
            if v == start:
                continue
            cand = dict(best, **{knob: v})
            sc = score(cand)
            if sc < best_s:
                best, best_s = cand, sc
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = path or cache_path()
    table = _load(path)
    table[serving_key(arch, compute)] = {"choice": best, "p99_ms": best_s, "trials": trials}
    _store(path, table)
    return {"choice": best, "p99_ms": best_s, "trials": trials}


def tuned_serving(compute="bf16", path=None) -> dict:
    """The cached serving widths for this device (empty when never tuned)."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return dict(_load(path or cache_path()).get(serving_key(arch, compute), {}).get("choice", {}))
