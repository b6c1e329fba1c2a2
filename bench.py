#!/usr/bin/env python3
"""Throughput of the IPFP sweep on one MI355X, in pair-evaluations per second.

A step is one IPFP sweep over the whole market (both half-sweeps: the row pass
s = K v / 2 with the quadratic update of u, then the column pass with the new
u, plus the residual of the previous state), so one step evaluates every
kernel entry twice: pair-evals = 2 N M per sweep.

Default workload: the fused BF16 path on the N = M = 1,000,000, d = 64
market (factors N(0, 1/64), sigma = 1, n = 1, m uniform on 1..10), with the
factors resident in HBM before timing starts. The same JSON line also reports
the plain FP32 (materialised K) and fused BF16 paths on the 20,000 x 20,000,
d = 32 market at a fixed 500 sweeps, the solve's outputs on the default
market (top-k lists, welfare gradient, stable factors), the serving mix (512
markets arriving at 200/s, p50/p99 solve latency), the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample of the default
workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-c2] [--no-serve]
                    [--no-outputs]
    python bench.py --probes | --paper | --precision SIGMA | --serve-only | --pass c5:fp8
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = ("IPFP pair-evals/s, fused BF16 vs plain FP32 @ stated margin err; "
          "p99 solve ms")
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 MFMA
PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f32": 157.3}   # dense MFMA, per operand type
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
# HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters, scaled by what the counters read for a 1 GiB copy; valid
# only while the kernel source is unchanged (sha256 recorded beside it).
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_fused_pass_traffic.json")
FUSED_SRC = os.path.join(ROOT, "paper_2411_19214_amd", "csrc", "fused.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def factor_tensors(torch, mk):
    dev = torch.device("cuda", 0)
    return tuple(torch.from_numpy(t).to(dev) for t in (mk.U, mk.Q, mk.V, mk.P, mk.n, mk.m))


def code_hash(path):
    """sha256 of a source file's code: comments and blank space removed, so a
    comment-only edit keeps the hash and any code change alters it."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def measured_traffic(n_rows):
    """Counter-derived bytes per launch, or None once the kernel source has
    changed or for a workload other than the profiled N = M = 10^6 one."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        sha = code_hash(FUSED_SRC)
    except OSError:
        return None
    if rec.get("code_sha256") != sha or n_rows != rec.get("N"):
        return None
    return rec["traffic_bytes_per_launch"]


def run_fused(torch, L, mk, steps, warmup, compute="bf16", outputs=False):
    """Resident market: warm up, then time exactly `steps` sweeps."""
    U, Q, V, P, n, m = factor_tensors(torch, mk)
    h = L.Market(U, Q, V, P, n, m, mk.sigma, tol=0.0, max_sweeps=warmup + steps + 1,
                 check_every=1, compute=compute, time_passes=True)
    if warmup:
        h.run(warmup)
    _, _, before = h.read()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    h.run(steps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    _, _, after = h.read()
    h.run(1)                       # final residual of the last state (untimed)
    _, _, fin = h.read()
    outs = run_outputs(torch, L, h, mk, (U, Q, V, P)) if outputs else None
    h.close()
    launches = after.pass_launches - before.pass_launches
    pass_ms = after.pass_ms - before.pass_ms
    return dict(ms=ms, pass_ms=pass_ms, launches=launches, final_res=fin.final_res,
                setup_ms=before.setup_ms, fixups=fin.fixups, sweeps=fin.sweeps, outputs=outs)


def run_outputs(torch, L, h, mk, factors, reps=3, k=10):
    """The solve's outputs at the market's final state, each call timed on the
    host around a synchronous library call (scratch allocation included):
    top-k lists for every candidate (one fused pass with a top-k epilogue,
    4d flops per pair), the welfare gradient for the candidates' factors (one
    fused pass of three products, 12d flops per pair) and the stable factors
    of eq. 11 (O((N + M) d))."""
    N, M, d = mk.N, mk.M, mk.d

    def timed(fn):
        fn()                                   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    res = {}
    dt, _ = timed(lambda: h.topk(k, 0))
    tf = 4.0 * d * N * M / dt / 1e12
    res["topk"] = {"k": k, "rows": N, "call_ms": dt * 1e3, "pair_evals_per_s": N * M / dt,
                   "tflops": tf, "frac_of_bf16_peak": tf / PEAK_BF16_TFLOPS}
    dt, _ = timed(lambda: h.gradient(0))
    tf = 12.0 * d * N * M / dt / 1e12
    res["gradient"] = {"rows": N, "width": 2 * d, "call_ms": dt * 1e3,
                       "pair_evals_per_s": N * M / dt, "tflops": tf,
                       "frac_of_bf16_peak": tf / PEAK_BF16_TFLOPS}
    a, b, _ = h.read()
    U, Q, V, P = factors
    dt, _ = timed(lambda: L.stable_factors(U, Q, V, P, mk.sigma, a, b))
    res["stable_factors"] = {"rows": N + M, "width": 2 * d + 2, "call_ms": dt * 1e3}
    return res


def run_c2(torch, L, sweeps=500):
    """Plain FP32 vs fused BF16 on the same 20k x 20k market: throughput at a
    fixed number of sweeps, then accuracy against the exact surplus. Each
    path's own residual is measured against its own K (the plain path's FP32 K,
    the fused path's BF16-operand K), so both are also checked with
    ipfp_margin_residuals, which forms Phi in FP64 from the factors as given:
    the true margin residual (eq. 5) after k sweeps, for both paths. The
    comparison at equal accuracy is made at the smallest power of ten that
    both paths' true residuals reach."""
    mk = workloads.config_market(2)
    U, Q, V, P, n, m = factor_tensors(torch, mk)
    out = {}
    for path, compute in (("plain", "f32"), ("fused", "bf16")):
        kw = dict(path=path, compute=compute, tol=0.0, max_sweeps=sweeps, check_every=50,
                  use_graph=path == "fused")
        L.solve_market(U, Q, V, P, n, m, mk.sigma, **dict(kw, max_sweeps=5))  # warm
        torch.cuda.synchronize()
        a, b, info = L.solve_market(U, Q, V, P, n, m, mk.sigma, **kw)
        torch.cuda.synchronize()
        loop_s = info.loop_ms / 1e3
        # loop_ms covers sweeps + 1 row passes (final residual)
        pe = 2.0 * mk.N * mk.M * sweeps / loop_s
        out[f"{path}_{compute}"] = dict(pair_evals_per_s=pe, sweeps=info.sweeps,
                                        loop_ms=info.loop_ms, setup_ms=info.setup_ms,
                                        final_res_own_kernel=info.final_res,
                                        ms_per_sweep=info.loop_ms / (sweeps + 1))
        # time to tol 1e-6 against the path's own kernel (the configuration's tolerance)
        a, b, info = L.solve_market(U, Q, V, P, n, m, mk.sigma,
                                    **dict(kw, tol=1e-6, check_every=1))
        out[f"{path}_{compute}"]["sweeps_to_1e-6_own_kernel"] = info.sweeps
        out[f"{path}_{compute}"]["ms_to_1e-6_own_kernel"] = info.loop_ms
        # true margin residuals (row and column, FP64 surplus) after k sweeps
        traj = []
        with L.Market(U, Q, V, P, n, m, mk.sigma, tol=0.0, max_sweeps=60, path=path,
                      compute=compute) as h:
            done = 0
            for k in (1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20, 30, 40, 60):
                h.run(k - done)
                done = k
                a, b, _ = h.read()
                _, _, mr, mc = L.margin_residuals(U, Q, V, P, n, m, mk.sigma, a, b)
                traj.append((k, mr, mc))
        out[f"{path}_{compute}"]["true_residual_after_sweeps"] = [
            {"sweeps": k, "row": r, "col": c} for k, r, c in traj]
    p, f = out["plain_f32"], out["fused_bf16"]
    out["fused_over_plain"] = f["pair_evals_per_s"] / p["pair_evals_per_s"]

    def floor(rec):
        return min(max(t["row"], t["col"]) for t in rec["true_residual_after_sweeps"])

    def sweeps_to(rec, tol):
        for t in rec["true_residual_after_sweeps"]:
            if max(t["row"], t["col"]) < tol:
                return t["sweeps"]
        return None

    common = 10.0 ** np.ceil(np.log10(max(floor(p), floor(f)) * 1.0000001))
    eq = {"tolerance": common}
    for key, rec in (("plain_f32", p), ("fused_bf16", f)):
        k = sweeps_to(rec, common)
        eq[key] = {"true_residual_floor": floor(rec), "sweeps": k,
                   "ms": None if k is None else k * rec["ms_per_sweep"]}
    if eq["plain_f32"]["ms"] and eq["fused_bf16"]["ms"]:
        eq["fused_speedup"] = eq["plain_f32"]["ms"] / eq["fused_bf16"]["ms"]
    out["equal_true_margin_accuracy"] = eq
    return out


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else None


def run_serving(torch, L, count=512, rate_hz=200.0, aging_ms=0.0, lane_blocks=0,
                max_sweeps=200, chunk=4, lanes=3):
    """The serving mix: `count` markets (N, M log-uniform in [1e3, 2e5], d = 32,
    sigma in {0.5, 1}, unit margins, tol 1e-6) submitted at Poisson(rate)
    arrival times to one continuous-batching server; factors are generated on
    the device before the clock starts."""
    reqs = workloads.serving_requests(count=count, rate_hz=rate_hz)
    log(f"serving: generating {count} markets on the device")
    tens = [workloads.device_request_factors(torch, r) for r in reqs]
    torch.cuda.synchronize()
    with L.Server(arena_bytes=16 << 30, max_active=256, lanes=lanes, chunk=chunk,
                  aging_ms=aging_ms, lane_blocks=lane_blocks) as srv:
        # load the grouped kernels once, outside the measured window
        w = srv.submit(*workloads.device_request_factors(
            torch, workloads.Request(-1, 0.0, 1000, 1000, 32, 1.0, 1)), 1.0, tol=1e-6)
        srv.wait(w)
        log(f"serving: submitting at {rate_hz:.0f}/s")
        handles = []
        t0 = L.clock_ms()
        for r, t in zip(reqs, tens):
            due = t0 + 1e3 * r.arrival_s
            while True:
                now = L.clock_ms()
                if now >= due:
                    break
                time.sleep(min(0.002, (due - now) / 1e3))
            handles.append(srv.submit(*t, r.sigma, tol=1e-6, max_sweeps=max_sweeps))
        log("serving: all submitted, waiting")
        for h in handles:
            srv.wait(h)
        st = srv.stats()
    t_end = max(h.t_done for h in handles)
    soj = [h.t_done - h.t_submit for h in handles]
    svc = [h.t_done - h.t_admit for h in handles]
    que = [h.t_admit - h.t_submit for h in handles]
    pe = sum(2.0 * h.N * h.M * h.info.sweeps for h in handles)
    conv = [h for h in handles if h.status == 0]
    small = [h for h in handles if h.N * h.M <= 1e8]
    # requests that stopped at the sweep cap: shape, sigma and the residual
    # history tail (a steady geometric decay means slow IPFP convergence, a
    # plateau would mean a precision floor)
    unconverged = []
    for r, h in zip(reqs, handles):
        if h.status == 0:
            continue
        res = h.info.residuals
        unconverged.append({
            "N": h.N, "M": h.M, "sigma": r.sigma, "status": h.status,
            "sweeps": h.info.sweeps, "final_res": h.info.final_res,
            "res_at": {str(k): res[k - 1] for k in (25, 50, 100, 150, len(res))
                       if 0 < k <= len(res)},
            "decay_per_sweep_last_50": (res[-1] / res[-51]) ** (1 / 50) if len(res) > 51
            else None})
    return {"requests": count, "rate_hz": rate_hz, "max_sweeps": max_sweeps,
            "converged": len(conv),
            "sojourn_ms_p50": pct(soj, 50), "sojourn_ms_p99": pct(soj, 99),
            "service_ms_p50": pct(svc, 50), "service_ms_p99": pct(svc, 99),
            "queue_ms_p50": pct(que, 50), "queue_ms_p99": pct(que, 99),
            "converged_only": {
                "sojourn_ms_p50": pct([h.t_done - h.t_submit for h in conv], 50),
                "sojourn_ms_p99": pct([h.t_done - h.t_submit for h in conv], 99),
                "service_ms_p50": pct([h.t_done - h.t_admit for h in conv], 50),
                "service_ms_p99": pct([h.t_done - h.t_admit for h in conv], 99)},
            "small_requests_service_ms_p50": pct([h.t_done - h.t_admit for h in small], 50),
            "small_requests": len(small),
            "makespan_ms": t_end - t0, "pair_evals_per_s": pe / ((t_end - t0) / 1e3),
            "mean_sweeps": float(np.mean([h.info.sweeps for h in handles])),
            "rounds": st["rounds"], "arena_peak_bytes": st["arena_peak"],
            "unconverged": unconverged}


def run_paper_sweeps(torch, L, sweeps=100):
    """The timing study's shapes (Sec. 4.2): N = M from 1e2 to 1e6 with D = 50
    factors per side, and D from 10 to 100 at N = M = 1e5; U[0, 1/sqrt(D)]
    factors, n = 1, m = N / M, beta = 1, a fixed number of loops. Mean ms per
    loop (one sweep) for the fused BF16 path, and for the plain FP32 path where
    K fits. Context only: the paper's own times are on other hardware."""
    rows = []

    def one(N, D):
        mk = workloads.paper_uniform(N, N, D)
        t = factor_tensors(torch, mk)
        rec = {"N": N, "M": N, "D": D, "sweeps": sweeps}
        for path, compute in (("fused", "bf16"), ("plain", "f32")):
            if path == "plain" and N > 100_000:
                continue
            L.solve_market(*t, mk.sigma, max_sweeps=2, path=path, compute=compute)
            _, _, info = L.solve_market(*t, mk.sigma, max_sweeps=sweeps, path=path,
                                        compute=compute, use_graph=True, check_every=sweeps)
            rec[f"{path}_{compute}_ms_per_loop"] = info.loop_ms / (sweeps + 1)
            rec[f"{path}_{compute}_setup_ms"] = info.setup_ms
        log(f"paper sweep {rec}")
        rows.append(rec)

    for N in (100, 1000, 10_000, 100_000, 1_000_000):
        one(N, 50)
    for D in (10, 20, 100):
        one(100_000, D)
    return rows


def run_paper_batch_and_memory(torch, L, sweeps=20):
    """The timing study's other two axes (Sec. 4.2): rows per mini-batch B and
    memory against N. B is the output-row height of the fused kernel's
    workgroup tile (128, 256 or 512 rows stand in for the paper's 1, 10 and
    100: one workgroup processes its rows against the whole other side, as a
    mini-batch does), timed at N = M = 10^5 and 10^6, D = 50; the result does
    not depend on it (Z7). Memory: the library's scratch bytes for a market
    (ipfp_footprint) and the device memory a resident market actually holds
    (free memory before and after opening it), fused and plain, for N = M from
    10^2 to 10^6."""
    rows = []
    for N in (100_000, 1_000_000):
        mk = workloads.paper_uniform(N, N, 50)
        t = factor_tensors(torch, mk)
        for tr in (128, 256, 512):
            L.solve_market(*t, mk.sigma, max_sweeps=2, tile_rows=tr)
            _, _, info = L.solve_market(*t, mk.sigma, max_sweeps=sweeps, tile_rows=tr,
                                        use_graph=True, check_every=sweeps)
            rec = {"N": N, "M": N, "D": 50, "tile_rows": tr,
                   "ms_per_loop": info.loop_ms / (sweeps + 1)}
            log(f"paper batch sweep {rec}")
            rows.append(rec)
        del t
        torch.cuda.empty_cache()
    mem = []
    for N in (100, 1000, 10_000, 100_000, 1_000_000):
        mk = workloads.paper_uniform(N, N, 50)
        t = factor_tensors(torch, mk)
        rec = {"N": N, "M": N, "D": 50}
        for path, compute in (("fused", "bf16"), ("plain", "f32")):
            if path == "plain" and N > 100_000:
                rec["plain_f32_footprint_bytes"] = L.footprint(N, N, 50, path="plain")
                continue
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            with L.Market(*t, mk.sigma, max_sweeps=2, path=path, compute=compute) as h:
                torch.cuda.synchronize()
                free1 = torch.cuda.mem_get_info()[0]
                h.run(1)
            rec[f"{path}_{compute}_footprint_bytes"] = L.footprint(N, N, 50, path=path,
                                                                   compute=compute)
            rec[f"{path}_{compute}_device_bytes_held"] = free0 - free1
        log(f"paper memory {rec}")
        mem.append(rec)
        del t
        torch.cuda.empty_cache()
    return {"batch": rows, "memory": mem}


def run_precision(torch, L, sigma, sweeps=200, samples=1 << 14, chunk=10):
    """The precision-stress market at full size (N = 2 x 10^6, M = 2 x 10^5,
    d = 128, m_y = min(Zipf(1.5), 1000)) solved for `sweeps` sweeps with FP32,
    BF16 and FP8 operands. The FP32 solve is the reference trajectory: BF16 and
    FP8 are compared with it on every a_x and b_y and on mu at sampled pairs
    (ipfp_mu_pairs: FP64 surplus from the factors as given, times each solve's
    a, b), and each solve's true margin residuals (eq. 5, FP64 surplus) are
    reported."""
    mk = workloads.config_market(5, sigma=sigma)
    t = factor_tensors(torch, mk)
    g = torch.Generator(device="cuda")
    g.manual_seed(19214)
    xs = torch.randint(0, mk.N, (samples,), device="cuda", generator=g)
    ys = torch.randint(0, mk.M, (samples,), device="cuda", generator=g)
    res = {"N": mk.N, "M": mk.M, "d": mk.d, "sigma": sigma, "sweeps": sweeps,
           "samples": samples}
    sol = {}
    for compute in ("f32", "bf16", "fp8"):
        t0 = time.perf_counter()
        with L.Market(*t, mk.sigma, tol=0.0, max_sweeps=sweeps, compute=compute,
                      use_graph=True, check_every=chunk) as h:
            done = 0
            while not h.run(chunk):
                done += chunk
                log(f"precision sigma={sigma} {compute}: {done} sweeps")
            a, b, info = h.read()
        wall = time.perf_counter() - t0
        mu = L.mu_pairs(*t[:4], mk.sigma, a, b, xs, ys)
        _, _, mr, mc = L.margin_residuals(*t, mk.sigma, a, b)
        sol[compute] = (a, b, mu)
        res[compute] = {"sweeps": info.sweeps, "loop_ms": info.loop_ms,
                        "wall_s": wall, "own_residual": info.final_res,
                        "true_residual_row": mr, "true_residual_col": mc}
        log(f"precision sigma={sigma} {compute}: {res[compute]}")
    a0, b0, mu0 = sol["f32"]
    for compute in ("bf16", "fp8"):
        a, b, mu = sol[compute]
        ra = ((a - a0).abs() / a0).cpu().numpy()
        rb = ((b - b0).abs() / b0).cpu().numpy()
        rm = ((mu - mu0).abs() / mu0).cpu().numpy()
        res[compute]["vs_f32"] = {
            "a_rms": float(np.sqrt(np.mean(ra ** 2))), "a_max": float(ra.max()),
            "b_rms": float(np.sqrt(np.mean(rb ** 2))), "b_max": float(rb.max()),
            "mu_rms": float(np.sqrt(np.mean(rm ** 2))), "mu_max": float(rm.max())}
    return res


def run_pass(torch, L, spec, steps, warmup):
    """One configuration's fused reduction pass alone (for profiling and the
    per-type roofline): spec "c2|c3|c5:bf16|fp8|f32[:sigma]"; the resident
    market runs warmup + steps sweeps with every pass launch timed."""
    parts = spec.split(":")
    cfg, compute = int(parts[0].lstrip("c")), parts[1]
    sigma = float(parts[2]) if len(parts) > 2 else None
    mk = workloads.config_market(cfg, sigma=sigma)
    log(f"pass {spec}: N={mk.N} M={mk.M} d={mk.d}")
    r = run_fused(torch, L, mk, steps, warmup, compute=compute)
    launch_s = r["pass_ms"] / r["launches"] / 1e3
    # both half-sweeps do 4 d N M flops and N M exp2 per launch
    tf = 4.0 * mk.d * mk.N * mk.M / launch_s / 1e12
    return {"config": f"C{cfg}", "compute": compute, "N": mk.N, "M": mk.M, "d": mk.d,
            "sigma": mk.sigma, "launch_ms": launch_s * 1e3, "tflops": tf,
            "peak_tflops": PEAK_TFLOPS[compute], "frac": tf / PEAK_TFLOPS[compute],
            "exp2_per_s": mk.N * mk.M / launch_s,
            "pair_evals_per_s": 2.0 * mk.N * mk.M * steps / (r["ms"] / 1e3)}


def run_tune_serving(torch, L, count=128, repeats=3):
    """Serving widths (sweeps per round, lane fill target, lanes) tuned on the
    first `count` requests of the serving mix, each candidate run `repeats`
    times (paper_2411_19214_amd.tune.tune_serving)."""
    from paper_2411_19214_amd import tune
    reqs = workloads.serving_requests()[:count]
    tens = [workloads.device_request_factors(torch, r) for r in reqs]
    torch.cuda.synchronize()
    return tune.tune_serving(tens, [r.arrival_s for r in reqs], [r.sigma for r in reqs],
                             repeats=repeats, log=log)


def run_probes(torch, L):
    """The roofline probes (ipfp_probe): exp2 results/s, dense MFMA flop/s of
    the BF16, FP8 and FP32 instructions the fused passes use, the streaming
    HBM read rate, and the matrix stream at the passes' occupancy bare and
    with their exp2/FMA epilogue beside it."""
    out = {}
    for kind in ("exp2", "mfma_bf16", "mfma_fp8", "mfma_f32", "hbm_read", "mfma_bf16_2w",
                 "mfma_bf16_epi", "mfma_fp8_epi"):
        L.probe(kind)
        rate, ms = L.probe(kind)
        out[kind] = {"rate": rate, "ms": ms,
                     "unit": {"exp2": "exp2/s", "hbm_read": "B/s"}.get(kind, "flop/s")}
        log(f"probe {kind}: {rate:.4g} ({ms:.2f} ms)")
    return out


def cpu_baseline(mk, budget_s=15.0):
    """The oracle's mini-batch half-step (FP64 GEMM + exp + matvec) on row
    blocks of the default workload, timed on the host until ~budget_s."""
    from oracle import ipfp as O
    X = np.concatenate([mk.U, mk.Q], 1).astype(np.float64)
    Y = np.concatenate([mk.V, mk.P], 1).astype(np.float64)
    v = np.ones(mk.M)
    B = 64
    rows = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and rows < mk.N:
        O.half_step_rows(X[rows:rows + B], Y, v, mk.sigma)
        rows += B
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rows * mk.M / dt, "unit": "pair-evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{rows} rows x {mk.M} columns of one row half-step (mini-batch "
                      f"blocks of {B} rows: FP64 surplus GEMM, exp, matvec), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--size", type=int, default=1_000_000,
                    help="N = M of the default workload (1e6 unless testing)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-outputs", action="store_true",
                    help="skip timing top-k, gradient and stable factors")
    ap.add_argument("--aging-ms", type=float, default=0.0,
                    help="serving: waiting time worth a halving of N*M (0 = library default)")
    ap.add_argument("--lane-blocks", type=int, default=0,
                    help="serving: workgroups per pass a lane admits up to (0 = default)")
    ap.add_argument("--paper", action="store_true",
                    help="run only the timing study's size, D, batch and memory sweeps")
    ap.add_argument("--precision", type=float, default=None, metavar="SIGMA",
                    help="run only the full-size precision report of the stress market "
                         "at this sigma (FP32 reference vs BF16 and FP8, 200 sweeps)")
    ap.add_argument("--probes", action="store_true",
                    help="run only the roofline probes (exp2, MFMA, HBM read)")
    ap.add_argument("--tune-serving", action="store_true",
                    help="run only the serving-width tuner on the first 128 requests")
    ap.add_argument("--pass", dest="pass_spec", default=None, metavar="CFG:TYPE[:SIGMA]",
                    help="run only one configuration's fused pass, e.g. c5:fp8 (profiling)")
    ap.add_argument("--max-sweeps", type=int, default=200,
                    help="serving: sweep cap per request")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving mix (testing)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2411_19214_amd as L

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    L.library()
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.paper:
        print(json.dumps({"paper_sweeps": run_paper_sweeps(torch, L),
                          "paper_batch_memory": run_paper_batch_and_memory(torch, L)}),
              flush=True)
        return
    if args.precision is not None:
        print(json.dumps({"precision": run_precision(torch, L, args.precision)}), flush=True)
        return
    if args.probes:
        print(json.dumps({"probes": run_probes(torch, L)}), flush=True)
        return
    if args.tune_serving:
        print(json.dumps({"tune_serving": run_tune_serving(torch, L)}), flush=True)
        return
    if args.pass_spec:
        print(json.dumps({"pass": run_pass(torch, L, args.pass_spec, args.steps, args.warmup)}),
              flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": run_serving(torch, L, aging_ms=args.aging_ms,
                                                 lane_blocks=args.lane_blocks,
                                                 max_sweeps=args.max_sweeps)}), flush=True)
        return
    cfg = workloads.CONFIGS[3]
    log(f"generating C3 market N=M={args.size} d={cfg['d']}")
    mk = workloads.config_market(3, N=args.size, M=args.size)
    log("timing fused BF16")
    r = run_fused(torch, L, mk, args.steps, args.warmup, outputs=not args.no_outputs)
    N, M, d = mk.N, mk.M, mk.d
    value = 2.0 * N * M * args.steps / (r["ms"] / 1e3)
    avg_launch_s = r["pass_ms"] / r["launches"] / 1e3
    flops_per_launch = 4.0 * d * N * M        # 2 flops x 2d contraction per pair
    achieved_tflops = flops_per_launch / avg_launch_s / 1e12
    exp_rate = N * M / avg_launch_s
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"fused BF16 IPFP sweep, N=M={N}, d={d} per side "
                               f"(Phi=[U|Q][V|P]^T, K=2d={2 * d}), sigma=1, n=1, m~U{{1..10}}",
                   "N": N, "M": M, "d": d, "sigma": mk.sigma, "path": "fused",
                   "compute": "bf16 MFMA, fp32 accumulate/exp2, fp64 sums+updates"},
        "final_res": r["final_res"],
        "sweeps_done": r["sweeps"],
        "fixups": r["fixups"],
        "pack_ms": r["setup_ms"],
        "roofline": {"bound": "mfma", "achieved": achieved_tflops,
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_BF16_TFLOPS,
                     "traffic": measured_traffic(N),
                     "kernel": "k_fused_pass", "launch_ms": avg_launch_s * 1e3,
                     "flops_per_launch": flops_per_launch,
                     "exp2_per_s": exp_rate},
    }
    if r["outputs"] is not None:
        line["outputs"] = r["outputs"]
    # the ceiling of the pass's own instruction mix on this device: the BF16
    # matrix stream at the pass's occupancy with its exp2/FMA epilogue beside
    # it (ipfp_probe, about 0.1 s per launch; outside the timed region)
    L.probe("mfma_bf16_epi")
    mix_rate, _ = L.probe("mfma_bf16_epi")
    line["roofline"]["mix_ceiling"] = {
        "probe": "mfma_bf16_epi", "achieved": mix_rate / 1e12, "unit": "TFLOP/s",
        "frac_of_peak": mix_rate / 1e12 / PEAK_BF16_TFLOPS,
        "pass_frac_of_ceiling": achieved_tflops / (mix_rate / 1e12)}
    log(f"mix ceiling {mix_rate / 1e12:.0f} TFLOP/s; the pass reaches "
        f"{achieved_tflops / (mix_rate / 1e12):.3f} of it")
    if not args.no_c2:
        log("C2: plain FP32 vs fused BF16, 500 sweeps")
        line["c2_20k"] = run_c2(torch, L)
    if not args.no_serve:
        log("serving mix: 512 markets, Poisson 200/s")
        line["serving"] = run_serving(torch, L, aging_ms=args.aging_ms,
                                      lane_blocks=args.lane_blocks, max_sweeps=args.max_sweeps)
    if not args.no_cpu:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(mk)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
