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
    """Plain FP32 vs fused BF16 on the same 20k x 20k market, fixed sweeps."""
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
                                        final_res=info.final_res)
        # time to tol 1e-6 (the configuration's tolerance)
        a, b, info = L.solve_market(U, Q, V, P, n, m, mk.sigma,
                                    **dict(kw, tol=1e-6, check_every=1))
        out[f"{path}_{compute}"]["sweeps_to_1e-6"] = info.sweeps
        out[f"{path}_{compute}"]["ms_to_1e-6"] = info.loop_ms
    p, f = out["plain_f32"], out["fused_bf16"]
    out["fused_over_plain"] = f["pair_evals_per_s"] / p["pair_evals_per_s"]
    return out


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else None


def run_serving(torch, L, count=512, rate_hz=200.0, aging_ms=0.0, lane_blocks=0):
    """The serving mix: `count` markets (N, M log-uniform in [1e3, 2e5], d = 32,
    sigma in {0.5, 1}, unit margins, tol 1e-6) submitted at Poisson(rate)
    arrival times to one continuous-batching server; factors are generated on
    the device before the clock starts."""
    reqs = workloads.serving_requests(count=count, rate_hz=rate_hz)
    log(f"serving: generating {count} markets on the device")
    tens = [workloads.device_request_factors(torch, r) for r in reqs]
    torch.cuda.synchronize()
    with L.Server(arena_bytes=16 << 30, max_active=256, lanes=3, chunk=4, aging_ms=aging_ms,
                  lane_blocks=lane_blocks) as srv:
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
            handles.append(srv.submit(*t, r.sigma, tol=1e-6, max_sweeps=200))
        log("serving: all submitted, waiting")
        for h in handles:
            srv.wait(h)
        st = srv.stats()
    t_end = max(h.t_done for h in handles)
    soj = [h.t_done - h.t_submit for h in handles]
    svc = [h.t_done - h.t_admit for h in handles]
    que = [h.t_admit - h.t_submit for h in handles]
    pe = sum(2.0 * h.N * h.M * h.info.sweeps for h in handles)
    ok = sum(1 for h in handles if h.status == 0)
    return {"requests": count, "rate_hz": rate_hz, "converged": ok,
            "sojourn_ms_p50": pct(soj, 50), "sojourn_ms_p99": pct(soj, 99),
            "service_ms_p50": pct(svc, 50), "service_ms_p99": pct(svc, 99),
            "queue_ms_p50": pct(que, 50), "queue_ms_p99": pct(que, 99),
            "makespan_ms": t_end - t0, "pair_evals_per_s": pe / ((t_end - t0) / 1e3),
            "mean_sweeps": float(np.mean([h.info.sweeps for h in handles])),
            "rounds": st["rounds"], "arena_peak_bytes": st["arena_peak"]}


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
                    help="run only the timing study's size and D sweeps (context)")
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
        print(json.dumps({"paper_sweeps": run_paper_sweeps(torch, L)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": run_serving(torch, L, aging_ms=args.aging_ms,
                                                 lane_blocks=args.lane_blocks)}), flush=True)
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
    if not args.no_c2:
        log("C2: plain FP32 vs fused BF16, 500 sweeps")
        line["c2_20k"] = run_c2(torch, L)
    if not args.no_serve:
        log("serving mix: 512 markets, Poisson 200/s")
        line["serving"] = run_serving(torch, L)
    if not args.no_cpu:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(mk)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
