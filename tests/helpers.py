"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

import workloads


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def to_dev(torch, arr, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def market_tensors(torch, mk: workloads.Market, dtype=None):
    dt = dtype or torch.float32
    return (to_dev(torch, mk.U, dt), to_dev(torch, mk.Q, dt), to_dev(torch, mk.V, dt),
            to_dev(torch, mk.P, dt), to_dev(torch, mk.n), to_dev(torch, mk.m))


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)))


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
