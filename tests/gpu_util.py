"""Shared helpers of the GPU parity tests (device placement, plan construction, caching
of dense oracle matrices)."""

import functools

import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype if dtype is not None else t.dtype)


def host(t):
    return t.detach().cpu().numpy()


@functools.lru_cache(maxsize=8)
def dense_Ba(N):
    from oracle import birkhoff as bk
    return bk.dense_Ba(N)


def rel_err(got, ref):
    """max |got - ref| / max |ref| (also printed with the normwise error for the log)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    e = float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))
    e2 = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    print(f"  max-rel {e:.3e}  norm-rel {e2:.3e}", flush=True)
    return e


def announce(msg):
    print(msg, flush=True)
