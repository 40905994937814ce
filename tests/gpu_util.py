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


def to_df32(x):
    """Double array -> interleaved double-float pairs (float32 [..., 2] flattened):
    hi = rn32(x), lo = rn32(x - hi)."""
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    lo = (x - hi.astype(np.float64)).astype(np.float32)
    return np.stack([hi, lo], axis=-1).reshape(*x.shape[:-1], 2 * x.shape[-1])


def from_df32(a):
    """Interleaved double-float pairs -> double (hi + lo)."""
    a = np.asarray(a, dtype=np.float32)
    pairs = a.reshape(*a.shape[:-1], a.shape[-1] // 2, 2)
    return pairs[..., 0].astype(np.float64) + pairs[..., 1].astype(np.float64)
