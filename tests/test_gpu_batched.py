"""GPU parity of products over batches of uneven instances (the 512-instance LTI
workload and samples of it), through the C ABI.

A plan over many instances of different N_n and n_x covers all of them with one fixed
set of launches per product.  Inputs are sparse Chebyshev series per component, whose
exact B^a v the oracle gives from the closed-form antiderivatives (B^a integrates
polynomials of degree <= N exactly); the transpose is checked against single-instance
plans (bit for bit: batching must mix nothing) and through the adjoint identity.
"""

import numpy as np
import pytest

from oracle import birkhoff as bk
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dev, from_df32, host, rel_err, to_df32

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5, "df32": 1e-13}


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need a GPU"
    from paper_2509_01855_amd import birk
    return birk


def _inputs(insts, count, seed):
    xs, refs = [], []
    for i, ins in enumerate(insts):
        N = ins.N_n - 1
        X = np.empty((ins.n_x, ins.N_n))
        R = np.empty_like(X)
        for c in range(ins.n_x):
            modes, alphas = wl.sparse_modes([seed, i, c], N, count=count)
            X[c] = bk.sparse_mode_values(N, modes, alphas)
            R[c] = bk.sparse_mode_exact(N, modes, alphas)
        xs.append(X)
        refs.append(R)
    return xs, refs


def _product(B, Nn, nx, prec, flat, transpose):
    import torch
    plan = B.birk_plan_create(Nn, nx, prec)
    if prec == B.BIRK_DF32:
        v = dev(to_df32(flat[None, :])[0], torch.float32)
    else:
        v = dev(flat, torch.float64 if prec == B.BIRK_F64 else torch.float32)
    out = torch.empty_like(v)
    (B.birk_apply_T if transpose else B.birk_apply)(plan, v, out)
    torch.cuda.synchronize()
    r = host(out)
    plan.destroy()
    return from_df32(r[None, :])[0] if prec == B.BIRK_DF32 else r.astype(np.float64)


def _split(flat, insts):
    o = 0
    for ins in insts:
        n = ins.n_x * ins.N_n
        yield flat[o:o + n].reshape(ins.n_x, ins.N_n)
        o += n


@pytest.mark.parametrize("prec", ["f64", "f32", "df32"])
def test_batched_sample_apply(B, prec):
    insts = wl.batched_instances(count=24)
    Nn = [i.N_n for i in insts]
    nx = [i.n_x for i in insts]
    announce(f"batched sample apply prec={prec} sizes={Nn}")
    xs, refs = _inputs(insts, 16, 21)
    flat = np.concatenate([x.ravel() for x in xs])
    p = {"f64": B.BIRK_F64, "f32": B.BIRK_F32, "df32": B.BIRK_DF32}[prec]
    got = _product(B, Nn, nx, p, flat, 0)
    for g, r in zip(_split(got, insts), refs):
        assert rel_err(g, r) <= TOL[prec]


def test_batched_sample_transpose_matches_single(B):
    insts = wl.batched_instances(count=24)
    Nn = [i.N_n for i in insts]
    nx = [i.n_x for i in insts]
    announce("batched sample transpose vs single-instance plans")
    rng = np.random.default_rng(22)
    flat = rng.standard_normal(sum(a * b for a, b in zip(Nn, nx)))
    got = _product(B, Nn, nx, B.BIRK_F64, flat, 1)
    fwd = _product(B, Nn, nx, B.BIRK_F64, flat, 0)
    o = 0
    for k, ins in enumerate(insts):
        n = ins.n_x * ins.N_n
        if k % 4 == 0:
            one = _product(B, [ins.N_n], [ins.n_x], B.BIRK_F64, flat[o:o + n], 1)
            assert np.array_equal(one, got[o:o + n])
        # adjoint identity <B^a v, g> = <v, B^aT g> with v = g = this instance's block
        v = flat[o:o + n].reshape(ins.n_x, ins.N_n)
        lhs = float(np.sum(fwd[o:o + n].reshape(ins.n_x, ins.N_n) * v))
        rhs = float(np.sum(v * got[o:o + n].reshape(ins.n_x, ins.N_n)))
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(v) ** 2 * 10
        o += n


def test_batched_full_512(B):
    """All 512 instances (N_n log-uniform in [2^8, 2^16], n_x in {4, 6, 12}) in one plan,
    double and float, every output against the exact sparse-series result."""
    insts = wl.batched_instances(count=512)
    Nn = [i.N_n for i in insts]
    nx = [i.n_x for i in insts]
    announce(f"batched 512 instances, {sum(a * b for a, b in zip(Nn, nx))} values")
    xs, refs = _inputs(insts, 6, 23)
    flat = np.concatenate([x.ravel() for x in xs])
    for prec, p in (("f64", B.BIRK_F64), ("f32", B.BIRK_F32)):
        got = _product(B, Nn, nx, p, flat, 0)
        worst = 0.0
        for g, r in zip(_split(got, insts), refs):
            e = float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))
            worst = max(worst, e)
        announce(f"  {prec}: worst instance max-rel {worst:.3e}")
        assert worst <= TOL[prec]
