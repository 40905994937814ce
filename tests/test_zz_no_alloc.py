"""GPU test of birk_apply_noalloc (the allocation-free product): its output equals that of
birk_apply / birk_apply_T on the same plan (same kernels, workspace in the library's
fixed device array), on two calls in a row with the second plan smaller than the first,
across the three storage types; plans needing more workspace than the array holds are
rejected on the host."""

import numpy as np
import pytest

from oracle import birkhoff as bk
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dev, host, rel_err, to_df32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_01855_amd import birk
    return birk


def _both(B, plan, v, transpose):
    import torch
    ref = torch.empty_like(v)
    got = torch.empty_like(v)
    (B.birk_apply_T if transpose else B.birk_apply)(plan, v, ref)
    got.fill_(float("nan"))
    B.birk_apply_noalloc(plan, v, got, transpose)
    torch.cuda.synchronize()
    return host(got), host(ref)


def test_noalloc_matches_apply_two_calls_second_smaller(B):
    import torch
    cases = [((1 << 20) + 1, 6, "million-point, power of two (two work buffers)"),
             (1000, 3, "N_n = 1000 (Bluestein, three work buffers)")]
    for Nn, nx, what in cases:
        announce(f"noalloc {what}")
        X = wl.random_vectors([31, Nn], (nx, Nn))[0]
        plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
        v = dev(X.ravel(), torch.float64)
        for t in (0, 1):
            got, ref = _both(B, plan, v, t)
            assert np.array_equal(got, ref)
            if Nn <= 4097:
                exact = bk.apply_Ba_extended(Nn - 1, X, transpose=bool(t))
                assert rel_err(got.reshape(nx, Nn), exact) <= 1e-12
        plan.destroy()


def test_noalloc_batched_float_and_double_float(B):
    import torch
    Nn_list, nx_list = [257, 4097, 1025, 33], [6, 2, 4, 12]
    n = sum(a * b for a, b in zip(Nn_list, nx_list))
    X = wl.random_vectors([32, n], (n,))[0]
    announce("noalloc batched plan, float and double-float")
    p32 = B.birk_plan_create(Nn_list, nx_list, B.BIRK_F32)
    v = dev(X, torch.float32)
    for t in (0, 1):
        got, ref = _both(B, p32, v, t)
        assert np.array_equal(got, ref)
    p32.destroy()
    pdf = B.birk_plan_create(Nn_list, nx_list, B.BIRK_DF32)
    vdf = torch.from_numpy(to_df32(X[None, :])[0]).to("cuda")
    for t in (0, 1):
        got, ref = _both(B, pdf, vdf, t)
        assert np.array_equal(got, ref)
    pdf.destroy()


def test_noalloc_rejects_plans_beyond_the_array(B):
    import torch
    Nn = (1 << 21) + 1       # six double components need ~202 MB of workspace
    plan = B.birk_plan_create([Nn], [6], B.BIRK_F64)
    v = torch.zeros(6 * Nn, dtype=torch.float64, device="cuda")
    out = torch.full_like(v, 7.0)
    with pytest.raises(B.BirkError) as ei:
        B.birk_apply_noalloc(plan, v, out, False)
    assert ei.value.status == B.BIRK_ERR_SIZE
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))      # nothing was enqueued
    B.birk_apply_noalloc(B.birk_plan_create([257], [6], B.BIRK_F64), v[:6 * 257], out[:6 * 257], True)
    torch.cuda.synchronize()
    plan.destroy()
