"""GPU parity of the compensated double-float (BIRK_DF32) products against the FP64
oracle, through the C ABI.

Every step of a BIRK_DF32 product (twiddles, butterflies, stencil, unpacking) runs in
double-float arithmetic: pairs (hi, lo) of floats with about 48 significant bits, the
error-free TwoSum / Fast2Sum / FMA-2Prod transformations and the double-word addition
and multiplication of Joldes, Muller and Popescu (2017), whose relative errors are
3u^2 and 5u^2 with u = 2^-24, i.e. about 1.1e-14 and 1.8e-14 per operation.  Two
transforms of depth log2(M) <= 20 keep the output error near 1e-14 of max |B^a v|;
the bar is 1e-13, the accuracy target of the compensated path.

The references take the double value hi + lo of the input pairs, so they measure the
product's error only.
"""

import numpy as np
import pytest

from oracle import birkhoff as bk
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dev, from_df32, host, rel_err, to_df32

pytestmark = pytest.mark.gpu

TOL_DF32 = 1e-13


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need a GPU"
    from paper_2509_01855_amd import birk
    return birk


def _run_df(B, Nn_list, nx_list, xdf, transpose):
    """Run a BIRK_DF32 product on interleaved pairs; returns the double value of the output."""
    import torch
    plan = B.birk_plan_create(Nn_list, nx_list, B.BIRK_DF32)
    v = dev(xdf, torch.float32)
    out = torch.empty_like(v)
    (B.birk_apply_T if transpose else B.birk_apply)(plan, v, out)
    torch.cuda.synchronize()
    r = from_df32(host(out))
    plan.destroy()
    return r


@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("Nn", [3, 4, 10, 33, 256, 257, 1000, 1025, 2049, 3000, 4097])
def test_df32_dense(B, Nn, transpose):
    """Sizes on every route: small and large Bluestein, power-of-two general path
    (N < 512) and the three-pass path (N = 1024, 2048, 4096)."""
    nx = 3
    announce(f"df32 product Nn={Nn} transpose={transpose}")
    X = wl.random_vectors([11, Nn], (nx, Nn))[0]
    xdf = to_df32(X)
    Xv = from_df32(xdf)
    got = _run_df(B, [Nn], [nx], xdf.ravel(), transpose).reshape(nx, Nn)
    ref = bk.apply_Ba_extended(Nn - 1, Xv, transpose=bool(transpose))
    assert rel_err(got, ref) <= TOL_DF32


def test_df32_beats_float(B):
    """The compensated path is at least 1e6 times closer to the oracle than plain float
    on the same input (the point of carrying the low word)."""
    import torch
    Nn, nx = 4097, 2
    X = wl.random_vectors([12, Nn], (nx, Nn))[0]
    xdf = to_df32(X)
    Xv = from_df32(xdf)
    ref = bk.apply_Ba_extended(Nn - 1, Xv)
    e_df = rel_err(_run_df(B, [Nn], [nx], xdf.ravel(), 0).reshape(nx, Nn), ref)
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F32)
    v = dev(Xv.ravel(), torch.float32)
    out = torch.empty_like(v)
    B.birk_apply(plan, v, out)
    torch.cuda.synchronize()
    e_32 = rel_err(host(out).astype(np.float64).reshape(nx, Nn), ref)
    plan.destroy()
    assert e_df * 1e6 <= e_32


def test_df32_many_rhs(B):
    """The many-RHS workload: 32 right-hand sides of N_n = 2^18 + 1, n_x = 6 in one plan
    (one group of 192 components, one launch per pass).  RHS 0 carries sparse Chebyshev
    series (exact B^a v from the closed-form antiderivatives); every RHS must equal the
    same product computed by a single-RHS plan bit for bit (batching mixes nothing)."""
    Nn, nx, R = (1 << 18) + 1, 6, 32
    N = Nn - 1
    announce(f"df32 many-RHS Nn={Nn} nx={nx} rhs={R}")
    rng = np.random.default_rng(4)
    X = rng.standard_normal((R * nx, Nn))
    refs = []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([4, c], N, count=64)
        X[c] = bk.sparse_mode_values(N, modes, alphas)
        refs.append(bk.sparse_mode_exact(N, modes, alphas))
    xdf = to_df32(X)
    got = _run_df(B, [Nn] * R, [nx] * R, xdf.ravel(), 0).reshape(R * nx, Nn)
    assert rel_err(got[:nx], np.stack(refs)) <= TOL_DF32
    for r in (0, 17, 31):
        one = _run_df(B, [Nn], [nx], xdf[r * nx:(r + 1) * nx].ravel(), 0).reshape(nx, Nn)
        assert np.array_equal(one, got[r * nx:(r + 1) * nx])


def test_df32_transpose_large(B):
    """B^aT g at N_n = 2^18 + 1 for g supported on a few nodes: a combination of rows of
    B^a that the oracle computes in O(N log N)."""
    Nn = (1 << 18) + 1
    N = Nn - 1
    rng = np.random.default_rng(Nn)
    idx = sorted(set([0, 1, N // 2, N - 1, N] + list(rng.integers(0, Nn, 5))))
    g = np.zeros(Nn)
    g[idx] = rng.standard_normal(len(idx))
    gdf = to_df32(g[None, :])[0]
    gv = from_df32(gdf[None, :])[0]
    announce(f"df32 sparse-g apply_T Nn={Nn}")
    ref = sum(gv[i] * bk.ba_row(N, i) for i in idx)
    got = _run_df(B, [Nn], [1], gdf, 1)
    assert rel_err(got, ref) <= TOL_DF32


def test_df32_rejected_where_unsupported(B):
    import torch
    plan = B.birk_plan_create([257], [2], B.BIRK_DF32)
    y = torch.zeros(2 * 2 * 257, dtype=torch.float32, device="cuda")
    J = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BirkError) as ei:
        B.birk_precond(plan, J, y, torch.empty_like(y), True, B.BIRK_J_CONSTANT)
    assert ei.value.status == B.BIRK_ERR_UNSUPPORTED
    plan.destroy()
