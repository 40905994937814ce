"""GPU parity of the b-form products birk_apply_b / birk_apply_bT (B^b = B^a - 1 w^T,
eq:xN=Birka+b) and of the endpoint row birk_endpoint (x^b = x^a + w^T V, eq:Prob-PNa)
against the FP64 oracle, through the C ABI.

References: the oracle's extended-precision b-form products at N <= 4096; at the
million-point size, exact antiderivatives of sparse Chebyshev series anchored at +1
(B^b is exact for polynomials of degree <= N), and O(N log N) rows of B^a for a g
supported on a few nodes (B^bT g = sum_i g_i (row_i(B^a) - w)).

Tolerances (relative to max |reference|): the products' own bars (1e-12 double, 2e-5
float, 1e-13 double-float); the correction is one subtraction per output in double.
The endpoint is one weighted sum of N + 1 terms in double: 1e-13 relative to
sum |w_k v_k| (about N eps / sqrt(N) for random signs, bounded by N eps = 1e-12 at
N = 4096 in the worst case; the tests use sizes where 1e-13 holds with margin).
"""

import numpy as np
import pytest

from oracle import birkhoff as bk
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dev, from_df32, host, rel_err, to_df32

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5, "df32": 1e-13}
SIZES = [3, 4, 9, 100, 257, 343, 1025, 1367, 2049, 3000, 4097]


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need a GPU"
    from paper_2509_01855_amd import birk
    return birk


def _prec(B, name):
    return {"f64": B.BIRK_F64, "f32": B.BIRK_F32, "df32": B.BIRK_DF32}[name]


def _to_dev(x, prec):
    import torch
    if prec == "f64":
        return dev(x, torch.float64)
    if prec == "f32":
        return dev(x, torch.float32)
    return dev(to_df32(x), torch.float32)


def _from_dev(t, prec):
    a = host(t)
    return from_df32(a) if prec == "df32" else a.astype(np.float64)


def _input_value(x, prec):
    """What the device holds for x in the plan's storage type, as double."""
    if prec == "f32":
        return x.astype(np.float32).astype(np.float64)
    if prec == "df32":
        return from_df32(to_df32(x))
    return x


def _run(B, Nn_list, nx_list, prec, x, transpose):
    import torch
    plan = B.birk_plan_create(Nn_list, nx_list, _prec(B, prec))
    v = _to_dev(x, prec)
    out = torch.empty_like(v)
    (B.birk_apply_bT if transpose else B.birk_apply_b)(plan, v, out)
    torch.cuda.synchronize()
    r = _from_dev(out, prec)
    plan.destroy()
    return r


@pytest.mark.parametrize("prec", ["f64", "f32", "df32"])
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("Nn", SIZES)
def test_bform_dense(B, Nn, transpose, prec):
    nx = 3 if Nn > 1000 else 5
    announce(f"b-form product Nn={Nn} nx={nx} transpose={transpose} prec={prec}")
    N = Nn - 1
    X = wl.random_vectors([21, Nn], (nx, Nn))[0]
    got = _run(B, [Nn], [nx], prec, X.ravel(), transpose).reshape(nx, Nn)
    ref = bk.apply_Bb_extended(N, _input_value(X, prec), transpose=bool(transpose))
    assert rel_err(got, ref) <= TOL[prec]
    if not transpose:
        assert np.all(got[:, N] == 0.0)          # B_j^b(1) = 0 exactly


def test_bform_batched_instances(B):
    Nn_list = [3, 256, 257, 1000, 4097, 65, 513]
    nx_list = [1, 6, 4, 5, 2, 12, 3]
    announce(f"b-form batched plan {Nn_list} {nx_list}")
    Xs = [wl.random_vectors([22, i], (nx, Nn))[0] for i, (Nn, nx) in enumerate(zip(Nn_list, nx_list))]
    flat = np.concatenate([x.ravel() for x in Xs])
    for transpose in (0, 1):
        got = _run(B, Nn_list, nx_list, "f64", flat, transpose)
        o = 0
        for X, Nn, nx in zip(Xs, Nn_list, nx_list):
            ref = bk.apply_Bb_extended(Nn - 1, X, transpose=bool(transpose))
            assert rel_err(got[o:o + nx * Nn].reshape(nx, Nn), ref) <= TOL["f64"]
            o += nx * Nn


@pytest.mark.parametrize("prec", ["f64", "df32"])
def test_bform_exact_sparse_modes_million(B, prec):
    """N_n = 2^20 + 1, n_x = 6 (the million-point launch configuration): v = 64 Chebyshev
    modes per component, exact B^b v from the antiderivatives anchored at +1."""
    Nn, nx = (1 << 20) + 1, 6
    N = Nn - 1
    announce(f"b-form sparse-mode apply Nn={Nn} nx={nx} prec={prec}")
    rows, refs = [], []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([23, c, Nn], N, count=64)
        rows.append(bk.sparse_mode_values(N, modes, alphas))
        refs.append(bk.sparse_mode_exact_b(N, modes, alphas))
    X = np.stack(rows)
    ref = np.stack(refs)
    if prec == "df32":
        # the reference of what the device holds: exact for the double input, plus the
        # first-order effect of the input's rounding, which is below the bar
        assert np.max(np.abs(_input_value(X, prec) - X)) <= 1e-14 * np.max(np.abs(X))
    got = _run(B, [Nn], [nx], prec, X.ravel(), 0).reshape(nx, Nn)
    assert rel_err(got, ref) <= TOL[prec]
    assert np.all(got[:, N] == 0.0)


def test_bform_T_sparse_rhs_million(B):
    """B^bT g for g supported on a few nodes of each component, N_n = 2^20 + 1, n_x = 6:
    sum_i g_i (row_i(B^a) - w) from O(N log N) oracle rows, compared at every output."""
    Nn, nx = (1 << 20) + 1, 6
    N = Nn - 1
    w = bk.ba_row(N, N)
    rng = np.random.default_rng(24)
    G = np.zeros((nx, Nn))
    refs = []
    row_cache = {}
    for c in range(nx):
        idx = sorted(set([0, N // 2, N] + [int(i) for i in rng.integers(0, Nn, 2)]))
        G[c, idx] = rng.standard_normal(len(idx))
        ref = np.zeros(Nn)
        for i in idx:
            if i not in row_cache:
                row_cache[i] = bk.ba_row(N, i)
            ref += G[c, i] * (row_cache[i] - w)
        refs.append(ref)
    announce(f"b-form sparse-g apply_bT Nn={Nn} nx={nx}")
    got = _run(B, [Nn], [nx], "f64", G.ravel(), 1).reshape(nx, Nn)
    assert rel_err(got, np.stack(refs)) <= TOL["f64"]


def test_bform_adjoint_large(B):
    """<B^b v, g> = <v, B^bT g> at N_n = 2^18 + 1 with B^b v exact (sparse modes)."""
    Nn = (1 << 18) + 1
    N = Nn - 1
    modes, alphas = wl.sparse_modes([25, Nn], N, count=32)
    v = bk.sparse_mode_values(N, modes, alphas)
    Bv = bk.sparse_mode_exact_b(N, modes, alphas)
    g = np.random.default_rng(26).standard_normal(Nn)
    announce(f"b-form adjoint Nn={Nn}")
    BTg = _run(B, [Nn], [1], "f64", g, 1)
    assert abs(float(Bv @ g) - float(v @ BTg)) <= 1e-11 * np.linalg.norm(Bv) * np.linalg.norm(g)


def _endpoint(B, Nn_list, nx_list, prec, x, xa, inplace=False):
    import torch
    plan = B.birk_plan_create(Nn_list, nx_list, _prec(B, prec))
    v = _to_dev(x, prec)
    xa_d = dev(xa, torch.float64)
    xb_d = xa_d if inplace else torch.full_like(xa_d, float("nan"))
    B.birk_endpoint(plan, xa_d, v, xb_d)
    torch.cuda.synchronize()
    r = host(xb_d).astype(np.float64)
    plan.destroy()
    return r


def _endpoint_bar(N, V, xa):
    """1e-13 relative to the size of the terms summed: |x^a| + sum |w_k v_k|."""
    w = bk.weights(N)
    return 1e-13 * (np.abs(xa) + np.abs(V) @ np.abs(w))


@pytest.mark.parametrize("prec", ["f64", "f32", "df32"])
@pytest.mark.parametrize("Nn", [3, 10, 257, 1366, 4097, 10001])
def test_endpoint_dense(B, Nn, prec):
    nx = 4
    N = Nn - 1
    announce(f"endpoint Nn={Nn} nx={nx} prec={prec}")
    X = wl.random_vectors([27, Nn], (nx, Nn))[0]
    xa = np.random.default_rng(Nn).standard_normal(nx)
    got = _endpoint(B, [Nn], [nx], prec, X.ravel(), xa)
    Xd = _input_value(X, prec)
    ref = bk.endpoint_b(N, xa, Xd)
    print(f"  max abs err {np.max(np.abs(got - ref)):.3e}", flush=True)
    assert np.all(np.abs(got - ref) <= _endpoint_bar(N, Xd, xa))


def test_endpoint_million_exact_integral(B):
    """x^b - x^a = integral over [-1, 1] of the interpolant of v; for v a sparse
    Chebyshev series that integral is exact (the last entry of its antiderivative)."""
    Nn, nx = (1 << 20) + 1, 6
    N = Nn - 1
    rows, ints = [], []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([28, c, Nn], N, count=64)
        rows.append(bk.sparse_mode_values(N, modes, alphas))
        ints.append(bk.sparse_mode_exact(N, modes, alphas)[N])
    X = np.stack(rows)
    xa = np.random.default_rng(29).standard_normal(nx)
    announce(f"endpoint sparse modes Nn={Nn} nx={nx}")
    got = _endpoint(B, [Nn], [nx], "f64", X.ravel(), xa)
    ref = xa + np.array(ints)
    print(f"  max abs err {np.max(np.abs(got - ref)):.3e}", flush=True)
    assert np.all(np.abs(got - ref) <= _endpoint_bar(N, X, xa))


def test_endpoint_batched_inplace(B):
    """Several instances in one plan, xb written over xa; the order of the entries is
    instance by instance, component by component."""
    Nn_list = [3, 300, (1 << 16) + 1, 4097, 65]
    nx_list = [2, 6, 3, 1, 12]
    Xs = [wl.random_vectors([30, i], (nx, Nn))[0] for i, (Nn, nx) in enumerate(zip(Nn_list, nx_list))]
    xa = np.random.default_rng(31).standard_normal(sum(nx_list))
    announce(f"endpoint batched {Nn_list} {nx_list}")
    got = _endpoint(B, Nn_list, nx_list, "f64", np.concatenate([x.ravel() for x in Xs]), xa, inplace=True)
    o = 0
    for X, Nn, nx in zip(Xs, Nn_list, nx_list):
        ref = bk.endpoint_b(Nn - 1, xa[o:o + nx], X)
        assert np.all(np.abs(got[o:o + nx] - ref) <= _endpoint_bar(Nn - 1, X, xa[o:o + nx]))
        o += nx


def test_endpoint_matches_last_node_of_trajectory(B):
    """x^a + B^a V and the endpoint row agree at node N (both on the GPU), and
    x^b + B^b V reproduces x^a + B^a V at every node (eq:xN=Birka+b)."""
    import torch
    Nn, nx = 4097, 3
    X = wl.random_vectors([32, Nn], (nx, Nn))[0]
    xa = np.random.default_rng(33).standard_normal(nx)
    announce("endpoint vs trajectory")
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    v = dev(X.ravel(), torch.float64)
    ya, yb = torch.empty_like(v), torch.empty_like(v)
    xa_d = dev(xa, torch.float64)
    xb_d = torch.empty_like(xa_d)
    B.birk_apply(plan, v, ya)
    B.birk_apply_b(plan, v, yb)
    B.birk_endpoint(plan, xa_d, v, xb_d)
    torch.cuda.synchronize()
    Ya = xa[:, None] + host(ya).reshape(nx, Nn)
    Yb = host(xb_d)[:, None] + host(yb).reshape(nx, Nn)
    plan.destroy()
    scale = np.max(np.abs(Ya))
    assert np.max(np.abs(Ya[:, -1] - host(xb_d))) <= 1e-13 * scale
    assert np.max(np.abs(Ya - Yb)) <= 1e-12 * scale


def test_bform_graph_mode_and_repeat_calls(B):
    """Graph mode covers the B^a part: three calls per direction with new data in the
    same buffers (eager, record + replay, replay) equal a second, eager plan's results
    bit for bit, and the oracle where it is dense; then a smaller plan follows."""
    import torch
    s = torch.cuda.Stream()
    for Nn, nx in (((1 << 16) + 1, 6), (257, 2)):
        announce(f"b-form graphs Nn={Nn} nx={nx}")
        plan_g = B.birk_plan_create([Nn], [nx], B.BIRK_F64, s)
        plan_e = B.birk_plan_create([Nn], [nx], B.BIRK_F64, s)
        B.birk_plan_set_graphs(plan_g, True)
        v = torch.empty(Nn * nx, dtype=torch.float64, device="cuda")
        out_g = {tr: torch.empty_like(v) for tr in (0, 1)}
        out_e = torch.empty_like(v)
        for it in range(3):
            X = wl.random_vectors([34, Nn, it], (nx, Nn))[0]
            with torch.cuda.stream(s):
                v.copy_(torch.from_numpy(X.ravel()).to("cuda"))
                for tr in (0, 1):
                    fn = B.birk_apply_bT if tr else B.birk_apply_b
                    fn(plan_g, v, out_g[tr])
                    fn(plan_e, v, out_e)
                    s.synchronize()
                    got = host(out_g[tr]).reshape(nx, Nn)
                    assert np.array_equal(got, host(out_e).reshape(nx, Nn))
                    if Nn < 5000:
                        assert rel_err(got, bk.apply_Bb_extended(Nn - 1, X, transpose=bool(tr))) <= TOL["f64"]
        plan_g.destroy()
        plan_e.destroy()


def test_bform_more_components_than_one_grid_row(B):
    """72,000 components (12,000 instances of n_x = 6 at N_n = 3 and 5): the component
    loops of the correction and reduction kernels wrap around the 65,535 grid rows."""
    import torch
    Nn_list = [3] * 11000 + [5] * 1000
    nx = 6
    announce(f"b-form with {len(Nn_list) * nx} components")
    rng = np.random.default_rng(35)
    flat = rng.standard_normal(sum(Nn_list) * nx)
    xa = rng.standard_normal(len(Nn_list) * nx)
    plan = B.birk_plan_create(Nn_list, [nx] * len(Nn_list), B.BIRK_F64)
    v = dev(flat, torch.float64)
    outs = []
    for fn in (B.birk_apply_b, B.birk_apply_bT):
        out = torch.empty_like(v)
        fn(plan, v, out)
        outs.append(out)
    xa_d = dev(xa, torch.float64)
    xb_d = torch.empty_like(xa_d)
    B.birk_endpoint(plan, xa_d, v, xb_d)
    torch.cuda.synchronize()
    got_b, got_bt, got_xb = host(outs[0]), host(outs[1]), host(xb_d)
    plan.destroy()
    o = 0
    c = 0
    for Nn, count in ((3, 11000), (5, 1000)):
        Bb = bk.dense_Bb_quadrature(Nn - 1)
        w = bk.weights(Nn - 1)
        m = count * nx
        V = flat[o:o + m * Nn].reshape(m, Nn)
        assert np.max(np.abs(got_b[o:o + m * Nn].reshape(m, Nn) - V @ Bb.T)) <= 1e-13 * max(1.0, np.max(np.abs(V)))
        assert np.max(np.abs(got_bt[o:o + m * Nn].reshape(m, Nn) - V @ Bb)) <= 1e-13 * max(1.0, np.max(np.abs(V)))
        assert np.max(np.abs(got_xb[c:c + m] - (xa[c:c + m] + V @ w))) <= 1e-13 * max(1.0, np.max(np.abs(V)))
        o += m * Nn
        c += m
