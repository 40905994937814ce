"""GPU parity of birk_apply / birk_apply_T (FastBV and its transpose) against the FP64
oracle, through the C ABI.

References: the extended-precision (80-bit) evaluation of the oracle's modal
definition at N <= 4096, exact sparse-mode antiderivatives and O(N log N) rows at
larger N.

Tolerances (relative to max |reference|):
* double: 1e-12, the accuracy target for the FP64 path.  Two FFT-based DCT-I of
  length <= 2^21 accumulate roughly 2 * c * log2(M) * eps64 ~ 1e-14; 1e-12 leaves room.
* float:  2e-5.  The same bound with eps32 = 6e-8 and log2(M) <= 22 gives
  ~2 * 22 * 6e-8 ~ 3e-6 for power-of-two transforms; Bluestein's chirp products add
  a few ulps more per output.
"""

import numpy as np
import pytest

from oracle import birkhoff as bk
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dense_Ba, dev, host, rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}

# Bluestein lengths M = 2^ceil(log2(3N)): 342 and 1366 fill M exactly (3N = M - 1), 343
# and 1367 step to the next M (1366 is the largest in one LDS kernel, 1367 the smallest
# in the three fused passes).
SIZES = [3, 4, 5, 6, 9, 10, 17, 33, 100, 256, 257, 342, 343, 1000, 1025, 1366, 1367, 2049, 3000, 4097]


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need a GPU"
    from paper_2509_01855_amd import birk
    return birk


def _run(B, Nn_list, nx_list, prec, X, transpose):
    import torch
    plan = B.birk_plan_create(Nn_list, nx_list, prec)
    dt = torch.float64 if prec == B.BIRK_F64 else torch.float32
    v = dev(X, dt)
    out = torch.empty_like(v)
    (B.birk_apply_T if transpose else B.birk_apply)(plan, v, out)
    torch.cuda.synchronize()
    r = host(out).astype(np.float64)
    plan.destroy()
    return r


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("Nn", SIZES)
def test_product_dense(B, Nn, transpose, prec):
    nx = 3 if Nn > 1000 else 7
    announce(f"product Nn={Nn} nx={nx} transpose={transpose} prec={prec}")
    N = Nn - 1
    X = wl.random_vectors([1, Nn], (nx, Nn))[0]
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32
    got = _run(B, [Nn], [nx], p, X.ravel(), transpose).reshape(nx, Nn)
    ref = bk.apply_Ba_extended(N, X, transpose=bool(transpose))
    assert rel_err(got, ref) <= TOL[prec]


def test_product_batched_instances(B):
    Nn_list = [3, 256, 257, 1000, 4097, 65]
    nx_list = [1, 6, 4, 5, 2, 12]
    announce(f"batched plan {Nn_list} {nx_list}")
    Xs = [wl.random_vectors([2, i], (nx, Nn))[0] for i, (Nn, nx) in enumerate(zip(Nn_list, nx_list))]
    flat = np.concatenate([x.ravel() for x in Xs])
    for transpose in (0, 1):
        got = _run(B, Nn_list, nx_list, B.BIRK_F64, flat, transpose)
        o = 0
        for X, Nn, nx in zip(Xs, Nn_list, nx_list):
            ref = bk.apply_Ba_extended(Nn - 1, X, transpose=bool(transpose))
            assert rel_err(got[o:o + nx * Nn].reshape(nx, Nn), ref) <= TOL["f64"]
            o += nx * Nn


@pytest.mark.parametrize("Nn", [(1 << 16) + 1, (1 << 20) + 1, 65521, 100003])
def test_apply_exact_sparse_modes_large(B, Nn):
    """At sizes without a dense matrix: v = sum of 64 Chebyshev modes, exact B^a v from the
    closed-form antiderivatives (B^a is exact for polynomials of degree <= N)."""
    N = Nn - 1
    nx = 2
    announce(f"sparse-mode apply Nn={Nn}")
    rows, refs = [], []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([7, c, Nn], N, count=64)
        rows.append(bk.sparse_mode_values(N, modes, alphas))
        refs.append(bk.sparse_mode_exact(N, modes, alphas))
    X = np.stack(rows)
    got = _run(B, [Nn], [nx], B.BIRK_F64, X.ravel(), 0).reshape(nx, Nn)
    assert rel_err(got, np.stack(refs)) <= TOL["f64"]
    got32 = _run(B, [Nn], [nx], B.BIRK_F32, X.ravel(), 0).reshape(nx, Nn)
    assert rel_err(got32, np.stack(refs)) <= TOL["f32"]


@pytest.mark.parametrize("Nn", [(1 << 16) + 1, (1 << 20) + 1, 100003])
def test_apply_T_sparse_rhs_large(B, Nn):
    """B^aT g for g supported on a few nodes is a combination of rows of B^a, each of
    which the oracle computes in O(N log N); compared at every output."""
    N = Nn - 1
    rng = np.random.default_rng(Nn)
    idx = sorted(set([0, 1, N // 2, N - 1, N] + list(rng.integers(0, Nn, 5))))
    g = np.zeros(Nn)
    g[idx] = rng.standard_normal(len(idx))
    announce(f"sparse-g apply_T Nn={Nn}")
    ref = sum(g[i] * bk.ba_row(N, i) for i in idx)
    got = _run(B, [Nn], [1], B.BIRK_F64, g, 1)
    assert rel_err(got, ref) <= TOL["f64"]


@pytest.mark.parametrize("Nn", [(1 << 18) + 1, 12345])
def test_transpose_is_adjoint_large(B, Nn):
    """<B^a v, g> = <v, B^aT g> with random v, g (both products from the GPU), and the
    B^a v side pinned exactly through sparse modes."""
    N = Nn - 1
    modes, alphas = wl.sparse_modes([9, Nn], N, count=32)
    v = bk.sparse_mode_values(N, modes, alphas)
    Bv = bk.sparse_mode_exact(N, modes, alphas)
    g = np.random.default_rng(3).standard_normal(Nn)
    announce(f"adjoint Nn={Nn}")
    BTg = _run(B, [Nn], [1], B.BIRK_F64, g, 1)
    lhs = float(Bv @ g)
    rhs = float(v @ BTg)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Bv) * np.linalg.norm(g) * 10


@pytest.mark.parametrize("Nn", [3, 10, 257, 4097, (1 << 20) + 1])
def test_weights(B, Nn):
    announce(f"weights Nn={Nn}")
    plan = B.birk_plan_create([Nn], [1], B.BIRK_F64)
    w = B.birk_weights(plan, 0)
    plan.destroy()
    N = Nn - 1
    ref = bk.cc_weights_closed_form(N) if Nn <= 4097 else bk.ba_row(N, N)
    assert np.max(np.abs(w - ref)) <= 1e-15 * 50 + 1e-12 * np.max(np.abs(ref))
    assert abs(w.sum() - 2.0) <= 1e-12


@pytest.mark.parametrize("Nn", [513, 1025, 4097, (1 << 16) + 1])
def test_general_path_matches_fast_path(B, Nn, monkeypatch):
    """Power-of-two N normally takes the three-pass path; BIRK_FAST=0 at plan creation
    routes it through the general FFT path.  Both must agree with the oracle."""
    nx = 3
    X = wl.random_vectors([3, Nn], (nx, Nn))[0]
    announce(f"general vs fast Nn={Nn}")
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BIRK_FAST", flag)
        outs.append([_run(B, [Nn], [nx], B.BIRK_F64, X.ravel(), t) for t in (0, 1)])
    for t in (0, 1):
        assert rel_err(outs[0][t], outs[1][t]) <= 1e-12
    if Nn <= 4097:
        ref = bk.apply_Ba_extended(Nn - 1, X)
        assert rel_err(outs[1][0].reshape(nx, Nn), ref) <= TOL["f64"]
        assert rel_err(outs[0][0].reshape(nx, Nn), ref) <= TOL["f64"]


@pytest.mark.parametrize("Nn,prec", [((1 << 16) + 1, "f64"), ((1 << 20) + 1, "f64"), ((1 << 18) + 1, "f32")])
def test_autotuned_schedule_keeps_results(B, Nn, prec):
    """birk_plan_tune times every candidate tile schedule of the power-of-two path and
    keeps the fastest; products and transposes afterwards still match the exact
    sparse-mode series (B^a) and the untuned plan."""
    import torch
    N = Nn - 1
    nx = 2
    announce(f"autotune Nn={Nn} prec={prec}")
    rows, refs = [], []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([11, c, Nn], N, count=64)
        rows.append(bk.sparse_mode_values(N, modes, alphas))
        refs.append(bk.sparse_mode_exact(N, modes, alphas))
    X = np.stack(rows).ravel()
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = B.birk_plan_create([Nn], [nx], p)
    v = dev(X, dt)
    before = []
    for t in (0, 1):
        out = torch.empty_like(v)
        (B.birk_apply_T if t else B.birk_apply)(plan, v, out)
        torch.cuda.synchronize()
        before.append(host(out).astype(np.float64))
    report = B.birk_plan_tune(plan)
    print(report, flush=True)
    # 24 candidates and the default, plus 12 with narrow pass-A/C tiles for each split
    # whose L1 is 2^9 or 2^10
    s = (2 * (Nn - 1) - 1).bit_length()
    l1s = (s - (s + 1) // 2, (s + 1) // 2)
    assert "chosen" in report and report.count("us;") == 25 + 12 * sum(l in (9, 10) for l in l1s)
    after = []
    for t in (0, 1):
        out = torch.empty_like(v)
        (B.birk_apply_T if t else B.birk_apply)(plan, v, out)
        torch.cuda.synchronize()
        after.append(host(out).astype(np.float64))
    plan.destroy()
    assert rel_err(after[0].reshape(nx, Nn), np.stack(refs)) <= TOL[prec]
    for t in (0, 1):
        assert rel_err(after[t], before[t]) <= (1e-13 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec", ["f64", "df32"])
def test_multi_stream_schedule_is_bit_identical(B, prec, monkeypatch):
    """BIRK_FAST_STREAMS=2 or 3 runs a group's components in that many parts on as many
    streams; every component's kernels and sums are unchanged, so the products are bit for
    bit those of the one-stream schedule."""
    import torch
    from tests.gpu_util import to_df32
    Nn, nx = (1 << 16) + 1, 5
    X = wl.random_vectors([17, Nn], (nx * Nn,))[0]
    if prec == "f64":
        v = dev(X, torch.float64)
        p = B.BIRK_F64
    else:
        v = torch.from_numpy(to_df32(X[None, :])[0]).to("cuda")
        p = B.BIRK_DF32
    outs = []
    for st in ("1", "2", "3"):
        monkeypatch.setenv("BIRK_FAST_STREAMS", st)
        plan = B.birk_plan_create([Nn], [nx], p)
        for t in (0, 1):
            out = torch.empty_like(v)
            (B.birk_apply_T if t else B.birk_apply)(plan, v, out)
            torch.cuda.synchronize()
            outs.append(host(out))
        plan.destroy()
    for k in (2, 4):
        assert np.array_equal(outs[0], outs[k]) and np.array_equal(outs[1], outs[k + 1])


def test_autotune_double_float_plan(B):
    """The tuner times the double-float kernels of a DF32 plan and keeps 1e-13 parity."""
    import torch
    from tests.gpu_util import from_df32, to_df32
    Nn, nx = (1 << 15) + 1, 2
    N = Nn - 1
    rows, refs = [], []
    for c in range(nx):
        modes, alphas = wl.sparse_modes([13, c, Nn], N, count=32)
        rows.append(bk.sparse_mode_values(N, modes, alphas))
        refs.append(bk.sparse_mode_exact(N, modes, alphas))
    X = np.stack(rows).ravel()
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_DF32)
    report = B.birk_plan_tune(plan)
    assert "chosen" in report
    v = torch.from_numpy(to_df32(X[None, :])[0]).to("cuda")
    out = torch.empty_like(v)
    B.birk_apply(plan, v, out)
    torch.cuda.synchronize()
    got = from_df32(host(out)[None, :])[0]
    plan.destroy()
    assert rel_err(got.reshape(nx, Nn), np.stack(refs)) <= 1e-13


def test_autotune_without_power_of_two_groups(B):
    plan = B.birk_plan_create([1000], [3], B.BIRK_F64)
    assert "no power-of-two groups" in B.birk_plan_tune(plan)
    plan.destroy()


# ---------------------------------------------------------------- the timed configuration
# The benchmark times B^a and B^aT at N_n = 2^20 + 1, n_x = 6 after birk_plan_tune; the
# tuner picks among the schedules below (split 0, two rows per pass-B tile, one to three
# streams, four- or eight-column pass-A/C tiles; also four rows per pass-B tile on both
# splits, which other plans pick).  Each is checked here on the same
# inputs: a random dense v at 16 rows (96 outputs) through O(N log N) rows and columns of
# the oracle, and six exact series (Chebyshev modes for B^a, node-sparse right-hand
# sides for B^aT) at every output.
HEAD_NN, HEAD_NX = (1 << 20) + 1, 6
HEAD_SCHEDULES = [{"BIRK_FAST_SPLIT": "0", "BIRK_FAST_TB": "2", "BIRK_FAST_XCD": "1",
                   "BIRK_FAST_NARROW": nw, "BIRK_FAST_STREAMS": st}
                  for nw in ("0", "1") for st in ("1", "2", "3")] + \
                 [{"BIRK_FAST_SPLIT": sp, "BIRK_FAST_TB": "4", "BIRK_FAST_XCD": "1", "BIRK_FAST_NARROW": "1",
                   "BIRK_FAST_STREAMS": "1"} for sp in ("0", "1")] + ["tuned"]


@pytest.fixture(scope="module")
def head_refs():
    N = HEAD_NN - 1
    rng = np.random.default_rng(2020)
    Xd = wl.random_vectors([21, HEAD_NN], (HEAD_NX, HEAD_NN))[0]
    idx = np.unique(np.concatenate([[0, 1, 2, N // 2, N - 1, N], rng.integers(0, HEAD_NN, 10)]))
    rows = np.stack([bk.ba_row(N, int(i)) for i in idx])        # [s, j]
    cols = np.stack([bk.ba_col(N, int(j)) for j in idx])        # [s, i]
    ref_dense = Xd @ rows.T                                      # (B^a x_c)_i at i in idx
    ref_dense_T = Xd @ cols.T                                    # (B^aT x_c)_j at j in idx
    Xs, ref_s = [], []
    for c in range(HEAD_NX):
        modes, alphas = wl.sparse_modes([23, c, HEAD_NN], N, count=64)
        Xs.append(bk.sparse_mode_values(N, modes, alphas))
        ref_s.append(bk.sparse_mode_exact(N, modes, alphas))
    Gs, ref_sT = [], []
    for c in range(HEAD_NX):
        nodes = np.unique(np.concatenate([[0, N], rng.integers(0, HEAD_NN, 8)]))
        g = np.zeros(HEAD_NN)
        g[nodes] = rng.standard_normal(len(nodes))
        Gs.append(g)
        ref_sT.append(sum(g[i] * bk.ba_row(N, int(i)) for i in nodes))
    return dict(Xd=Xd, idx=idx, ref_dense=ref_dense, ref_dense_T=ref_dense_T, Xs=np.stack(Xs),
                ref_s=np.stack(ref_s), Gs=np.stack(Gs), ref_sT=np.stack(ref_sT))


@pytest.mark.parametrize("sched", HEAD_SCHEDULES, ids=lambda s: "tuned" if s == "tuned" else
                         f"split{s['BIRK_FAST_SPLIT']}-tb{s['BIRK_FAST_TB']}-narrow{s['BIRK_FAST_NARROW']}"
                         f"-streams{s['BIRK_FAST_STREAMS']}")
def test_timed_configuration_schedules(B, head_refs, sched, monkeypatch):
    import torch
    r = head_refs
    if sched == "tuned":
        plan = B.birk_plan_create([HEAD_NN], [HEAD_NX], B.BIRK_F64)
        rep = B.birk_plan_tune(plan)
        announce("timed configuration, tuned: " + rep.split(" chosen ")[-1].strip())
    else:
        for k, v in sched.items():
            monkeypatch.setenv(k, v)
        announce(f"timed configuration, schedule {sched}")
        plan = B.birk_plan_create([HEAD_NN], [HEAD_NX], B.BIRK_F64)

    def run(X, transpose):
        v = dev(X.ravel(), torch.float64)
        out = torch.empty_like(v)
        (B.birk_apply_T if transpose else B.birk_apply)(plan, v, out)
        torch.cuda.synchronize()
        return host(out).reshape(HEAD_NX, HEAD_NN)

    idx = r["idx"]
    assert rel_err(run(r["Xd"], 0)[:, idx], r["ref_dense"]) <= TOL["f64"]
    assert rel_err(run(r["Xd"], 1)[:, idx], r["ref_dense_T"]) <= TOL["f64"]
    assert rel_err(run(r["Xs"], 0), r["ref_s"]) <= TOL["f64"]
    assert rel_err(run(r["Gs"], 1), r["ref_sT"]) <= TOL["f64"]
    plan.destroy()


def test_autotuned_general_path_keeps_results(B):
    """birk_plan_tune on a batch of non-power-of-two sizes times every two-step split of each
    Bluestein length 2^13..2^18 and moves the filter spectra into the chosen order; the
    products afterwards match the exact sparse-mode series (B^a), node-sparse rows (B^aT)
    and the untuned plan."""
    import torch
    Nns = [2000, 5000, 9000, 12000, 30000, 60001]
    nx = 1
    announce(f"general-path autotune N_n {Nns}")
    X, refs, G, refsT = [], [], [], []
    rng = np.random.default_rng(404)
    for k, Nn in enumerate(Nns):
        N = Nn - 1
        modes, alphas = wl.sparse_modes([41, k, Nn], N, count=32)
        X.append(bk.sparse_mode_values(N, modes, alphas))
        refs.append(bk.sparse_mode_exact(N, modes, alphas))
        nodes = np.unique(np.concatenate([[0, N], rng.integers(0, Nn, 4)]))
        g = np.zeros(Nn)
        g[nodes] = rng.standard_normal(len(nodes))
        G.append(g)
        refsT.append(sum(g[i] * bk.ba_row(N, int(i)) for i in nodes))
    plan = B.birk_plan_create(Nns, [nx] * len(Nns), B.BIRK_F64)

    def run(vec, transpose):
        v = dev(np.concatenate(vec), torch.float64)
        out = torch.empty_like(v)
        (B.birk_apply_T if transpose else B.birk_apply)(plan, v, out)
        torch.cuda.synchronize()
        return host(out)

    before = [run(X, 0), run(G, 1)]
    report = B.birk_plan_tune(plan)
    print(report, flush=True)
    lines = [ln for ln in report.splitlines() if ln.startswith("general path M=2^")]
    assert len(lines) == 6 and all(" chosen [M1 2^" in ln for ln in lines), report
    after = [run(X, 0), run(G, 1)]
    plan.destroy()
    o = 0
    for k, Nn in enumerate(Nns):
        assert rel_err(after[0][o:o + Nn], refs[k]) <= TOL["f64"]
        assert rel_err(after[1][o:o + Nn], refsT[k]) <= TOL["f64"]
        o += Nn
    for t in (0, 1):
        assert rel_err(after[t], before[t]) <= 1e-13
