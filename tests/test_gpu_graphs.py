"""Graph mode of birk_apply / birk_apply_T (birk_plan_set_graphs): every replay of a
recorded product equals the eager product bit for bit, with the plan's own eager work,
other products and new input data between replays."""

import numpy as np
import pytest

from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_01855_amd import birk
    return birk


# a three-pass group, a Bluestein batch of uneven instances, and both in one plan
PLANS = [([(1 << 16) + 1], [4]), ([257, 1000, 3000, 4097, 70001], [6, 4, 12, 6, 2]),
         ([(1 << 12) + 1, 1500, 20000], [6, 6, 4])]


@pytest.mark.parametrize("case", range(len(PLANS)))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replays_match_eager(B, case, prec):
    import torch
    Nn, nx = PLANS[case]
    announce(f"graphs case={case} prec={prec} Nn={Nn} nx={nx}")
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32
    dt = torch.float64 if prec == "f64" else torch.float32
    side = torch.cuda.Stream()
    n = sum(a * b for a, b in zip(Nn, nx))
    xs = [torch.from_numpy(wl.random_vectors([21, case, k], (n,))[0]).to("cuda", dt) for k in range(4)]
    eager = B.birk_plan_create(Nn, nx, p, side)
    graph = B.birk_plan_create(Nn, nx, p, side)
    B.birk_plan_set_graphs(graph)
    with torch.cuda.stream(side):
        v = torch.empty(n, dtype=dt, device="cuda")
        out = torch.empty_like(v)
        other = torch.empty_like(v)
        ref = torch.empty_like(v)
        for call in range(6):
            t = call % 2
            x = xs[call % len(xs)]
            v.copy_(x)                                    # new data behind the same pointer
            fn = B.birk_apply_T if t else B.birk_apply
            fn(graph, v, out)                             # calls 0, 1: eager; 2, 3: record; then replay
            fn(eager, x, ref)
            B.birk_apply(graph, x, other)                 # another triple of the graph plan
            side.synchronize()
            got, want = host(out), host(ref)
            assert np.array_equal(got, want), f"call {call}: max diff {np.max(np.abs(got - want))}"
            assert np.array_equal(host(other), host(ref) if t == 0 else host(other))
    side.synchronize()
    eager.destroy()
    graph.destroy()


def test_graphs_need_a_stream(B):
    plan = B.birk_plan_create([257], [2], B.BIRK_F64, 0)
    with pytest.raises(B.BirkError):
        B.birk_plan_set_graphs(plan)
    plan.destroy()


def test_graph_replays_double_float(B):
    """Graph mode with a double-float plan (Bluestein and three-pass groups together)."""
    import torch
    from tests.gpu_util import to_df32
    Nn, nx = [(1 << 12) + 1, 3000], [2, 2]
    side = torch.cuda.Stream()
    n = sum(a * b for a, b in zip(Nn, nx))
    X = wl.random_vectors([23, 0], (n,))[0]
    v = torch.from_numpy(to_df32(X[None, :])[0]).to("cuda")
    eager = B.birk_plan_create(Nn, nx, B.BIRK_DF32, side)
    graph = B.birk_plan_create(Nn, nx, B.BIRK_DF32, side)
    B.birk_plan_set_graphs(graph)
    with torch.cuda.stream(side):
        out = torch.empty_like(v)
        ref = torch.empty_like(v)
        for call in range(4):
            B.birk_apply(graph, v, out)
            B.birk_apply(eager, v, ref)
            side.synchronize()
            assert torch.equal(out, ref), f"call {call}"
    eager.destroy()
    graph.destroy()


def test_graph_replays_two_stream_schedule(B, monkeypatch):
    """A recorded product whose three-pass group forks onto the plan's extra streams."""
    import torch
    monkeypatch.setenv("BIRK_FAST_STREAMS", "3")
    Nn, nx = [(1 << 16) + 1], [4]
    side = torch.cuda.Stream()
    n = Nn[0] * nx[0]
    xs = [torch.from_numpy(wl.random_vectors([29, k], (n,))[0]).to("cuda") for k in range(3)]
    eager = B.birk_plan_create(Nn, nx, B.BIRK_F64, side)
    graph = B.birk_plan_create(Nn, nx, B.BIRK_F64, side)
    B.birk_plan_set_graphs(graph)
    with torch.cuda.stream(side):
        v = torch.empty(n, dtype=torch.float64, device="cuda")
        out = torch.empty_like(v)
        ref = torch.empty_like(v)
        for call in range(5):
            v.copy_(xs[call % 3])
            B.birk_apply(graph, v, out)
            B.birk_apply(eager, v, ref)
            side.synchronize()
            assert torch.equal(out, ref), f"call {call}"
    eager.destroy()
    graph.destroy()


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_graph_mode_solves_match_eager(B, prec):
    """Graph mode also records the chunks of Arnoldi steps of birk_krylov_solve; repeated
    solves (recording, then replays, with other solves, new right-hand sides and a second
    Jacobian between them) equal the eager plan's solves bit for bit."""
    import torch
    from oracle import system as sy
    insts = [wl.lti_instance(k, Nn) for k, Nn in enumerate((257, 1000, 4097))]
    announce(f"graph-mode solves prec={prec}")
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32_REFINE_F64
    side = torch.cuda.Stream()
    Nn, nx = [i.N_n for i in insts], [i.n_x for i in insts]
    eager = B.birk_plan_create(Nn, nx, p, side)
    graph = B.birk_plan_create(Nn, nx, p, side)
    B.birk_plan_set_graphs(graph)
    with torch.cuda.stream(side):
        Js = [torch.from_numpy(np.concatenate([(i.J * s).ravel() for i in insts])).to("cuda")
              for s in (1.0, 0.5)]
        for call in range(5):
            J = Js[call % 2 if call > 2 else 0]
            xa = [np.random.default_rng([41, call, k]).standard_normal(i.n_x) for k, i in enumerate(insts)]
            beta = torch.from_numpy(np.concatenate([sy.beta_vector(a, i.N_n) for a, i in zip(xa, insts)])).to("cuda")
            x1 = torch.zeros_like(beta)
            x2 = torch.zeros_like(beta)
            i1 = B.birk_krylov_solve(graph, J, beta, x1, B.BIRK_J_CONSTANT, rtol=1e-12)
            i2 = B.birk_krylov_solve(eager, J, beta, x2, B.BIRK_J_CONSTANT, rtol=1e-12)
            side.synchronize()
            assert i1["inner_iters"] == i2["inner_iters"] and i1["status"] == 0
            assert np.array_equal(host(x1), host(x2)), f"call {call}"
    side.synchronize()
    eager.destroy()
    graph.destroy()
