"""GPU parity of birk_precond (P y and P^{-1} y) and birk_fast_ax against the FP64 oracle.

Tolerance: double 1e-12 relative to max |reference| (the forward substitution and the
prefix sums are reordered into parallel scans; each output is a short chain of
well-conditioned operations).  float storage: 2e-6 (one float rounding of inputs and
outputs, arithmetic in double)."""

import numpy as np
import pytest

from oracle import birkhoff as bk
from oracle import system as sy
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dense_Ba, dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_01855_amd import birk
    return birk


def _inst(kind, Nn, nx, seed):
    if kind == "kepler":
        return wl.kepler_instance(seed, Nn)
    return wl.lti_instance(seed, Nn, nx)


def _J_dev(inst):
    import torch
    return dev(inst.J.ravel(), torch.float64)


# n_x <= 8 runs the wave-scan path (tiles of 1024 nodes: 1024 and 1025 sit on a tile
# edge), larger n_x the hierarchical scan (20000 nodes at n_x = 9 takes two levels); P y
# of every n_x from 1 to 8 runs its own compiled n_x.
CASES = [("lti", 3, 1), ("lti", 17, 4), ("lti", 256, 6), ("lti", 257, 12), ("kepler", 257, 6),
         ("lti", 1000, 5), ("lti", 1024, 6), ("lti", 1025, 8), ("lti", 3000, 7), ("kepler", 4097, 6),
         ("lti", 5000, 3), ("lti", 20000, 2), ("lti", 20000, 9), ("kepler", 70001, 6)]


@pytest.mark.parametrize("kind,Nn,nx", CASES)
@pytest.mark.parametrize("inverse", [0, 1])
def test_precond_f64(B, kind, Nn, nx, inverse):
    import torch
    announce(f"precond kind={kind} Nn={Nn} nx={nx} inverse={inverse}")
    inst = _inst(kind, Nn, nx, 5)
    nx = inst.n_x
    w = bk.weights(Nn - 1)
    y = wl.random_vectors([4, Nn], (nx * Nn,))[0]
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    jk = B.BIRK_J_PER_NODE if inst.per_node else B.BIRK_J_CONSTANT
    yd = dev(y, torch.float64)
    out = torch.empty_like(yd)
    B.birk_precond(plan, _J_dev(inst), yd, out, inverse, jk)
    torch.cuda.synchronize()
    got = host(out)
    plan.destroy()
    if inverse:
        ref = sy.precond_inverse(w, inst.J, y)
    else:
        ref = sy.precond_apply(w, inst.J, y)
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("Nn,nx", [(300, 17), (5000, 20)])
def test_precond_forward_many_states(B, Nn, nx):
    """P y for n_x above 16, where each component's passes form their own u_r from J and y
    (double plans up to n_x = 16 form u once for all components)."""
    import torch
    announce(f"precond forward Nn={Nn} nx={nx}")
    inst = _inst("lti", Nn, nx, 6)
    w = bk.weights(Nn - 1)
    y = wl.random_vectors([6, Nn], (nx * Nn,))[0]
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    yd = dev(y, torch.float64)
    out = torch.empty_like(yd)
    B.birk_precond(plan, _J_dev(inst), yd, out, 0, B.BIRK_J_CONSTANT)
    torch.cuda.synchronize()
    got = host(out)
    plan.destroy()
    assert rel_err(got, sy.precond_apply(w, inst.J, y)) <= 1e-12


@pytest.mark.parametrize("Nn", [(1 << 16) + 1, (1 << 20) + 1])
def test_precond_inverse_roundtrip_large(B, Nn):
    """P (P^{-1} y) = y with P applied by the oracle (vectorised prefix sums)."""
    import torch
    announce(f"precond roundtrip Nn={Nn}")
    inst = wl.kepler_instance(6, Nn)
    w = bk.weights(Nn - 1)
    y = wl.random_vectors([5, Nn], (6 * Nn,))[0]
    plan = B.birk_plan_create([Nn], [6], B.BIRK_F64)
    yd = dev(y, torch.float64)
    out = torch.empty_like(yd)
    B.birk_precond(plan, _J_dev(inst), yd, out, 1, B.BIRK_J_PER_NODE)
    torch.cuda.synchronize()
    xi = host(out)
    plan.destroy()
    assert rel_err(sy.precond_apply(w, inst.J, xi), y) <= 1e-11


@pytest.mark.parametrize("Nn,nx", [(3001, 9), (3001, 10), (20000, 11), (20000, 12), (70001, 12)])
def test_precond_inverse_per_node_large_nx(B, Nn, nx):
    """P^{-1} with a per-node Jacobian on the sixteen-lane hierarchical scan (n_x > 8): odd
    and even n_x (scalar and 16-byte row loads), one to three levels, against the
    oracle's block forward substitution."""
    import torch
    announce(f"precond inverse per-node J Nn={Nn} nx={nx}")
    rng = np.random.default_rng([nx, Nn])
    A = wl.lti_matrix(rng, nx)
    C = rng.standard_normal((nx, nx)) / np.sqrt(nx)
    tau = -np.cos(np.pi * np.arange(Nn) / (Nn - 1))
    J = A[:, :, None] + 0.25 * np.sin(3.0 * tau)[None, None, :] * C[:, :, None]
    w = bk.weights(Nn - 1)
    y = wl.random_vectors([7, Nn], (nx * Nn,))[0]
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    yd = dev(y, torch.float64)
    out = torch.empty_like(yd)
    B.birk_precond(plan, dev(J.ravel(), torch.float64), yd, out, 1, B.BIRK_J_PER_NODE)
    torch.cuda.synchronize()
    got = host(out)
    plan.destroy()
    assert rel_err(got, sy.precond_inverse(w, J, y)) <= 1e-12


@pytest.mark.parametrize("nx,jkind", [(7, "per_node"), (8, "per_node"), (8, "constant"), (5, "constant")])
def test_precond_inverse_many_tiles(B, nx, jkind):
    """P^{-1} on the wave-scan path with 293 tiles of 1024 nodes, so that the tile scan
    gives most of its threads two tiles and one thread a single tile (256 threads above
    n_x = 6, 512 at n_x = 5, where some threads hold none), against the oracle's forward
    substitution."""
    import torch
    Nn = 300001
    announce(f"precond inverse many tiles Nn={Nn} nx={nx} J={jkind}")
    rng = np.random.default_rng([nx, 293])
    if jkind == "per_node":
        J = rng.standard_normal((nx, nx, Nn)) / np.sqrt(nx) - 2.0 * np.eye(nx)[:, :, None]
        jk = B.BIRK_J_PER_NODE
    else:
        J = wl.lti_matrix(rng, nx)
        jk = B.BIRK_J_CONSTANT
    w = bk.weights(Nn - 1)
    y = rng.standard_normal(nx * Nn)
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    yd = dev(y, torch.float64)
    out = torch.empty_like(yd)
    B.birk_precond(plan, dev(J.ravel(), torch.float64), yd, out, 1, jk)
    torch.cuda.synchronize()
    got = host(out)
    plan.destroy()
    assert rel_err(got, sy.precond_inverse(w, J, y)) <= 1e-12


def test_precond_f32_storage(B):
    import torch
    Nn = 1025
    inst = wl.kepler_instance(8, Nn)
    w = bk.weights(Nn - 1)
    y = wl.random_vectors([6, Nn], (6 * Nn,))[0].astype(np.float32)
    plan = B.birk_plan_create([Nn], [6], B.BIRK_F32)
    yd = dev(y, torch.float32)
    for inverse in (0, 1):
        out = torch.empty_like(yd)
        B.birk_precond(plan, _J_dev(inst), yd, out, inverse, B.BIRK_J_PER_NODE)
        torch.cuda.synchronize()
        y64 = y.astype(np.float64)
        ref = sy.precond_inverse(w, inst.J, y64) if inverse else sy.precond_apply(w, inst.J, y64)
        assert rel_err(host(out), ref) <= 2e-6
    plan.destroy()


@pytest.mark.parametrize("kind,Nn,nx", [("lti", 256, 6), ("kepler", 513, 6), ("lti", 3000, 3)])
def test_fast_ax(B, kind, Nn, nx):
    import torch
    announce(f"fast_ax {kind} Nn={Nn}")
    inst = _inst(kind, Nn, nx, 9)
    nx = inst.n_x
    x = wl.random_vectors([8, Nn], (nx * Nn,))[0]
    plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64)
    jk = B.BIRK_J_PER_NODE if inst.per_node else B.BIRK_J_CONSTANT
    xd = dev(x, torch.float64)
    out = torch.empty_like(xd)
    B.birk_fast_ax(plan, _J_dev(inst), xd, out, jk)
    torch.cuda.synchronize()
    ref = sy.apply_A(dense_Ba(Nn - 1), inst.J, x)
    assert rel_err(host(out), ref) <= 1e-12
    plan.destroy()


@pytest.mark.parametrize("jkind", ["per_node", "constant"])
def test_precond_batched_instances(B, jkind):
    """P y and P^{-1} y over a batch of uneven instances in one plan (one set of launches
    for the whole batch), each instance against the oracle; 2^18 + 1 nodes give a
    component more than 256 tiles, so the scan of the tile sums takes two chunks."""
    import torch
    Nn_list = [3, 300, 1025, 4097, (1 << 18) + 1, 70001]
    nx_list = [1, 6, 4, 12, 3, 2]
    announce(f"precond batched {jkind}")
    rng = np.random.default_rng(70)
    Js, ys = [], []
    for Nn, nx in zip(Nn_list, nx_list):
        if jkind == "per_node":
            J = rng.standard_normal((nx, nx, Nn)) / np.sqrt(nx) - 2.0 * np.eye(nx)[:, :, None]
        else:
            J = rng.standard_normal((nx, nx)) / np.sqrt(nx) - 2.0 * np.eye(nx)
        Js.append(J)
        ys.append(rng.standard_normal(nx * Nn))
    jk = B.BIRK_J_PER_NODE if jkind == "per_node" else B.BIRK_J_CONSTANT
    plan = B.birk_plan_create(Nn_list, nx_list, B.BIRK_F64)
    Jd = dev(np.concatenate([J.ravel() for J in Js]), torch.float64)
    yd = dev(np.concatenate(ys), torch.float64)
    for inverse in (0, 1):
        out = torch.empty_like(yd)
        B.birk_precond(plan, Jd, yd, out, inverse, jk)
        torch.cuda.synchronize()
        got = host(out)
        o = 0
        for Nn, nx, J, y in zip(Nn_list, nx_list, Js, ys):
            w = bk.weights(Nn - 1)
            ref = sy.precond_inverse(w, J, y) if inverse else sy.precond_apply(w, J, y)
            assert rel_err(got[o:o + nx * Nn], ref) <= 1e-12
            o += nx * Nn
    plan.destroy()
