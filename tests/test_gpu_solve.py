"""GPU parity of birk_krylov_solve against the FP64 oracle: dense LU at sizes where it
exists, exact ODE solutions at 2^16 + 1 and 2^20 + 1 nodes, Krylov counts against the
oracle's plain GMRES, and the error paths.

Tolerances: the system is well conditioned (kappa ~ 5 for these workloads, pinned in the
oracle tests), so a relative residual rho bounds the relative solution error by about
kappa * rho.  FP64 solves run to rtol 1e-13 and are held to 1e-12 (the accuracy target
of the double path); mixed solves (float Krylov inside double refinement) run to rtol
1e-11 and are held to 1e-10 (the target after refinement).  The collocation solution
meets the exact ODE solution to rounding at these N (spectral convergence), so the
closed-form pins use the same bars."""

import math

import numpy as np
import pytest
import scipy.linalg

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


def _solve(B, inst, beta, prec, **opts):
    import torch
    plan = B.birk_plan_create([inst.N_n], [inst.n_x], prec)
    jk = B.BIRK_J_PER_NODE if inst.per_node else B.BIRK_J_CONSTANT
    Jd = dev(inst.J.ravel(), torch.float64)
    bd = dev(beta, torch.float64)
    xd = torch.zeros_like(bd)
    info = B.birk_krylov_solve(plan, Jd, bd, xd, jk, raise_on_error=False, **opts)
    torch.cuda.synchronize()
    x = host(xd)
    plan.destroy()
    return x, info


@pytest.mark.parametrize("kind,Nn", [("lti", 3), ("lti", 17), ("lti", 256), ("lti", 257),
                                     ("kepler", 257), ("kepler", 1025), ("lti", 1000)])
@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_solve_vs_dense_lu(B, kind, Nn, prec):
    announce(f"solve {kind} Nn={Nn} prec={prec}")
    inst = wl.kepler_instance(2, Nn) if kind == "kepler" else wl.lti_instance(0, Nn)
    beta = sy.beta_vector(inst.x_a, Nn)
    A = sy.dense_A(Nn - 1, inst.J, dense_Ba(Nn - 1))
    ref = sy.solve_dense(A, beta)
    if prec == "f64":
        x, info = _solve(B, inst, beta, B.BIRK_F64, rtol=1e-13)
        tol = 1e-12
    else:
        x, info = _solve(B, inst, beta, B.BIRK_F32_REFINE_F64, rtol=1e-11)
        tol = 1e-10
    assert info["status"] == 0, info
    assert info["rel_resid"][0] <= (1e-13 if prec == "f64" else 1e-11)
    assert sy.rel_residual(lambda z: A @ z, beta, x) <= (1e-12 if prec == "f64" else 2e-11)
    assert rel_err(x, ref) <= tol


def test_iteration_count_matches_oracle_gmres(B):
    Nn = 257
    for inst in (wl.lti_instance(0, Nn), wl.kepler_instance(2, Nn)):
        beta = sy.beta_vector(inst.x_a, Nn)
        A = sy.dense_A(Nn - 1, inst.J, dense_Ba(Nn - 1))
        w = bk.weights(Nn - 1)
        _, its, _ = sy.gmres_right(lambda z: A @ z, lambda y: sy.precond_inverse(w, inst.J, y), beta,
                                   tol=1e-12)
        _, info = _solve(B, inst, beta, B.BIRK_F64, rtol=1e-12)
        announce(f"iterations oracle={its} gpu={info['inner_iters'][0]}")
        assert abs(info["inner_iters"][0] - its) <= 1


def test_lti_closed_form_65537(B):
    Nn = (1 << 16) + 1
    announce("LTI closed form Nn=65537")
    inst = wl.lti_instance(1, Nn)
    beta = sy.beta_vector(inst.x_a, Nn)
    tau = bk.cgl_nodes(Nn - 1)
    idx = np.unique(np.linspace(0, Nn - 1, 257).astype(int))
    Xe = np.stack([scipy.linalg.expm(inst.J * (tau[k] + 1.0)) @ inst.x_a for k in idx], axis=1)
    for prec, rtol, tol in ((B.BIRK_F64, 1e-13, 1e-12), (B.BIRK_F32_REFINE_F64, 1e-11, 1e-10)):
        x, info = _solve(B, inst, beta, prec, rtol=rtol)
        assert info["status"] == 0, info
        X = x.reshape(inst.n_x, Nn)[:, idx]
        assert rel_err(X, Xe) <= tol


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_kepler_time_shift_solution_million_points(B, prec):
    """Config with 2^20 + 1 nodes: the linearised two-body flow started at Z(-1) =
    (v, a)(t_0) has the exact solution Z(t) = (v(t), a(t)) (derivative of the orbit)."""
    Nn = (1 << 20) + 1
    announce(f"Kepler 2^20+1 prec={prec}")
    inst = wl.kepler_instance(2, Nn)
    ex = inst.extra
    Z = np.concatenate([ex["v"], ex["acc"]])
    beta = sy.beta_vector(Z[:, 0], Nn)
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32_REFINE_F64
    # kappa(A) ~ 720 for the Kepler systems (oracle pin), so the residual is taken two
    # orders below each bar
    rtol, tol = (1e-14, 1e-12) if prec == "f64" else (1e-12, 1e-10)
    x, info = _solve(B, inst, beta, p, rtol=rtol)
    assert info["status"] == 0, info
    assert info["rel_resid"][0] <= rtol
    assert rel_err(x.reshape(6, Nn), Z) <= tol


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_kepler_headline_residual_1e10(B, prec):
    """The timed configuration's tolerance: 2^20 + 1 nodes, Kepler Jacobian, solved to the
    relative residual 1e-10 (the time-shift right-hand side, whose solution is known);
    the error is held to the bound kappa * rtol with kappa(A) < 1000 (oracle pin)."""
    Nn = (1 << 20) + 1
    announce(f"Kepler 2^20+1 time-shift, rtol 1e-10, prec={prec}")
    inst = wl.kepler_instance(2, Nn)
    ex = inst.extra
    Z = np.concatenate([ex["v"], ex["acc"]])
    beta = sy.beta_vector(Z[:, 0], Nn)
    p = B.BIRK_F64 if prec == "f64" else B.BIRK_F32_REFINE_F64
    x, info = _solve(B, inst, beta, p, rtol=1e-10)
    assert info["status"] == 0, info
    assert info["rel_resid"][0] <= 1e-10
    assert rel_err(x.reshape(6, Nn), Z) <= 1000 * 1e-10


def test_error_paths(B):
    import torch
    Nn = 65
    inst = wl.kepler_instance(3, Nn)
    beta = sy.beta_vector(inst.x_a, Nn)
    # non-finite Jacobian
    bad = wl.Instance(N_n=Nn, n_x=6, J=inst.J.copy(), x_a=inst.x_a, per_node=True)
    bad.J[2, 3, 10] = np.nan
    _, info = _solve(B, bad, beta, B.BIRK_F64)
    assert info["status"] in (B.BIRK_ERR_NONFINITE, B.BIRK_ERR_SINGULAR), info
    # singular pivot: I - w_k J_k / 2 = 0 at node 7
    w = bk.weights(Nn - 1)
    sing = wl.Instance(N_n=Nn, n_x=6, J=inst.J.copy(), x_a=inst.x_a, per_node=True)
    sing.J[:, :, 7] = (2.0 / w[7]) * np.eye(6)
    _, info = _solve(B, sing, beta, B.BIRK_F64)
    assert info["status"] == B.BIRK_ERR_SINGULAR, info
    # iteration limit
    _, info = _solve(B, inst, beta, B.BIRK_F64, rtol=1e-15, max_iter=1)
    assert info["status"] == B.BIRK_ERR_NOCONV, info
    # MINRES (method 1) runs on double plans without a starting point
    _, info = _solve(B, inst, beta, B.BIRK_F64, method=1, rtol=1e-12)
    assert info["status"] == B.BIRK_OK
    _, info = _solve(B, inst, beta, B.BIRK_F32_REFINE_F64, method=1)
    assert info["status"] == B.BIRK_ERR_UNSUPPORTED
    _, info = _solve(B, inst, beta, B.BIRK_F64, method=1, use_x0=1)
    assert info["status"] == B.BIRK_ERR_UNSUPPORTED
    _, info = _solve(B, inst, beta, B.BIRK_F64, method=2)
    assert info["status"] == B.BIRK_ERR_ARG
    # plain float plans do not solve
    _, info = _solve(B, inst, beta, B.BIRK_F32)
    assert info["status"] == B.BIRK_ERR_UNSUPPORTED
    # restart lengths 1..31 (the multi-dot kernels hold 32 vectors: the basis and u)
    _, info = _solve(B, inst, beta, B.BIRK_F64, restart=32)
    assert info["status"] == B.BIRK_ERR_ARG
    x, info = _solve(B, inst, beta, B.BIRK_F64, restart=31, rtol=1e-12)
    assert info["status"] == B.BIRK_OK
