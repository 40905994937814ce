"""GPU parity of the Newton solve of the nonlinear IVP (birk_newton_ivp, eq:X-V=nonlin,
eq:Newton-ivp) and of the two-body model kernel (birk_two_body), through the C ABI.

References: the oracle's Newton iteration with dense linear solves at N = 200 (the same
iterate to rounding, the same step count within one); Kepler's closed-form orbit at
every size (the discrete solution is spectrally accurate over one period, so the
solution at the nodes must match it to ~1e-12 of the orbit size; the bars below leave
one to two orders of margin for the conditioning of the one-period flow); the oracle's
f and df/dx for the model kernel (same formulas, a few ulps).
"""

import ctypes

import numpy as np
import pytest

from oracle import newton as nw
from paper_2509_01855_amd import workloads as wl
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need a GPU"
    from paper_2509_01855_amd import birk
    return birk


def _solve(B, ivps, prec=None, **kw):
    import torch
    Nn_list = [v["exact"].shape[1] for v in ivps]
    plan = B.birk_plan_create(Nn_list, [6] * len(ivps), B.BIRK_F64 if prec is None else prec)
    X = dev(np.concatenate([v["guess"].ravel() for v in ivps]), torch.float64)
    xa = dev(np.concatenate([v["x_a"] for v in ivps]), torch.float64)
    scale = ivps[0]["scale"]
    info = B.birk_newton_ivp(plan, xa, X, mu=1.0, scale=scale, **kw)
    torch.cuda.synchronize()
    out = host(X)
    plan.destroy()
    res, o = [], 0
    for Nn in Nn_list:
        res.append(out[o:o + 6 * Nn].reshape(6, Nn))
        o += 6 * Nn
    print(f"  newton {info['newton_iters']} linear {info['linear_iters']} resid {info['rel_resid']}", flush=True)
    return res, info


def test_two_body_kernel_matches_oracle(B):
    import torch
    Nn_list = [257, 1000]
    rng = np.random.default_rng(50)
    Xs = []
    for Nn in Nn_list:
        X = rng.standard_normal((6, Nn))
        X[:3] += 1.5 * np.sign(X[:3])
        Xs.append(X)
    announce("two-body kernel")
    plan = B.birk_plan_create(Nn_list, [6, 6], B.BIRK_F64)
    Xd = dev(np.concatenate([x.ravel() for x in Xs]), torch.float64)
    F = torch.empty_like(Xd)
    J = torch.empty(sum(36 * n for n in Nn_list), dtype=torch.float64, device="cuda")
    B.birk_two_body(plan, Xd, F, J, mu=0.8, scale=2.5)
    torch.cuda.synchronize()
    Fh, Jh = host(F), host(J)
    plan.destroy()
    o = jo = 0
    for X, Nn in zip(Xs, Nn_list):
        refF = nw.two_body_rhs(X, 2.5, 0.8)
        refJ = nw.two_body_jacobian(X, 2.5, 0.8)
        assert np.max(np.abs(Fh[o:o + 6 * Nn].reshape(6, Nn) - refF)) <= 1e-14 * np.max(np.abs(refF))
        assert np.max(np.abs(Jh[jo:jo + 36 * Nn].reshape(6, 6, Nn) - refJ)) <= 1e-14 * np.max(np.abs(refJ))
        o += 6 * Nn
        jo += 36 * Nn


@pytest.mark.parametrize("e", [0.1, 0.2])
def test_newton_matches_oracle_and_kepler(B, e):
    N = 200
    ivp = wl.kepler_ivp(42, N + 1, e)
    announce(f"newton N={N} e={e}")
    Xo, its, _, _ = nw.newton_ivp(N, ivp["x_a"], ivp["guess"], ivp["scale"], ivp["mu"])
    (X,), info = _solve(B, [ivp])
    assert info["inst_status"] == [0]
    assert abs(info["newton_iters"][0] - its) <= 1
    assert np.max(np.abs(X - Xo)) <= 1e-12 * np.max(np.abs(Xo))
    assert np.max(np.abs(X - ivp["exact"])) <= 1e-11


def test_newton_million_point_orbit(B):
    """N_n = 2^20 + 1: one period of a seeded Kepler orbit from the circular guess."""
    Nn = (1 << 20) + 1
    ivp = wl.kepler_ivp(44, Nn, 0.15)
    announce(f"newton Nn={Nn} e=0.15")
    (X,), info = _solve(B, [ivp])
    assert info["inst_status"] == [0]
    assert info["newton_iters"][0] <= 12
    err = np.max(np.abs(X - ivp["exact"]))
    print(f"  max |X - Kepler| = {err:.3e}", flush=True)
    assert err <= 1e-10


def test_newton_batched_instances(B):
    sizes = [201, 513, 4097, 65537]
    ecc = [0.05, 0.2, 0.1, 0.15]
    ivps = [wl.kepler_ivp([45, i], Nn, e) for i, (Nn, e) in enumerate(zip(sizes, ecc))]
    announce(f"newton batched {sizes}")
    Xs, info = _solve(B, ivps)
    assert info["inst_status"] == [0] * len(sizes)
    for X, ivp in zip(Xs, ivps):
        assert np.max(np.abs(X - ivp["exact"])) <= 1e-10


def test_newton_line_search_from_poor_guess(B):
    """e = 0.3 from the circular orbit needs damped steps (as in the oracle pin)."""
    N = 120
    ivp = wl.kepler_ivp(43, N + 1, 0.3)
    announce("newton damped e=0.3")
    Xo, its, _, steps = nw.newton_ivp(N, ivp["x_a"], ivp["guess"], ivp["scale"], ivp["mu"])
    assert min(steps) < 1.0
    (X,), info = _solve(B, [ivp])
    assert info["inst_status"] == [0]
    assert np.max(np.abs(X - Xo)) <= 1e-11 * np.max(np.abs(Xo))


def test_newton_mixed_precision_linear_solves(B):
    Nn = 4097
    ivp = wl.kepler_ivp(46, Nn, 0.1)
    announce("newton with refinement plan")
    (X,), info = _solve(B, [ivp], prec=B.BIRK_F32_REFINE_F64)
    assert info["inst_status"] == [0]
    assert np.max(np.abs(X - ivp["exact"])) <= 1e-10


def test_newton_callback_model_equals_built_in(B):
    """A caller-supplied right-hand side (here the library's own two-body kernel called
    back through the C ABI) gives the built-in model's iterates bit for bit."""
    import torch
    Nn = 1025
    ivp = wl.kepler_ivp(47, Nn, 0.12)
    announce("newton callback model")
    (Xb,), ib = _solve(B, [ivp])
    plan = B.birk_plan_create([Nn], [6], B.BIRK_F64)
    calls = []

    def rhs(x, f, j, stream):
        calls.append(bool(j))
        return B._lib.birk_two_body(plan.handle, 1.0, ivp["scale"], ctypes.c_void_p(x),
                                    ctypes.c_void_p(f) if f else None, ctypes.c_void_p(j) if j else None)

    X = dev(ivp["guess"].ravel(), torch.float64)
    xa = dev(ivp["x_a"], torch.float64)
    info = B.birk_newton_ivp(plan, xa, X, rhs=rhs)
    torch.cuda.synchronize()
    Xc = host(X).reshape(6, Nn)
    plan.destroy()
    assert info["newton_iters"] == ib["newton_iters"]
    assert any(calls) and not all(calls)
    assert np.array_equal(Xc, Xb)


def test_newton_status_paths(B):
    import torch
    Nn = 257
    ivp = wl.kepler_ivp(48, Nn, 0.2)
    announce("newton status paths")
    # one step only: NOCONV, with the first damped or full step applied
    (X1,), info = _solve(B, [ivp], raise_on_error=False, max_newton=1)
    assert info["status"] == B.BIRK_ERR_NOCONV and info["newton_iters"] == [1]
    assert np.max(np.abs(X1 - ivp["exact"])) < np.max(np.abs(ivp["guess"] - ivp["exact"]))
    # the callback's own error status ends the solve
    plan = B.birk_plan_create([Nn], [6], B.BIRK_F64)
    X = dev(ivp["guess"].ravel(), torch.float64)
    xa = dev(ivp["x_a"], torch.float64)
    out = B.birk_newton_ivp(plan, xa, X, rhs=lambda x, f, j, s: B.BIRK_ERR_NONFINITE, raise_on_error=False)
    assert out["status"] == B.BIRK_ERR_NONFINITE
    # argument errors found on the host
    lib = B._lib
    assert lib.birk_newton_ivp(plan.handle, None, B._ptr(xa), B._ptr(X), None, None) == B.BIRK_ERR_ARG
    with pytest.raises(B.BirkError):
        B.birk_newton_ivp(plan, xa, X, max_newton=0)
    with pytest.raises(B.BirkError):
        B.birk_newton_ivp(plan, xa, X, linear={"restart": 0})
    plan.destroy()
    # the two-body model needs n_x = 6; float plans are not supported
    p5 = B.birk_plan_create([Nn], [5], B.BIRK_F64)
    v5 = torch.zeros(5 * Nn, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BirkError) as ex:
        B.birk_newton_ivp(p5, torch.zeros(5, dtype=torch.float64, device="cuda"), v5)
    assert ex.value.status == B.BIRK_ERR_UNSUPPORTED
    p5.destroy()
    p32 = B.birk_plan_create([Nn], [6], B.BIRK_F32)
    with pytest.raises(B.BirkError) as ex:
        B.birk_newton_ivp(p32, xa, X)
    assert ex.value.status == B.BIRK_ERR_UNSUPPORTED
    p32.destroy()
