"""Pins of the KKT oracle (oracle/kkt.py), CPU only: the backward substitution P^{-T}
against LAPACK on the dense P^T, the saddle-point matrix against its definition and its
inertia, the dense KKT solution against elimination through A, and the plain MINRES
against dense solves, its finite termination on a matrix with few distinct eigenvalues,
its monotone residual estimates and N-independent preconditioned iteration counts."""

import numpy as np
import pytest

from oracle import birkhoff as bk
from oracle import kkt
from oracle import system as sy
from paper_2509_01855_amd import workloads as wl


def _inst(kind, N_n, seed=0):
    return wl.kepler_instance(2 + seed, N_n) if kind == "kepler" else wl.lti_instance(seed, N_n)


@pytest.mark.parametrize("kind", ["lti", "kepler"])
def test_transpose_inverse_matches_lapack(kind):
    N_n = 33
    inst = _inst(kind, N_n)
    N = N_n - 1
    w = bk.weights(N)
    P = sy.dense_P(N, inst.J, w)
    y = np.random.default_rng(3).standard_normal(inst.n)
    assert np.max(np.abs(kkt.precond_transpose_inverse(w, inst.J, y) - np.linalg.solve(P.T, y))) <= 1e-13
    # and it is the adjoint of the forward substitution: <P^{-1} a, b> = <a, P^{-T} b>
    a = np.random.default_rng(4).standard_normal(inst.n)
    lhs = sy.precond_inverse(w, inst.J, a) @ y
    rhs = a @ kkt.precond_transpose_inverse(w, inst.J, y)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(y)


@pytest.mark.parametrize("kind", ["lti", "kepler"])
def test_kkt_matrix_symmetry_inertia_and_products(kind):
    N_n = 17
    inst = _inst(kind, N_n)
    N = N_n - 1
    h = 0.5 + np.random.default_rng(5).random(inst.n)
    Ba = bk.dense_Ba(N)
    K = kkt.dense_K(N, inst.J, h, Ba)
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 0) == inst.n and np.sum(ev < 0) == inst.n
    z = np.random.default_rng(6).standard_normal(2 * inst.n)
    assert np.max(np.abs(kkt.kkt_apply(Ba, inst.J, h, z) - K @ z)) <= 1e-13 * np.max(np.abs(K @ z)) * 10


@pytest.mark.parametrize("kind", ["lti", "kepler"])
def test_kkt_dense_solution_matches_elimination(kind):
    N_n = 33
    inst = _inst(kind, N_n)
    N = N_n - 1
    rng = np.random.default_rng(7)
    h = 0.5 + rng.random(inst.n)
    f, g = rng.standard_normal(inst.n), rng.standard_normal(inst.n)
    A = sy.dense_A(N, inst.J)
    chi, lam = kkt.kkt_solve_dense(kkt.dense_K(N, inst.J, h), f, g)
    chi2, lam2 = kkt.kkt_solve_by_elimination(A, h, f, g)
    assert np.max(np.abs(chi - chi2)) <= 1e-12 * np.max(np.abs(chi2))
    assert np.max(np.abs(lam - lam2)) <= 1e-11 * np.max(np.abs(lam2))


def test_minres_finite_termination_on_few_eigenvalues():
    """A symmetric indefinite matrix with 4 distinct eigenvalues: MINRES (unpreconditioned)
    reaches the solution in at most 4 steps."""
    rng = np.random.default_rng(8)
    q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.repeat([-3.0, -0.5, 2.0, 7.0], 10)
    A = (q * lam) @ q.T
    b = rng.standard_normal(40)
    x, its, hist = kkt.minres(lambda v: A @ v, lambda v: v, b, tol=1e-13)
    assert its <= 4
    assert np.max(np.abs(x - np.linalg.solve(A, b))) <= 1e-11


@pytest.mark.parametrize("kind", ["lti", "kepler"])
@pytest.mark.parametrize("precond", [False, True])
def test_minres_reaches_dense_kkt_solution(kind, precond):
    N_n = 33
    inst = _inst(kind, N_n)
    N = N_n - 1
    rng = np.random.default_rng(9)
    h = 0.5 + rng.random(inst.n)
    f, g = rng.standard_normal(inst.n), rng.standard_normal(inst.n)
    Ba = bk.dense_Ba(N)
    w = bk.weights(N)
    K = kkt.dense_K(N, inst.J, h, Ba)
    chi, lam = kkt.kkt_solve_dense(K, f, g)
    prec = (lambda r: kkt.kkt_precond_apply(w, inst.J, h, r)) if precond else (lambda r: r)
    z, its, hist = kkt.minres(lambda v: kkt.kkt_apply(Ba, inst.J, h, v), prec, np.concatenate([f, g]),
                              tol=1e-13, max_iter=4000)
    ref = np.concatenate([chi, lam])
    assert np.max(np.abs(z - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert all(hist[k + 1] <= hist[k] * (1 + 1e-12) for k in range(len(hist) - 1))
    if precond:
        assert its <= 40


def test_preconditioned_minres_counts_do_not_grow_with_N():
    """With the Birkhoff-preconditioned block-diagonal M the MINRES counts do not grow with
    N, and fall at first (the KKT analogue of the paper's observation on its Krylov
    counts); without it they stay near 58 for this system."""
    counts = []
    for N_n in (33, 65, 129):
        inst = wl.lti_instance(0, N_n)
        N = N_n - 1
        h = np.ones(inst.n)
        Ba = bk.dense_Ba(N)
        w = bk.weights(N)
        b = np.concatenate([np.zeros(inst.n), sy.beta_vector(inst.x_a, N_n)])
        _, its, _ = kkt.minres(lambda v: kkt.kkt_apply(Ba, inst.J, h, v),
                               lambda r: kkt.kkt_precond_apply(w, inst.J, h, r), b, tol=1e-12)
        counts.append(its)
    assert all(counts[k + 1] <= counts[k] for k in range(len(counts) - 1)), counts
    assert counts[0] <= 20, counts
