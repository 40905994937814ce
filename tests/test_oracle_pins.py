"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests touches the HIP path.  Each check is chosen so that a plausible
slip in the oracle (a dropped term, a wrong sign or index, a transposed operand)
breaks at least one of them:

* printed worked examples (B^a and B~^a for 10 CGL points);
* two independent constructions of B^a (Lagrange quadrature vs modal route);
* closed forms: CC weights, B^a row 0 = 0, last row = weights, B^a 1 = tau + 1,
  exact antiderivatives of arbitrary polynomials of degree <= N (monomial basis);
* the preconditioner's forward substitution vs a dense LAPACK solve, and the paper's
  printed recursions (FastBccV as printed; FastPinvY's running-sum line as printed
  does not invert P, which is why the oracle reads it as exact forward substitution);
* exact ODE solutions: the LTI flow expm(A (tau + 1)) x_a and the time-shift,
  rotation and scaling solutions of the linearised two-body flow;
* brute force: a textbook LU against LAPACK; GMRES against the dense solve;
* the paper's qualitative claim that preconditioned Krylov counts do not grow with N.
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import birkhoff as bk
from oracle import system as sy
from paper_2509_01855_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- worked examples
def test_printed_Ba10():
    printed = np.loadtxt(os.path.join(GOLDEN, "ba10_printed.txt"))
    B = bk.dense_Ba_quadrature(9)
    assert printed.shape == (10, 10)
    assert np.max(np.abs(B - printed)) <= 0.01
    # all but the four entries listed in the fixture header round exactly
    off = np.argwhere(np.abs(B - printed) > 0.005 + 1e-12)
    assert sorted(map(tuple, off)) == [(3, 6), (3, 7), (3, 8), (4, 9)]


def test_printed_Btilde10():
    printed = np.loadtxt(os.path.join(GOLDEN, "btilde10_printed.txt"))
    Bt = bk.btilde_dense(bk.weights(9))
    assert np.max(np.abs(Bt - printed)) <= 0.005 + 1e-12


# ---------------------------------------------------------------- B^a itself
@pytest.mark.parametrize("N", [2, 3, 4, 5, 9, 16, 31, 64, 127])
def test_two_constructions_agree(N):
    B1 = bk.dense_Ba_quadrature(N)
    B2 = bk.dense_Ba_modal(N)
    assert np.max(np.abs(B1 - B2)) <= 5e-14


@pytest.mark.parametrize("N", [2, 3, 9, 16, 255, 256])
def test_rows_and_weights(N):
    B = bk.dense_Ba(N)
    w_cc = bk.cc_weights_closed_form(N)
    assert np.max(np.abs(B[0])) <= 1e-15                  # B_j^a(-1) = 0
    assert np.max(np.abs(B[N] - w_cc)) <= 1e-14           # last row = CC weights
    assert abs(w_cc.sum() - 2.0) <= 1e-13
    assert np.max(np.abs(w_cc - w_cc[::-1])) <= 1e-15
    assert np.all(w_cc > 0)
    w0 = 1.0 / (N * N - 1.0) if N % 2 == 0 else 1.0 / (N * N)
    assert abs(w_cc[0] - w0) <= 1e-15 and abs(w_cc[N] - w0) <= 1e-15
    # one-row route agrees with the dense matrix everywhere
    for i in {0, 1, N // 2, N - 1, N}:
        assert np.max(np.abs(bk.ba_row(N, i) - B[i])) <= 1e-14


@pytest.mark.parametrize("N", [3, 10, 255, 1024])
def test_Ba_times_ones(N):
    B = bk.dense_Ba(N)
    tau = bk.cgl_nodes(N)
    assert np.max(np.abs(B @ np.ones(N + 1) - (tau + 1.0))) <= 1e-13


@pytest.mark.parametrize("N", [4, 9, 33, 64])
def test_exact_for_polynomials_monomial_basis(N):
    """B^a p(tau) = P(tau) - P(-1) for any p of degree <= N, P' = p.

    The polynomial is built in the monomial basis (numpy Polynomial), so this does not
    reuse the Chebyshev antiderivative formulas.
    """
    rng = np.random.default_rng(N)
    deg = min(N, 12)                        # keep monomial coefficients well scaled
    p = np.polynomial.Polynomial(rng.standard_normal(deg + 1))
    Pint = p.integ(lbnd=-1.0)
    tau = bk.cgl_nodes(N)
    B = bk.dense_Ba_quadrature(N)
    assert np.max(np.abs(B @ p(tau) - Pint(tau))) <= 1e-12


@pytest.mark.parametrize("N", [5, 16, 63])
def test_exact_on_every_chebyshev_mode(N):
    B = bk.dense_Ba_quadrature(N)
    for k in range(N + 1):
        v = bk.cheb_T_at_nodes(N, k)
        assert np.max(np.abs(B @ v - bk.cheb_antiderivative_at_nodes(N, k))) <= 1e-13


def test_aliasing_identity():
    """T_{N+1} = T_{N-1} at the CGL nodes (App. C)."""
    for N in (2, 7, 64, 1 << 20):
        d = bk.cheb_T_at_nodes(N, N + 1) - bk.cheb_T_at_nodes(N, N - 1)
        assert np.max(np.abs(d)) <= 1e-15


@pytest.mark.parametrize("N", [4, 9, 100])
def test_T_inverse_closed_form(N):
    assert np.max(np.abs(bk.T_inverse_closed_form(N) - np.linalg.inv(bk.T_matrix(N)))) <= 1e-13


def test_chebyshev_node_values():
    N = 12
    tau = bk.cgl_nodes(N)
    assert tau[0] == -1.0 and tau[-1] == 1.0
    assert np.all(tau[::-1] == -tau)
    for k in range(N + 2):
        assert np.max(np.abs(bk.cheb_T_at_nodes(N, k)
                             - np.polynomial.chebyshev.chebval(tau, np.eye(N + 2)[k]))) <= 1e-14


@pytest.mark.parametrize("N", [8, 255])
def test_sparse_mode_exact_matches_dense(N):
    modes, alphas = wl.sparse_modes(11, N, count=16)
    v = bk.sparse_mode_values(N, modes, alphas)
    assert np.max(np.abs(bk.dense_Ba(N) @ v - bk.sparse_mode_exact(N, modes, alphas))) <= 1e-13


def test_sparse_mode_exact_large_N_against_rows():
    """Two independent routes at N = 2^16: closed-form antiderivatives vs single rows."""
    N = 1 << 16
    modes, alphas = wl.sparse_modes(5, N, count=24)
    v = bk.sparse_mode_values(N, modes, alphas)
    exact = bk.sparse_mode_exact(N, modes, alphas)
    for i in (0, 1, 7, N // 3, N // 2, N - 1, N):
        assert abs(bk.ba_row(N, i) @ v - exact[i]) <= 1e-12 * max(1.0, np.abs(exact).max())


@pytest.mark.parametrize("N", [2, 3, 9, 16, 31, 64])
def test_columns_match_quadrature_construction(N):
    """ba_col against the columns of B^a built by Gauss-Legendre quadrature of the
    Lagrange basis (construction 1, independent of the modal route ba_col takes)."""
    B = bk.dense_Ba_quadrature(N)
    for j in range(N + 1):
        assert np.max(np.abs(bk.ba_col(N, j) - B[:, j])) <= 5e-15


def test_columns_match_rows_at_4096():
    """(B^a)_ij from a row (ba_row) and from a column (ba_col) at N = 4096, where the two
    take different routes through the modal definition; plus the first and last rows
    seen through the columns: 0 and the textbook CC weights."""
    N = 4096
    rng = np.random.default_rng(5)
    pairs = [(0, 5), (7, 0), (N, N), (N, 0), (1, N)] + [tuple(rng.integers(0, N + 1, 2)) for _ in range(8)]
    for i, j in pairs:
        r = bk.ba_row(N, int(i))[int(j)]
        c = bk.ba_col(N, int(j))[int(i)]
        assert abs(r - c) <= 1e-14 * (2.0 / N)            # entries are O(1/N)
    w = bk.cc_weights_closed_form(N)
    for j in (0, 1, N // 2, N):
        col = bk.ba_col(N, j)
        assert abs(col[0]) <= 1e-18                       # row 0 of B^a is zero
        assert abs(col[N] - w[j]) <= 1e-14 * (2.0 / N)    # row N is the CC weights


def test_transpose_properties():
    N = 40
    B = bk.dense_Ba(N)
    eN = np.zeros(N + 1)
    eN[N] = 1.0
    e0 = np.zeros(N + 1)
    e0[0] = 1.0
    assert np.max(np.abs(B.T @ eN - bk.cc_weights_closed_form(N))) <= 1e-14
    assert np.max(np.abs(B.T @ e0)) <= 1e-15


# ---------------------------------------------------------------- preconditioner
def test_btilde_apply_against_row_sums():
    """B~^a v from its row definition (0 above the diagonal, w_j / 2 on it, w_j below it),
    summed term by term, against the dense matrix and against btilde_apply."""
    rng = np.random.default_rng(1)
    N = 50
    w = bk.weights(N)
    v = rng.standard_normal(N + 1)
    ref = bk.btilde_dense(w) @ v
    brute = np.array([sum(w[j] * v[j] for j in range(k)) + 0.5 * w[k] * v[k] for k in range(N + 1)])
    assert np.max(np.abs(brute - ref)) <= 1e-14
    assert np.max(np.abs(bk.btilde_apply(w, v) - ref)) <= 1e-14
    # The columns of B~^a are constant below the diagonal, so consecutive outputs differ
    # by the mean of the neighbouring terms w_j v_j: the property that lets FastBccV run
    # as a single pass over the nodes.
    out = bk.btilde_apply(w, v)
    wv = w * v
    assert np.max(np.abs(np.diff(out) - 0.5 * (wv[:-1] + wv[1:]))) <= 1e-14


@pytest.mark.parametrize("kind", ["lti", "kepler"])
def test_precond_inverse(kind):
    N_n = 33
    inst = wl.lti_instance(4, N_n) if kind == "lti" else wl.kepler_instance(4, N_n)
    N = N_n - 1
    w = bk.weights(N)
    P = sy.dense_P(N, inst.J, w)
    y = np.random.default_rng(2).standard_normal(inst.n)
    x_lapack = np.linalg.solve(P, y)
    assert np.max(np.abs(sy.precond_inverse(w, inst.J, y) - x_lapack)) <= 1e-13
    assert np.max(np.abs(sy.precond_inverse_dense(P, y, inst.n_x) - x_lapack)) <= 1e-13
    assert np.max(np.abs(sy.precond_apply(w, inst.J, x_lapack) - y)) <= 1e-13
    assert np.max(np.abs(P @ y - sy.precond_apply(w, inst.J, y))) <= 1e-13


def test_running_sum_must_carry_the_solution():
    """Scalar case of P = I - B~^a diag(d).  Row k of P xi = y reads
    (1 - w_k d_k / 2) xi_k - sum_{j<k} w_j d_j xi_j = y_k, so the running sum that forward
    substitution carries is built from the solution values xi_j.  The FastPinvY box
    builds it from the right-hand side values instead (with the opposite sign); that
    variant, evaluated here with a cumulative sum over y, misses P^{-1} y by O(1), while
    the oracle's forward substitution reaches the LAPACK solve."""
    rng = np.random.default_rng(0)
    N = 30
    w = bk.weights(N)
    d = rng.standard_normal(N + 1) - 1.0
    Y = rng.standard_normal(N + 1)
    P = np.eye(N + 1) - bk.btilde_dense(w) @ np.diag(d)
    exact = np.linalg.solve(P, Y)
    wdy = w * d * Y
    t = np.cumsum(wdy) - wdy                  # sum_{j<k} w_j d_j y_j
    from_inputs = (Y - t) / (1.0 - 0.5 * w * d)
    assert np.max(np.abs(from_inputs - exact)) > 1e-3
    xi = sy.precond_inverse(w, d[None, None, :], Y)
    assert np.max(np.abs(xi - exact)) <= 1e-13
    # and xi satisfies every row of P xi = y written out as above
    wdx = w * d * xi
    rows = (1.0 - 0.5 * w * d) * xi - (np.cumsum(wdx) - wdx)
    assert np.max(np.abs(rows - Y)) <= 1e-13


# ---------------------------------------------------------------- the linear system
@pytest.mark.parametrize("N_n", [32, 256, 257])
def test_lti_solution_matches_matrix_exponential(N_n):
    inst = wl.lti_instance(0, N_n)
    N = N_n - 1
    A = sy.dense_A(N, inst.J)
    X = sy.solve_dense(A, sy.beta_vector(inst.x_a, N_n)).reshape(inst.n_x, N_n)
    tau = bk.cgl_nodes(N)
    Xe = np.stack([scipy.linalg.expm(inst.J * (t + 1.0)) @ inst.x_a for t in tau], axis=1)
    assert np.max(np.abs(X - Xe)) <= 1e-13


@pytest.mark.parametrize("which", ["shift", "rotation", "scaling"])
def test_kepler_exact_solutions(which):
    N_n = 257
    inst = wl.kepler_instance(2, N_n)
    ex = inst.extra
    r, v, acc, t = ex["r"], ex["v"], ex["acc"], ex["t"]
    if which == "shift":
        Z = np.concatenate([v, acc])
    elif which == "rotation":
        om = np.array([0.3, -0.7, 0.5])
        Z = np.concatenate([np.cross(om, r.T).T, np.cross(om, v.T).T])
    else:
        Z = np.concatenate([r - 1.5 * t * v, -0.5 * v - 1.5 * t * acc])
    A = sy.dense_A(N_n - 1, inst.J)
    X = sy.solve_dense(A, sy.beta_vector(Z[:, 0], N_n)).reshape(6, N_n)
    assert np.max(np.abs(X - Z)) <= 1e-11 * max(1.0, np.abs(Z).max())


def test_textbook_lu_matches_lapack():
    inst = wl.kepler_instance(7, 17)
    A = sy.dense_A(16, inst.J)
    b = sy.beta_vector(inst.x_a, 17)
    x1 = sy.lu_solve_textbook(A, b)
    x2 = sy.solve_dense(A, b)
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.abs(x2).max()
    assert np.max(np.abs(A @ x1 - b)) <= 1e-12


@pytest.mark.parametrize("kind", ["lti", "kepler"])
def test_gmres_reaches_dense_solution(kind):
    N_n = 129
    inst = wl.lti_instance(0, N_n) if kind == "lti" else wl.kepler_instance(2, N_n)
    N = N_n - 1
    A = sy.dense_A(N, inst.J)
    b = sy.beta_vector(inst.x_a, N_n)
    w = bk.weights(N)
    x, its, hist = sy.gmres_right(lambda z: A @ z, lambda y: sy.precond_inverse(w, inst.J, y), b,
                                  tol=1e-12)
    assert sy.rel_residual(lambda z: A @ z, b, x) <= 1e-12
    xd = sy.solve_dense(A, b)
    assert np.max(np.abs(x - xd)) <= 1e-10 * np.abs(xd).max()
    # unpreconditioned GMRES needs several times more iterations
    x2, its2, _ = sy.gmres_right(lambda z: A @ z, lambda y: y, b, tol=1e-12)
    assert its2 >= 3 * its


def test_krylov_counts_do_not_grow_with_N():
    counts = []
    for N_n in (65, 129, 257, 513):
        inst = wl.kepler_instance(2, N_n)
        N = N_n - 1
        A = sy.dense_A(N, inst.J)
        b = sy.beta_vector(inst.x_a, N_n)
        w = bk.weights(N)
        _, its, _ = sy.gmres_right(lambda z: A @ z, lambda y: sy.precond_inverse(w, inst.J, y), b,
                                   tol=1e-12)
        counts.append(its)
    assert all(c2 <= c1 for c1, c2 in zip(counts, counts[1:])), counts


def test_apply_A_matches_dense():
    inst = wl.kepler_instance(3, 20)
    N = 19
    Ba = bk.dense_Ba(N)
    x = np.random.default_rng(0).standard_normal(inst.n)
    assert np.max(np.abs(sy.apply_A(Ba, inst.J, x) - sy.dense_A(N, inst.J, Ba) @ x)) <= 1e-14


def test_condition_number_is_order_one():
    """kappa(I - B^a (x) A) stays O(1) as N grows (the Birkhoff property the paper builds on)."""
    ks = []
    for N_n in (33, 65, 129, 257):
        inst = wl.lti_instance(0, N_n)
        ks.append(np.linalg.cond(sy.dense_A(N_n - 1, inst.J)))
    assert max(ks) < 20.0 and max(ks) / min(ks) < 1.5, ks


def test_condition_number_kepler_systems():
    """kappa of the Kepler-linearised operator (orbit of the million-point workload, seed 2)
    is flat in N near 720; the GPU solve tests derive their error bars from it."""
    ks = [np.linalg.cond(sy.dense_A(N_n - 1, wl.kepler_instance(2, N_n).J)) for N_n in (65, 129, 257)]
    assert 500.0 < min(ks) and max(ks) < 1000.0 and max(ks) / min(ks) < 1.05, ks


# ---------------------------------------------------------------- extended-precision products
@pytest.mark.parametrize("N", [2, 9, 64, 255])
def test_extended_products_match_quadrature_construction(N):
    X = np.random.default_rng(N).standard_normal((3, N + 1))
    B1 = bk.dense_Ba_quadrature(N)
    assert np.max(np.abs(bk.apply_Ba_extended(N, X) - X @ B1.T)) <= 1e-13
    assert np.max(np.abs(bk.apply_Ba_extended(N, X, transpose=True) - X @ B1)) <= 1e-13


def test_extended_products_match_rows_at_3000():
    """At N = 2999 the extended evaluation and the O(N log N) row route agree to ~1e-15,
    which the double dense matrix (LAPACK inverse + O(N^3) product) does not reach."""
    N = 2999
    X = np.random.default_rng(1).standard_normal((2, N + 1))
    R = np.array([bk.ba_row(N, i) for i in range(N + 1)])
    for tr, ref in ((False, X @ R.T), (True, X @ R)):
        e = bk.apply_Ba_extended(N, X, transpose=tr)
        assert np.max(np.abs(e - ref)) / np.max(np.abs(e)) <= 1e-14


def test_extended_products_exact_on_modes():
    N = 200
    modes, alphas = wl.sparse_modes(3, N, count=20)
    v = bk.sparse_mode_values(N, modes, alphas)
    assert np.max(np.abs(bk.apply_Ba_extended(N, v)[0] - bk.sparse_mode_exact(N, modes, alphas))) <= 1e-15


# ---------------------------------------------------------------- b-form and endpoint row
@pytest.mark.parametrize("N", [2, 3, 9, 16, 64, 127])
def test_bform_two_constructions_agree(N):
    """B^b from its own conditions (anchor +1, quadrature on [tau_i, 1]) against
    B^a - 1 w^T (eq:xN=Birka+b); the two share only the Lagrange basis."""
    assert np.max(np.abs(bk.dense_Bb_quadrature(N) - bk.dense_Bb(N))) <= 5e-14


@pytest.mark.parametrize("N", [2, 9, 16, 255, 256])
def test_bform_rows(N):
    B = bk.dense_Bb(N)
    assert np.max(np.abs(B[N])) <= 1e-15                                   # B_j^b(1) = 0
    assert np.max(np.abs(B[0] + bk.cc_weights_closed_form(N))) <= 1e-14     # B_j^b(-1) = -w_j
    tau = bk.cgl_nodes(N)
    assert np.max(np.abs(B @ np.ones(N + 1) - (tau - 1.0))) <= 1e-13       # integral from 1 of 1


@pytest.mark.parametrize("N", [4, 9, 33, 64])
def test_bform_exact_for_polynomials_monomial_basis(N):
    """B^b p(tau) = P(tau) - P(1), P' = p, p of degree <= N (monomial basis)."""
    rng = np.random.default_rng(100 + N)
    p = np.polynomial.Polynomial(rng.standard_normal(min(N, 12) + 1))
    Pint = p.integ(lbnd=1.0)
    tau = bk.cgl_nodes(N)
    assert np.max(np.abs(bk.dense_Bb_quadrature(N) @ p(tau) - Pint(tau))) <= 1e-12


@pytest.mark.parametrize("N", [2, 9, 64, 255])
def test_bform_extended_products(N):
    X = np.random.default_rng(N + 7).standard_normal((3, N + 1))
    Bq = bk.dense_Bb_quadrature(N)
    assert np.max(np.abs(bk.apply_Bb_extended(N, X) - X @ Bq.T)) <= 1e-13
    # the transposed product sums N + 1 quadrature entries per output, each off by a
    # few ulps of the barycentric evaluation: 5e-13 at N = 255
    assert np.max(np.abs(bk.apply_Bb_extended(N, X, transpose=True) - X @ Bq)) <= 5e-13


def test_bform_sparse_modes():
    N = 64
    modes, alphas = wl.sparse_modes(5, N, count=12)
    v = bk.sparse_mode_values(N, modes, alphas)
    ref = bk.sparse_mode_exact_b(N, modes, alphas)
    assert np.max(np.abs(bk.dense_Bb_quadrature(N) @ v - ref)) <= 1e-13
    assert abs(ref[N]) == 0.0


@pytest.mark.parametrize("N", [5, 16, 63])
def test_endpoint_row(N):
    """x^b = x^a + w^T V (eq:Prob-PNa): for V = p(tau), x^b - x^a is the integral of p
    over [-1, 1], and it equals the last node of X = x^a + B^a V."""
    rng = np.random.default_rng(200 + N)
    tau = bk.cgl_nodes(N)
    ps = [np.polynomial.Polynomial(rng.standard_normal(min(N, 10) + 1)) for _ in range(3)]
    V = np.stack([p(tau) for p in ps])
    xa = rng.standard_normal(3)
    xb = bk.endpoint_b(N, xa, V)
    exact = xa + np.array([p.integ(lbnd=-1.0)(1.0) for p in ps])
    assert np.max(np.abs(xb - exact)) <= 1e-13
    X = xa[:, None] + V @ bk.dense_Ba_quadrature(N).T
    assert np.max(np.abs(X[:, N] - xb)) <= 1e-13
    # the two forms describe the same trajectory: x^a + B^a V = x^b + B^b V
    Xb = xb[:, None] + V @ bk.dense_Bb_quadrature(N).T
    assert np.max(np.abs(X - Xb)) <= 1e-13


# ---------------------------------------------------------------- Newton on the nonlinear IVP
from oracle import newton as nw  # noqa: E402


def test_two_body_jacobian_matches_finite_differences():
    rng = np.random.default_rng(40)
    X = rng.standard_normal((6, 7))
    X[:3] += 2.0 * np.sign(X[:3])          # keep |r| away from 0
    J = nw.two_body_jacobian(X, 1.7, 0.9)
    h = 1e-6
    for c in range(6):
        E = np.zeros_like(X)
        E[c] = h
        fd = (nw.two_body_rhs(X + E, 1.7, 0.9) - nw.two_body_rhs(X - E, 1.7, 0.9)) / (2 * h)
        assert np.max(np.abs(fd - J[:, c, :])) <= 1e-8


def test_two_body_rhs_is_the_orbit_derivative():
    """f(X) on the closed-form orbit equals s dX/dt, by central differences in time of
    Kepler's solution (independent of the formula for f)."""
    R = np.linalg.qr(np.random.default_rng(41).standard_normal((3, 3)))[0]
    t = np.linspace(0.3, 6.0, 9)
    h = 1e-5
    rp, vp, _ = wl.kepler_orbit(t + h, 0.15, R)
    rm, vm, _ = wl.kepler_orbit(t - h, 0.15, R)
    r, v, _ = wl.kepler_orbit(t, 0.15, R)
    dX = np.concatenate([rp - rm, vp - vm]) / (2 * h)
    F = nw.two_body_rhs(np.concatenate([r, v]), 2.5)
    assert np.max(np.abs(F - 2.5 * dX)) <= 1e-8


@pytest.mark.parametrize("e", [0.0, 0.1, 0.2])
def test_newton_ivp_reaches_kepler_closed_form(e):
    """Newton on eq:X-V=nonlin from the circular orbit reaches Kepler's solution at the
    nodes (spectral accuracy at N = 200 over one period), with quadratic convergence at
    the end."""
    N = 200
    ivp = wl.kepler_ivp(42, N + 1, e)
    X, its, hist, steps = nw.newton_ivp(N, ivp["x_a"], ivp["guess"], ivp["scale"], ivp["mu"])
    assert np.max(np.abs(X - ivp["exact"])) <= 1e-11
    assert its <= 10
    if its >= 3:
        # quadratic: the last reductions outpace any linear rate
        assert hist[-2] <= 1e-3 * hist[-3] or hist[-2] <= 1e-10
    # the exact orbit satisfies the discrete equations to the interpolation error
    Ba = bk.dense_Ba(N)
    G = nw.ivp_residual(Ba, ivp["x_a"], ivp["exact"], nw.two_body_rhs(ivp["exact"], ivp["scale"]))
    assert np.max(np.abs(G)) <= 1e-11


def test_newton_ivp_line_search_engages():
    """From a poor guess (the circular orbit at e = 0.3) full steps are rejected at
    first and the damped iteration still converges."""
    N = 120
    ivp = wl.kepler_ivp(43, N + 1, 0.3)
    X, its, hist, steps = nw.newton_ivp(N, ivp["x_a"], ivp["guess"], ivp["scale"], ivp["mu"])
    assert np.max(np.abs(X - ivp["exact"])) <= 1e-9
    assert min(steps) < 1.0 and steps[-1] == 1.0
    assert all(b < a for a, b in zip(hist, hist[1:]))


@pytest.mark.parametrize("kind,N_n", [("lti", 17), ("kepler", 33)])
def test_dense_A_is_the_kronecker_form(kind, N_n):
    """The block-by-block construction of A equals I - kron(I, B^a) blockdiag(J) formed
    literally, bit for bit."""
    inst = wl.lti_instance(0, N_n) if kind == "lti" else wl.kepler_instance(2, N_n)
    N = N_n - 1
    Ba = bk.dense_Ba(N)
    Jf = sy.expand_jacobian(inst.J, N_n)
    lit = np.eye(inst.n) - np.kron(np.eye(inst.n_x), Ba) @ sy.dense_jacobian(Jf, N_n)
    assert np.array_equal(sy.dense_A(N, inst.J, Ba), lit)
