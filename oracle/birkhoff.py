"""Birkhoff-Chebyshev operators on the CGL grid, written out from their definitions.

Test infrastructure only (see the package docstring).  Float64 throughout.

Paper references are to arXiv 2509.01855 ("A Million-Point Fast Trajectory
Optimization Solver"):

* eq:CGLpts            CGL nodes tau_j = -cos(j pi / N), j = 0..N.
* eq:birk-conditions   B_j^a(-1) = 0 and dB_j^a/dtau(tau_i) = delta_ij, so B_j^a is
                       the antiderivative from -1 of the Lagrange basis l_j.
* eq:manyDefs          [B^a]_ij = B_j^a(tau_i); w_B = Clenshaw-Curtis weights.
* eq:Tkj=coskj         T_k(tau_j) = cos(k (N - j) pi / N).
* eq:intChebPoly=      closed-form antiderivatives of T_k from -1.
* App. B, eq:ak=3      modal coefficients from nodal values (discrete orthogonality).
* Sec. "Development of a Special Birkhoff-Centric Preconditioner"
                       last row of B^a = CC weights; the lower-triangular B~^a.
* eq:xN=Birka+b        the b-form: B_j^b(+1) = 0 with the same derivative conditions,
                       so B_j^b = B_j^a - B_j^a(+1) and B^b = B^a - 1 w_B^T.
* eq:Prob-PNa          the endpoint row x^b = x^a + w_B^T V.
"""

from __future__ import annotations

import functools

import numpy as np
import scipy.fft

__all__ = [
    "cgl_nodes",
    "cheb_T_at_nodes",
    "T_matrix",
    "T_inverse_closed_form",
    "cheb_antiderivative_at_nodes",
    "lagrange_basis",
    "dense_Ba_quadrature",
    "dense_Ba_modal",
    "dense_Ba",
    "weights",
    "cc_weights_closed_form",
    "btilde_dense",
    "btilde_apply",
    "ba_row",
    "ba_col",
    "sparse_mode_exact",
    "sparse_mode_values",
    "apply_Ba_extended",
    "dense_Bb_quadrature",
    "dense_Bb",
    "sparse_mode_exact_b",
    "apply_Bb_extended",
    "endpoint_b",
]


def cgl_nodes(N: int) -> np.ndarray:
    """CGL nodes tau_j = -cos(j pi / N), j = 0..N (eq:CGLpts).

    Evaluated as sin(pi (2j - N) / (2N)), the same number, so that tau_{N-j} = -tau_j
    holds exactly in floating point and the ends are exactly -1 and +1.
    """
    j = np.arange(N + 1, dtype=np.float64)
    return np.sin(np.pi * (2.0 * j - N) / (2.0 * N))


def cheb_T_at_nodes(N: int, k: int) -> np.ndarray:
    """T_k(tau_j) for j = 0..N via eq:Tkj=coskj, cos(pi * (k (N - j) mod 2N) / N).

    The integer argument is reduced exactly before the cosine; valid for any k >= 0,
    including k = N + 1 (evaluated directly, without the aliasing identity).
    """
    j = np.arange(N + 1, dtype=np.int64)
    m = (np.int64(k) * (N - j)) % (2 * N)
    return np.cos(np.pi * m.astype(np.float64) / N)


def T_matrix(N: int) -> np.ndarray:
    """Modal-to-nodal matrix of eq:V=Ta: T[j, k] = T_k(tau_j), (N+1) x (N+1)."""
    j = np.arange(N + 1, dtype=np.int64)[:, None]
    k = np.arange(N + 1, dtype=np.int64)[None, :]
    m = (k * (N - j)) % (2 * N)
    return np.cos(np.pi * m.astype(np.float64) / N)


def T_inverse_closed_form(N: int) -> np.ndarray:
    """Inverse of T from App. B (eq:ak=3): a_k = 2/(N c_k) sum_j e_j T_k(tau_j) v_j.

    c_0 = c_N = 2, otherwise 1; e_0 = e_N = 1/2, otherwise 1 (CGL quadrature end weights).
    """
    T = T_matrix(N)
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    e = np.ones(N + 1)
    e[0] = e[N] = 0.5
    return (2.0 / N) * (T.T / c[:, None]) * e[None, :]


def cheb_antiderivative_at_nodes(N: int, k: int) -> np.ndarray:
    """I_k(tau_j) = integral_{-1}^{tau_j} T_k, j = 0..N, by eq:intChebPoly=.

    k >= 2:  T_{k+1}/(2(k+1)) - T_{k-1}/(2(k-1)) - (-1)^k/(k^2 - 1)
    k == 1:  T_2/4 - 1/4
    k == 0:  T_1 + 1
    T_{k+1} is evaluated directly at the nodes (no aliasing), so this is exact for
    every k, including k = N.
    """
    if k == 0:
        return cheb_T_at_nodes(N, 1) + 1.0
    if k == 1:
        return cheb_T_at_nodes(N, 2) / 4.0 - 0.25
    sgn = 1.0 if k % 2 == 0 else -1.0
    return (cheb_T_at_nodes(N, k + 1) / (2.0 * (k + 1))
            - cheb_T_at_nodes(N, k - 1) / (2.0 * (k - 1))
            - sgn / (k * k - 1.0))


def lagrange_basis(N: int, x: np.ndarray) -> np.ndarray:
    """Values l_j(x) of the degree-N Lagrange basis on the CGL nodes; shape (len(x), N+1).

    Barycentric form with the CGL weights (-1)^j e_j (e_0 = e_N = 1/2, otherwise 1).
    A point that coincides with a node gets the Kronecker row.
    """
    tau = cgl_nodes(N)
    lam = np.ones(N + 1)
    lam[1::2] = -1.0
    lam[0] *= 0.5
    lam[N] *= 0.5
    x = np.asarray(x, dtype=np.float64)
    diff = x[:, None] - tau[None, :]
    hit = diff == 0.0
    diff[hit] = 1.0
    q = lam[None, :] / diff
    L = q / q.sum(axis=1, keepdims=True)
    rows = hit.any(axis=1)
    if rows.any():
        L[rows] = hit[rows].astype(np.float64)
    return L


def dense_Ba_quadrature(N: int) -> np.ndarray:
    """Construction 1 of B^a: [B^a]_ij = integral_{-1}^{tau_i} l_j (eq:birk-conditions).

    Each integral is taken by Gauss-Legendre quadrature on [-1, tau_i] with
    N//2 + 2 points, which integrates the degree-N integrand exactly.
    Cost O(N^3); for N up to a few hundred.
    """
    tau = cgl_nodes(N)
    nq = N // 2 + 2
    t, wq = np.polynomial.legendre.leggauss(nq)
    B = np.zeros((N + 1, N + 1))
    for i in range(1, N + 1):
        half = 0.5 * (tau[i] + 1.0)
        x = -1.0 + half * (t + 1.0)
        L = lagrange_basis(N, x)
        B[i] = half * (wq @ L)
    return B


def dense_Ba_modal(N: int) -> np.ndarray:
    """Construction 2 of B^a: nodal -> modal (inverse of T), integrate, evaluate.

    B^a = I T^{-1} with I[i, k] = integral_{-1}^{tau_i} T_k (eq:V=Ta, eq:BVt-1,
    eq:intChebPoly=).  T^{-1} is taken from a LAPACK solve, not from the closed form,
    so this construction does not lean on App. B.  Cost O(N^3) in BLAS/LAPACK.
    """
    T = T_matrix(N)
    Int = np.empty((N + 1, N + 1))
    for k in range(N + 1):
        Int[:, k] = cheb_antiderivative_at_nodes(N, k)
    Tinv = np.linalg.solve(T, np.eye(N + 1))
    return Int @ Tinv


def dense_Ba(N: int) -> np.ndarray:
    """Dense B^a = I T^{-1} with the closed-form inverse of App. B (eq:ak=3).

    Same definition as construction 2; the closed-form inverse keeps entries accurate
    to a few ulps at N in the thousands, where the LAPACK inverse loses ~3 digits.
    """
    Int = np.empty((N + 1, N + 1))
    for k in range(N + 1):
        Int[:, k] = cheb_antiderivative_at_nodes(N, k)
    return Int @ T_inverse_closed_form(N)


def weights(N: int) -> np.ndarray:
    """w_B: the last row of B^a, which equals the CC weights (Sec. on B~^a)."""
    return ba_row(N, N)


def cc_weights_closed_form(N: int) -> np.ndarray:
    """Textbook Clenshaw-Curtis weights on the CGL nodes, independent of B^a.

    w_j = integral_{-1}^{1} l_j, with l_j expanded by discrete orthogonality,
    l_j = 2 e_j / N * sum_k T_k(tau_j) T_k / c_k, and integral_{-1}^{1} T_k =
    2 / (1 - k^2) for even k, 0 for odd k.
    """
    T = T_matrix(N)
    k = np.arange(N + 1)
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    e = np.ones(N + 1)
    e[0] = e[N] = 0.5
    kf = k.astype(np.float64)
    even = k % 2 == 0
    mom = np.zeros(N + 1)
    mom[even] = 2.0 / (1.0 - kf[even] ** 2)
    return (2.0 / N) * e * (T @ (mom / c))


def btilde_dense(w: np.ndarray) -> np.ndarray:
    """Dense B~^a: 0 above the diagonal, w_j/2 on it, w_j below it (Sec. on B~^a)."""
    n = w.shape[0]
    B = np.tril(np.ones((n, n)), -1) * w[None, :]
    B[np.diag_indices(n)] = 0.5 * w
    return B


def btilde_apply(w: np.ndarray, V: np.ndarray) -> np.ndarray:
    """B~^a V along the last axis: (B~ V)_k = sum_{j<k} w_j v_j + w_k v_k / 2.

    This is the row-by-row definition of B~^a with the exclusive prefix sum taken by
    numpy's cumsum; the recursion in FastBccV reaches the same numbers.
    """
    wv = w * V
    excl = np.cumsum(wv, axis=-1) - wv
    return excl + 0.5 * wv


def ba_row(N: int, i: int) -> np.ndarray:
    """Row i of B^a, (B^a)_{ij} for j = 0..N, in O(N log N).

    (B^a)_{ij} = sum_k I_k(tau_i) (T^{-1})_{kj} with I_k from eq:intChebPoly= and
    T^{-1} from App. B, so (B^a)_{ij} = e_j sum_k u_k T_k(tau_j), u_k = 2 I_k(tau_i)/(N c_k).
    The cosine sum over k is one type-I DCT (scipy), used here as a library step.
    Lets the tests check single outputs at sizes where the dense matrix cannot exist.
    """
    k = np.arange(N + 1, dtype=np.int64)
    # I_k(tau_i) for all k at one node: theta_i = (N - i) pi / N, T_m(tau_i) = cos(m theta_i)
    def Tm(m):
        mm = (m.astype(np.int64) * (N - i)) % (2 * N)
        return np.cos(np.pi * mm.astype(np.float64) / N)
    Ik = np.empty(N + 1)
    Ik[0] = Tm(np.array([1]))[0] + 1.0
    Ik[1] = Tm(np.array([2]))[0] / 4.0 - 0.25
    kk = k[2:]
    sgn = np.where(kk % 2 == 0, 1.0, -1.0)
    Ik[2:] = (Tm(kk + 1) / (2.0 * (kk + 1)) - Tm(kk - 1) / (2.0 * (kk - 1))
              - sgn / (kk.astype(np.float64) ** 2 - 1.0))
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    u = 2.0 * Ik / (N * c)
    # S_m = sum_k u_k cos(pi k m / N); scipy's unnormalised DCT-I doubles interior terms
    x = u.copy()
    x[1:N] *= 0.5
    S = scipy.fft.dct(x, type=1)
    e = np.ones(N + 1)
    e[0] = e[N] = 0.5
    # T_k(tau_j) = cos(pi k (N - j) / N)  ->  S evaluated at m = N - j
    return e * S[::-1]


def ba_col(N: int, j: int) -> np.ndarray:
    """Column j of B^a, (B^a)_{ij} for i = 0..N, in O(N log N).

    Column j is B^a e_j = Int T^{-1} e_j (construction 2 with the inverse of App. B,
    eq:ak=3): the modal coefficients of the Lagrange polynomial l_j are
    u_k = (T^{-1})_{kj} = 2 e_j T_k(tau_j) / (N c_k), and the column holds the
    antiderivative sum_k u_k I_k(tau_i).  Each I_k is expanded by eq:intChebPoly= into
    T_{k+1}, T_{k-1} and a constant; the resulting cosine series of degree N + 1 is
    evaluated at the nodes by one type-I DCT (scipy, a library step) for degrees 0..N
    and directly for T_{N+1}.  Lets the tests check single outputs of B^aT g at sizes
    where the dense matrix cannot exist.
    """
    k = np.arange(N + 1, dtype=np.int64)
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    ej = 0.5 if j in (0, N) else 1.0
    Tkj = np.cos(np.pi * ((k * (N - j)) % (2 * N)).astype(np.float64) / N)
    u = 2.0 * ej * Tkj / (N * c)
    alpha = np.zeros(N + 2)      # coefficient of T_m, m = 0..N+1
    const = 0.0
    alpha[1] += u[0]             # I_0 = T_1 + 1
    const += u[0]
    alpha[2] += u[1] / 4.0       # I_1 = T_2 / 4 - 1 / 4
    const -= u[1] / 4.0
    kk = k[2:]
    kf = kk.astype(np.float64)
    sgn = np.where(kk % 2 == 0, 1.0, -1.0)
    np.add.at(alpha, kk + 1, u[2:] / (2.0 * (kf + 1.0)))
    np.add.at(alpha, kk - 1, -u[2:] / (2.0 * (kf - 1.0)))
    const -= float(np.sum(u[2:] * sgn / (kf * kf - 1.0)))
    # sum_{m<=N} alpha_m cos(pi m n / N) at n = 0..N; scipy's DCT-I doubles the interior
    x = alpha[:N + 1].copy()
    x[1:N] *= 0.5
    S = scipy.fft.dct(x, type=1)
    # T_m(tau_i) = cos(pi m (N - i) / N): the series at n = N - i, plus T_{N+1} directly
    return S[::-1] + alpha[N + 1] * cheb_T_at_nodes(N, N + 1) + const


def sparse_mode_values(N: int, modes, alphas) -> np.ndarray:
    """Nodal values v_j = sum_s alpha_s T_{k_s}(tau_j) of a sparse Chebyshev series."""
    v = np.zeros(N + 1)
    for k, a in zip(modes, alphas):
        v += a * cheb_T_at_nodes(N, int(k))
    return v


def sparse_mode_exact(N: int, modes, alphas) -> np.ndarray:
    """Exact B^a v for v = sum_s alpha_s T_{k_s} sampled at the nodes (k_s <= N).

    B^a reproduces the antiderivative from -1 of any polynomial of degree <= N at the
    nodes (its rows are integrals of the interpolant), so the exact result is
    sum_s alpha_s integral_{-1}^{tau_j} T_{k_s}, taken from eq:intChebPoly=.
    Cost O(len(modes) * N); usable at N = 2^20.
    """
    out = np.zeros(N + 1)
    for k, a in zip(modes, alphas):
        if not 0 <= int(k) <= N:
            raise ValueError("mode index must lie in [0, N]")
        out += a * cheb_antiderivative_at_nodes(N, int(k))
    return out


def apply_Ba_extended(N: int, X: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Rows of X times B^a^T (transpose=False: each row x -> B^a x) or times B^a
    (transpose=True: x -> B^aT x), evaluated in x87 extended precision (np.longdouble).

    Same definition as construction 2, B^a = I T^{-1}, with T^{-1} from App. B
    (eq:ak=3) and I from eq:intChebPoly=; the factors are applied one after the other
    (X T^{-T} I^T, or X I T^{-1}) so the dense B^a is never rounded to double.  Used as
    the product reference where the double-precision dense matrix is itself only good
    to ~1e-12 relative (N in the thousands).  Cost O(N^2) per row plus O(N^2) set-up.
    """
    return _apply_Ba_ld(N, X, transpose).astype(np.float64)


def _apply_Ba_ld(N: int, X: np.ndarray, transpose: bool) -> np.ndarray:
    ld = np.longdouble
    X = np.atleast_2d(np.asarray(X, dtype=np.float64)).astype(ld)
    Tinv, Int = _extended_factors(N)
    if transpose:
        return (X @ Int) @ Tinv
    return (X @ Tinv.T) @ Int.T


@functools.lru_cache(maxsize=1)
def _extended_factors(N: int):
    ld = np.longdouble
    pi = ld(4) * np.arctan(ld(1))
    j = np.arange(N + 1, dtype=np.int64)
    k = np.arange(N + 2, dtype=np.int64)
    # T_m(tau_j) for m = 0..N+1 (column N+1 feeds the antiderivative of T_N)
    Tm = np.cos(pi * ((k[None, :] * (N - j[:, None])) % (2 * N)).astype(ld) / ld(N))
    c = np.ones(N + 1, dtype=ld)
    c[0] = c[N] = ld(2)
    e = np.ones(N + 1, dtype=ld)
    e[0] = e[N] = ld(0.5)
    Tinv = (ld(2) / ld(N)) * (Tm[:, :N + 1].T / c[:, None]) * e[None, :]   # [k, j]
    Int = np.empty((N + 1, N + 1), dtype=ld)                              # [i, k]
    Int[:, 0] = Tm[:, 1] + ld(1)
    Int[:, 1] = Tm[:, 2] / ld(4) - ld(0.25)
    kk = np.arange(2, N + 1)
    sgn = np.where(kk % 2 == 0, ld(1), ld(-1))
    Int[:, 2:] = (Tm[:, 3:N + 2] / (ld(2) * (kk + 1).astype(ld))
                  - Tm[:, 1:N] / (ld(2) * (kk - 1).astype(ld))
                  - sgn / (kk.astype(ld) ** 2 - ld(1)))
    return Tinv, Int


# ------------------------------------------------------------------------ b-form
def dense_Bb_quadrature(N: int) -> np.ndarray:
    """B^b from its own conditions (eq:xN=Birka+b, eq:birk-conditions with the anchor at
    tau = +1): B_j^b(1) = 0 and dB_j^b/dtau(tau_i) = delta_ij, so
    [B^b]_ij = -integral_{tau_i}^{1} l_j.

    Gauss-Legendre quadrature with N//2 + 2 points on [tau_i, 1], exact for the
    degree-N integrand; independent of B^a and of the CC weights.  Cost O(N^3).
    """
    tau = cgl_nodes(N)
    nq = N // 2 + 2
    t, wq = np.polynomial.legendre.leggauss(nq)
    B = np.zeros((N + 1, N + 1))
    for i in range(N):
        half = 0.5 * (1.0 - tau[i])
        x = tau[i] + half * (t + 1.0)
        B[i] = -half * (wq @ lagrange_basis(N, x))
    return B


def dense_Bb(N: int) -> np.ndarray:
    """Dense B^b = B^a - 1 w_B^T: B_j^b and B_j^a share their derivative at the nodes
    and B_j^b vanishes at +1, so B_j^b = B_j^a - B_j^a(1), and B_j^a(1) = (w_B)_j."""
    return dense_Ba(N) - np.outer(np.ones(N + 1), weights(N))


def sparse_mode_exact_b(N: int, modes, alphas) -> np.ndarray:
    """Exact B^b v for v = sum_s alpha_s T_{k_s} (k_s <= N): the antiderivative of the
    series anchored at +1, integral_{1}^{tau_j} v = I(tau_j) - I(1) with I from
    eq:intChebPoly= (tau_N = 1).  Cost O(len(modes) * N)."""
    full = sparse_mode_exact(N, modes, alphas)
    return full - full[N]


def apply_Bb_extended(N: int, X: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Rows of X times B^b^T (transpose=False: x -> B^b x) or times B^b (transpose=True:
    x -> B^bT x) in x87 extended precision.

    B^b x = B^a x - 1 (w_B^T x), and w_B^T x is the last entry of B^a x;
    B^bT g = B^aT g - w_B (1^T g), with w_B = B^aT e_N.  Both from the extended
    factors of apply_Ba_extended, rounded to double once at the end.
    """
    ld = np.longdouble
    Y = _apply_Ba_ld(N, X, transpose)
    if not transpose:
        return (Y - Y[:, N:N + 1]).astype(np.float64)
    e_N = np.zeros((1, N + 1))
    e_N[0, N] = 1.0
    w = _apply_Ba_ld(N, e_N, True)[0]
    Xl = np.atleast_2d(np.asarray(X, dtype=np.float64)).astype(ld)
    return (Y - Xl.sum(axis=1, keepdims=True) * w[None, :]).astype(np.float64)


def endpoint_b(N: int, xa: np.ndarray, V: np.ndarray) -> np.ndarray:
    """x^b = x^a + w_B^T V per component (eq:Prob-PNa): xa has shape (n_x,), V has
    shape (n_x, N + 1); the weights are the last row of B^a."""
    V = np.atleast_2d(np.asarray(V, dtype=np.float64))
    return np.asarray(xa, dtype=np.float64) + V @ weights(N)
