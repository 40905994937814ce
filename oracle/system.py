"""The Newton/IVP linear system, the Birkhoff preconditioner and plain solvers.

Test infrastructure only (see the package docstring).  Float64 throughout.

Vectors use the component-major layout of the library boundary: a state sequence
X with n_x components on N_n = N + 1 nodes is stored as X[r * N_n + k] (component r,
node k).  The operator of eq:Newton-ivp with vector states is the Kronecker form
A = I - (I_{n_x} (x) B^a) . blockdiag_k(J_k), where J_k = df/dx at node k
(eq:diag-partialf), and beta = x^a (x) b (eq:Achibetadef).

Paper references (arXiv 2509.01855):
* eq:Newton-ivp, eq:Achibetadef   the system A chi = beta.
* eq:rightP, eq:rightPx2          right preconditioning A P^{-1} Upsilon = beta, P chi = Upsilon.
* Sec. on B~^a                    P = I - B~^a df.
* FastPinvY box                   forward substitution for P^{-1}.  The update of the
                                  running sum printed there does not invert P; the
                                  reading used here is exact block forward substitution,
                                  xi_k = (I - w_k J_k / 2)^{-1} (y_k + S_k),
                                  S_{k+1} = S_k + w_k J_k xi_k.
* Sec. "A Preconditioned Algorithm", FastLinSol box, and the text after it: GMRES
  is the Krylov method used for the preconditioned system.
"""

from __future__ import annotations

import numpy as np

from . import birkhoff as bk

__all__ = [
    "expand_jacobian",
    "dense_jacobian",
    "dense_A",
    "dense_P",
    "beta_vector",
    "apply_A",
    "precond_apply",
    "precond_inverse_dense",
    "precond_inverse",
    "solve_dense",
    "lu_solve_textbook",
    "gmres_right",
    "rel_residual",
]


def expand_jacobian(J: np.ndarray, N_n: int) -> np.ndarray:
    """Return per-node Jacobians with shape (n_x, n_x, N_n).

    J is either constant, shape (n_x, n_x), or already per node, shape (n_x, n_x, N_n).
    """
    J = np.asarray(J, dtype=np.float64)
    if J.ndim == 2:
        return np.repeat(J[:, :, None], N_n, axis=2)
    if J.ndim == 3 and J.shape[2] == N_n:
        return J
    raise ValueError("J must have shape (n_x, n_x) or (n_x, n_x, N_n)")


def dense_jacobian(J: np.ndarray, N_n: int) -> np.ndarray:
    """blockdiag_k(J_k) as a dense n x n matrix in component-major order (eq:diag-partialf)."""
    Jf = expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    D = np.zeros((n_x * N_n, n_x * N_n))
    idx = np.arange(N_n)
    for r in range(n_x):
        for c in range(n_x):
            D[r * N_n + idx, c * N_n + idx] = Jf[r, c]
    return D


def dense_A(N: int, J: np.ndarray, Ba: np.ndarray | None = None) -> np.ndarray:
    """A = I - (I (x) B^a) blockdiag(J) (eq:Newton-ivp / eq:Achibetadef).

    Written block by block: component block (r, c) of (I (x) B^a) blockdiag(J) is B^a with
    its column k scaled by J_k[r, c], so A_rc = delta_rc I - B^a diag(J[r, c, :]).  (The
    same numbers as forming the Kronecker product and multiplying by the block-diagonal
    Jacobian: each entry of that product has a single nonzero term.)"""
    N_n = N + 1
    if Ba is None:
        Ba = bk.dense_Ba(N)
    Jf = expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    A = np.zeros((n_x * N_n, n_x * N_n))
    for r in range(n_x):
        for c in range(n_x):
            blk = A[r * N_n:(r + 1) * N_n, c * N_n:(c + 1) * N_n]
            blk -= Ba * Jf[r, c][None, :]
            if r == c:
                blk[np.diag_indices(N_n)] += 1.0
    return A


def dense_P(N: int, J: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """P = I - (I (x) B~^a) blockdiag(J) (Birkhoff preconditioner)."""
    N_n = N + 1
    if w is None:
        w = bk.weights(N)
    Jf = expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    BJ = np.kron(np.eye(n_x), bk.btilde_dense(w)) @ dense_jacobian(Jf, N_n)
    return np.eye(n_x * N_n) - BJ


def beta_vector(x_a: np.ndarray, N_n: int) -> np.ndarray:
    """beta = x^a (x) b with b = ones(N_n), component-major (eq:Achibetadef)."""
    return np.repeat(np.asarray(x_a, dtype=np.float64), N_n)


def _jx(Jf: np.ndarray, x: np.ndarray) -> np.ndarray:
    n_x, _, N_n = Jf.shape
    X = x.reshape(n_x, N_n)
    return np.einsum("rck,ck->rk", Jf, X)


def apply_A(Ba: np.ndarray, J: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x = x - B^a (J x), with a dense B^a applied per component (FastAX steps, densely)."""
    N_n = Ba.shape[0]
    Jf = expand_jacobian(J, N_n)
    y = _jx(Jf, x)
    return x - (y @ Ba.T).reshape(-1)


def precond_apply(w: np.ndarray, J: np.ndarray, x: np.ndarray) -> np.ndarray:
    """P x = x - B~^a (J x) per component, B~^a applied by its row definition."""
    N_n = w.shape[0]
    Jf = expand_jacobian(J, N_n)
    y = _jx(Jf, x)
    return x - bk.btilde_apply(w, y).reshape(-1)


def precond_inverse_dense(P: np.ndarray, y: np.ndarray, n_x: int) -> np.ndarray:
    """P^{-1} y by block forward substitution on the dense P (blocks = nodes).

    P is block lower triangular in node order; for node k,
    xi_k = P_kk^{-1} (y_k - sum_{j<k} P_kj xi_j).
    """
    N_n = P.shape[0] // n_x
    comp = np.arange(n_x) * N_n
    xi = np.zeros_like(y)
    for k in range(N_n):
        rows = comp + k
        rhs = y[rows].copy()
        if k > 0:
            prev = (comp[None, :] + np.arange(k)[:, None]).reshape(-1)
            rhs -= P[np.ix_(rows, prev)] @ xi[prev]
        xi[rows] = np.linalg.solve(P[np.ix_(rows, rows)], rhs)
    return xi


def precond_inverse(w: np.ndarray, J: np.ndarray, y: np.ndarray) -> np.ndarray:
    """P^{-1} y by forward substitution with a running sum, O(N n_x^3).

    Below the diagonal, block (k, j) of P is -w_j J_j, so the sum over earlier nodes
    is carried as S_k = sum_{j<k} w_j J_j xi_j:
        xi_k = (I - w_k J_k / 2)^{-1} (y_k + S_k),   S_{k+1} = S_k + w_k J_k xi_k.
    (FastPinvY box, with the running-sum update read as exact forward substitution.)
    """
    N_n = w.shape[0]
    Jf = expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    Y = y.reshape(n_x, N_n)
    X = np.zeros_like(Y)
    S = np.zeros(n_x)
    I = np.eye(n_x)
    for k in range(N_n):
        Jk = Jf[:, :, k]
        xk = np.linalg.solve(I - 0.5 * w[k] * Jk, Y[:, k] + S)
        X[:, k] = xk
        S = S + w[k] * (Jk @ xk)
    return X.reshape(-1)


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Dense LU with partial pivoting (LAPACK gesv)."""
    return np.linalg.solve(A, b)


def lu_solve_textbook(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Doolittle LU with partial pivoting, then forward and back substitution.

    The textbook algorithm, with each row elimination vectorised; a cross-check of the
    LAPACK solve at small sizes.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    b = np.array(b, dtype=np.float64, copy=True)
    n = A.shape[0]
    for p in range(n):
        piv = p + int(np.argmax(np.abs(A[p:, p])))
        if A[piv, p] == 0.0:
            raise np.linalg.LinAlgError("singular matrix")
        if piv != p:
            A[[p, piv]] = A[[piv, p]]
            b[[p, piv]] = b[[piv, p]]
        f = A[p + 1:, p] / A[p, p]
        A[p + 1:, p] = f
        A[p + 1:, p + 1:] -= np.outer(f, A[p, p + 1:])
    y = np.zeros(n)
    for i in range(n):
        y[i] = b[i] - A[i, :i] @ y[:i]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - A[i, i + 1:] @ x[i + 1:]) / A[i, i]
    return x


def rel_residual(matvec, b: np.ndarray, x: np.ndarray) -> float:
    """||b - A x||_2 / ||b||_2."""
    return float(np.linalg.norm(b - matvec(x)) / np.linalg.norm(b))


def gmres_right(matvec, prec_inv, b: np.ndarray, restart: int = 30, tol: float = 1e-12,
                max_iter: int = 300, x0: np.ndarray | None = None):
    """Plain right-preconditioned GMRES(m): modified Gram-Schmidt and Givens rotations.

    Solves A P^{-1} u = b, x = P^{-1} u (eq:rightPx2; Algorithm 2), starting from x0
    (zero by default).  Stops when the GMRES residual estimate falls to tol * ||b||
    and the true residual confirms it.  Returns (x, iterations, history of estimates).
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros(n), 0, [0.0]
    its = 0
    hist = []
    while True:
        r = b - matvec(x)
        rn = float(np.linalg.norm(r))
        hist.append(rn / bnorm)
        if rn <= tol * bnorm or its >= max_iter:
            return x, its, hist
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = rn
        V[0] = r / rn
        j_end = 0
        for j in range(m):
            wv = matvec(prec_inv(V[j]))
            for i in range(j + 1):
                H[i, j] = wv @ V[i]
                wv = wv - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(wv)
            if H[j + 1, j] != 0.0:
                V[j + 1] = wv / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or its >= max_iter:
                break
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:j_end]) / H[i, i]
        x = x + prec_inv(V[:j_end].T @ y)
