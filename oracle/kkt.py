"""A symmetric saddle-point (KKT) form of the collocated linear system, and MINRES.

Test infrastructure only (see the package docstring).  Float64 throughout.

The paper's orbit-transfer runs count "matrix-free KKT solves" per SQP iteration
(Table 1 and the results section on the low-thrust transfer) but do not write the KKT
system down.  Reading used here (state-only setting of eq:Newton-ivp): the equality-
constrained quadratic model of one SQP step,

    minimise   1/2 (chi - chi_r)^T H (chi - chi_r)   subject to   A chi = g,

with the collocation constraints A = I - (I (x) B^a) blockdiag(J_k) of eq:Newton-ivp and a
positive diagonal Hessian model H = diag(h).  Its optimality conditions are the KKT system

    [ H   A^T ] [ chi    ]   [ f ]
    [ A   0   ] [ lambda ] = [ g ],      f = H chi_r,

symmetric and indefinite (n positive and n negative eigenvalues when A is invertible), so
MINRES (Paige and Saunders, 1975) applies.  Its preconditioner must be symmetric positive
definite; here the block-diagonal M = blockdiag(H, P H^{-1} P^T) with the Birkhoff
preconditioner P = I - B~^a J of the paper standing in for A in the Schur complement
A H^{-1} A^T.  Applying M^{-1} needs P^{-T}, which is backward substitution with P^T.
"""

from __future__ import annotations

import numpy as np

from . import birkhoff as bk
from . import system as sy

__all__ = [
    "dense_K",
    "kkt_solve_dense",
    "kkt_solve_by_elimination",
    "precond_transpose_inverse",
    "kkt_precond_apply",
    "kkt_apply",
    "minres",
]


def dense_K(N: int, J: np.ndarray, h: np.ndarray, Ba: np.ndarray | None = None) -> np.ndarray:
    """The 2n x 2n KKT matrix [[diag(h), A^T], [A, 0]] with A of eq:Newton-ivp."""
    A = sy.dense_A(N, J, Ba)
    n = A.shape[0]
    K = np.zeros((2 * n, 2 * n))
    K[:n, :n] = np.diag(np.asarray(h, dtype=np.float64))
    K[:n, n:] = A.T
    K[n:, :n] = A
    return K


def kkt_solve_dense(K: np.ndarray, f: np.ndarray, g: np.ndarray):
    """(chi, lambda) from a dense LU solve of the KKT system."""
    n = f.shape[0]
    z = np.linalg.solve(K, np.concatenate([f, g]))
    return z[:n], z[n:]


def kkt_solve_by_elimination(A: np.ndarray, h: np.ndarray, f: np.ndarray, g: np.ndarray):
    """The same solution without the saddle-point matrix: A square and invertible fixes
    chi = A^{-1} g through the constraint, and the first block row gives
    lambda = A^{-T} (f - H chi)."""
    chi = np.linalg.solve(A, g)
    lam = np.linalg.solve(A.T, f - h * chi)
    return chi, lam


def precond_transpose_inverse(w: np.ndarray, J: np.ndarray, y: np.ndarray) -> np.ndarray:
    """P^{-T} y by block backward substitution with P^T, O(N n_x^3).

    P = I - (B~^a (x) I) J has block (k, j) = delta_kj I - B~_kj J_j (B~ from the weights,
    Sec. on B~^a), so P^T has block (j, k) = delta_jk I - B~_kj J_j^T: upper triangular in
    node order.  Row j of P^T x = y reads
        (I - w_j J_j^T / 2) x_j - w_j J_j^T sum_{k>j} x_k = y_j,
    solved from the last node down with the running sum T_j = sum_{k>j} x_k."""
    N_n = w.shape[0]
    Jf = sy.expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    Y = y.reshape(n_x, N_n)
    X = np.zeros_like(Y)
    T = np.zeros(n_x)
    I = np.eye(n_x)
    for j in range(N_n - 1, -1, -1):
        JT = Jf[:, :, j].T
        xj = np.linalg.solve(I - 0.5 * w[j] * JT, Y[:, j] + w[j] * (JT @ T))
        X[:, j] = xj
        T = T + xj
    return X.reshape(-1)


def kkt_precond_apply(w: np.ndarray, J: np.ndarray, h: np.ndarray, r: np.ndarray) -> np.ndarray:
    """M^{-1} r for M = blockdiag(H, P H^{-1} P^T): [r1 / h ; P^{-T} (h * P^{-1} r2)]."""
    n = r.shape[0] // 2
    top = r[:n] / h
    bot = precond_transpose_inverse(w, J, h * sy.precond_inverse(w, J, r[n:]))
    return np.concatenate([top, bot])


def kkt_apply(Ba: np.ndarray, J: np.ndarray, h: np.ndarray, z: np.ndarray) -> np.ndarray:
    """K z = [h chi + A^T lambda ; A chi] with A applied factor by factor (densely)."""
    N_n = Ba.shape[0]
    n = z.shape[0] // 2
    chi, lam = z[:n], z[n:]
    Jf = sy.expand_jacobian(J, N_n)
    n_x = Jf.shape[0]
    # A^T lambda = lambda - blockdiag(J)^T (I (x) B^aT) lambda
    BTl = (lam.reshape(n_x, N_n) @ Ba)                       # B^aT per component
    JTBTl = np.einsum("crk,ck->rk", Jf, BTl).reshape(-1)     # J_k^T per node
    return np.concatenate([h * chi + lam - JTBTl, sy.apply_A(Ba, J, chi)])


def minres(matvec, prec, b: np.ndarray, tol: float = 1e-12, max_iter: int = 500):
    """Preconditioned MINRES for a symmetric (possibly indefinite) operator with a symmetric
    positive definite preconditioner prec ~ operator^{-1}.

    The Lanczos process on the preconditioned operator builds v_k with the three-term
    recurrence; each new tridiagonal column is reduced by the previous two Givens
    rotations and a new one, whose sines and cosines update the solution along the
    directions w_k = (v_k - eps_k w_{k-2} - delta_k w_{k-1}) / gamma_k.  phibar is the
    preconditioned residual norm sqrt(r^T M^{-1} r); the iteration stops when it falls
    below tol times its initial value.  Returns (x, iterations, [phibar after each step])."""
    n = b.shape[0]
    x = np.zeros(n)
    r1 = b.copy()
    y = prec(r1)
    beta1 = float(np.sqrt(r1 @ y))
    if beta1 == 0.0:
        return x, 0, [0.0]
    r2 = r1.copy()
    w = np.zeros(n)
    w2 = np.zeros(n)
    oldb, beta = 0.0, beta1
    dbar, eps = 0.0, 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    hist = [phibar]
    for it in range(1, max_iter + 1):
        v = y / beta
        y = matvec(v)
        if it >= 2:
            y = y - (beta / oldb) * r1
        alpha = float(v @ y)
        y = y - (alpha / beta) * r2
        r1, r2 = r2, y
        y = prec(r2)
        oldb = beta
        beta = float(np.sqrt(r2 @ y))
        oldeps = eps
        delta = cs * dbar + sn * alpha
        gbar = sn * dbar - cs * alpha
        eps = sn * beta
        dbar = -cs * beta
        gamma = float(np.hypot(gbar, beta))
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        hist.append(abs(phibar))
        if abs(phibar) <= tol * beta1:
            return x, it, hist
    return x, max_iter, hist
