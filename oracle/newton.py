"""Newton's method for the nonlinear initial value problem on the Birkhoff grid.

Test infrastructure only (see the package docstring).  Float64 throughout.

The a-form discretisation of x' = f(x), x(-1) = x^a (eq:X-V=nonlin) is
    G(X) = X - x^a b - B^a V = 0,   V = f(X) node by node,
with b = ones (eq:Prob-PNa with no control).  The Newton step solves
    [I - B^a df(X)] dX = -G(X)
(eq:Newton-ivp, Jacobian per node as in eq:diag-partialf).  The paper gives the Newton
system only; the globalisation here is plain Armijo backtracking on ||G||_2 (halve the
step until ||G(X + l dX)|| <= (1 - 1e-4 l) ||G(X)||, give up below l = 2^-12), and the
iteration stops when ||G||_2 <= tol ||X||_2.  The linear systems are solved densely.

Model: the two-body problem in normalised units, state x = (r, v) in R^6 and
dx/dtau = s (v, -mu r / |r|^3), s = (t_b - t_a) / 2 the time scale of [-1, 1] (R6).
"""

from __future__ import annotations

import numpy as np

from . import birkhoff as bk
from . import system as sy

__all__ = ["two_body_rhs", "two_body_jacobian", "ivp_residual", "newton_ivp"]

ARMIJO = 1e-4
MIN_STEP = 2.0 ** -12


def two_body_rhs(X: np.ndarray, scale: float, mu: float = 1.0) -> np.ndarray:
    """f(X) node by node for X of shape (6, N_n): scale * (v, -mu r / |r|^3)."""
    r, v = X[:3], X[3:]
    rn = np.sqrt(np.sum(r * r, axis=0))
    return scale * np.concatenate([v, -mu * r / rn ** 3])


def two_body_jacobian(X: np.ndarray, scale: float, mu: float = 1.0) -> np.ndarray:
    """df/dx per node, shape (6, 6, N_n): scale * [[0, I], [mu (3 rr^T / |r|^2 - I) / |r|^3, 0]]."""
    r = X[:3]
    n = X.shape[1]
    rn = np.sqrt(np.sum(r * r, axis=0))
    J = np.zeros((6, 6, n))
    for i in range(3):
        J[i, 3 + i] = scale
        for j in range(3):
            J[3 + i, j] = scale * mu * (3.0 * r[i] * r[j] / rn ** 2 - (1.0 if i == j else 0.0)) / rn ** 3
    return J


def ivp_residual(Ba: np.ndarray, xa: np.ndarray, X: np.ndarray, F: np.ndarray) -> np.ndarray:
    """G = X - x^a b - B^a F, component by component (eq:X-V=nonlin)."""
    return X - np.asarray(xa)[:, None] - F @ Ba.T


def newton_ivp(N: int, xa: np.ndarray, X0: np.ndarray, scale: float, mu: float = 1.0,
               tol: float = 1e-13, max_iter: int = 30):
    """Solve G(X) = 0 for the two-body model from the guess X0 (shape (6, N + 1)).

    Returns (X, newton_iterations, [||G||_2 before each step and at the end],
    [accepted step length of each step]).
    Raises RuntimeError when the line search or the iteration limit fails.
    """
    Ba = bk.dense_Ba(N)
    X = np.array(X0, dtype=np.float64)
    G = ivp_residual(Ba, xa, X, two_body_rhs(X, scale, mu))
    g = float(np.linalg.norm(G))
    hist = [g]
    steps = []
    for it in range(max_iter + 1):
        if g <= tol * np.linalg.norm(X):
            return X, it, hist, steps
        if it == max_iter:
            break
        A = sy.dense_A(N, two_body_jacobian(X, scale, mu), Ba)
        dX = np.linalg.solve(A, -G.ravel()).reshape(X.shape)
        lam = 1.0
        while True:
            Xt = X + lam * dX
            Gt = ivp_residual(Ba, xa, Xt, two_body_rhs(Xt, scale, mu))
            gt = float(np.linalg.norm(Gt))
            if gt <= (1.0 - ARMIJO * lam) * g or gt <= tol * np.linalg.norm(Xt):
                break
            lam *= 0.5
            if lam < MIN_STEP:
                raise RuntimeError("line search failed")
        X, G, g = Xt, Gt, gt
        hist.append(g)
        steps.append(lam)
    raise RuntimeError("Newton iteration limit reached")
