"""Seeded synthetic inputs for the Birkhoff products and the linearised-dynamics solve.

This module holds input generation only: random vectors, LTI system matrices, and the
Jacobian of the two-body problem along a Keplerian orbit evaluated at the grid times.
None of the fast method's arithmetic (transforms, integration recurrence, weights,
preconditioner, Krylov) is here.  Both the GPU path and the FP64 oracle are fed the
same float64 arrays produced by these functions.

Workloads (shapes of the paper's astrodynamics problem, sizes as named in the
benchmark configuration list):

* ``lti``      -- n_x = 6 states, A = randn(6, 6)/sqrt(6) - 2 I, x_a ~ N(0, 1),
                  constant Jacobian (N_n = 256, 4097, 65537, ...).
* ``kepler``   -- n_x = 6 states (r, v), time-varying J(t) = [[0, I], [G(r(t)), 0]],
                  G(r) = (3 r^ r^T - I)/|r|^3, canonical units (mu = 1, semi-major axis
                  a = 1 standing for 7000 km, period T = 2 pi), e ~ U(0, 0.2), orbit plane
                  from a seeded uniform rotation, periapsis at the left end point.
                  The time map t = (tau + 1) T / 2 contributes the factor T/2, which is
                  folded into J.
* ``batched``  -- independent LTI instances with N_n = round(2^U(8, 16)) and
                  n_x uniform in {4, 6, 12}.
* ``sparse_modes`` -- random Chebyshev mode sets used for exact checks at large N.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "grid_times",
    "lti_matrix",
    "lti_instance",
    "kepler_orbit",
    "kepler_jacobian",
    "kepler_instance",
    "batched_instances",
    "sparse_modes",
    "sparse_series",
    "node_sparse",
    "random_vectors",
    "kepler_ivp",
    "Instance",
]


def grid_times(N: int) -> np.ndarray:
    """Normalised time points -cos(j pi / N), j = 0..N, at which J is sampled.

    Evaluated as sin(pi (2j - N) / (2N)) so that the ends are exactly -1 and +1.
    """
    j = np.arange(N + 1, dtype=np.float64)
    return np.sin(np.pi * (2.0 * j - N) / (2.0 * N))


def lti_matrix(rng: np.random.Generator, n_x: int) -> np.ndarray:
    """A = randn(n_x, n_x)/sqrt(n_x) - 2 I (a stable random linear system)."""
    return rng.standard_normal((n_x, n_x)) / math.sqrt(n_x) - 2.0 * np.eye(n_x)


@dataclass
class Instance:
    """One linear system [I - B^a J] X = x_a b on N_n nodes with n_x states."""

    N_n: int
    n_x: int
    J: np.ndarray                 # (n_x, n_x) constant or (n_x, n_x, N_n) per node
    x_a: np.ndarray               # (n_x,)
    per_node: bool
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.N_n - 1

    @property
    def n(self) -> int:
        return self.N_n * self.n_x


def lti_instance(seed, N_n: int, n_x: int = 6) -> Instance:
    rng = np.random.default_rng(seed)
    A = lti_matrix(rng, n_x)
    x_a = rng.standard_normal(n_x)
    return Instance(N_n=N_n, n_x=n_x, J=A, x_a=x_a, per_node=False)


def random_vectors(seed, shape, count: int = 1):
    """`count` standard-normal float64 arrays of the given shape from one seeded stream."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) for _ in range(count)]


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _solve_kepler(M: np.ndarray, e: float) -> np.ndarray:
    """Eccentric anomaly E from E - e sin E = M by Newton's method to ~1e-15."""
    E = M + e * np.sin(M)
    for _ in range(50):
        f = E - e * np.sin(E) - M
        d = f / (1.0 - e * np.cos(E))
        E = E - d
        if np.max(np.abs(d)) < 1e-15:
            break
    return E


def kepler_orbit(t: np.ndarray, e: float, R: np.ndarray):
    """Position, velocity and acceleration at times t (mu = a = 1, periapsis at t = 0)."""
    E = _solve_kepler(t, e)
    cE, sE = np.cos(E), np.sin(E)
    b = math.sqrt(1.0 - e * e)
    denom = 1.0 - e * cE
    r_pf = np.stack([cE - e, b * sE, np.zeros_like(E)])
    v_pf = np.stack([-sE / denom, b * cE / denom, np.zeros_like(E)])
    r = R @ r_pf
    v = R @ v_pf
    rn = np.linalg.norm(r, axis=0)
    acc = -r / rn ** 3
    return r, v, acc


def kepler_jacobian(r: np.ndarray, scale: float) -> np.ndarray:
    """Per-node Jacobian scale * [[0, I], [G(r), 0]], G = (3 r^ r^T - I)/|r|^3; (6, 6, N_n)."""
    N_n = r.shape[1]
    rn = np.linalg.norm(r, axis=0)
    rh = r / rn
    J = np.zeros((6, 6, N_n))
    for i in range(3):
        J[i, 3 + i] = scale
        for j in range(3):
            J[3 + i, j] = scale * (3.0 * rh[i] * rh[j] - (1.0 if i == j else 0.0)) / rn ** 3
    return J


def kepler_instance(seed, N_n: int, e: float | None = None) -> Instance:
    """Linearised two-body dynamics along one period of a seeded Keplerian orbit.

    extra holds the orbit (r, v, acceleration) at the nodes and the eccentricity, from
    which the exact solutions of the linearised flow (time shift, rotation, scaling)
    can be built.
    """
    rng = np.random.default_rng(seed)
    if e is None:
        e = float(rng.uniform(0.0, 0.2))
    R = _random_rotation(rng)
    x_a = rng.standard_normal(6)
    period = 2.0 * math.pi
    tau = grid_times(N_n - 1)
    t = (tau + 1.0) * (0.5 * period)
    r, v, acc = kepler_orbit(t, e, R)
    J = kepler_jacobian(r, 0.5 * period)
    return Instance(N_n=N_n, n_x=6, J=J, x_a=x_a, per_node=True,
                    extra={"e": e, "R": R, "t": t, "r": r, "v": v, "acc": acc,
                           "period": period})


def batched_instances(count: int = 512, log2_lo: float = 8.0, log2_hi: float = 16.0,
                      nx_choices=(4, 6, 12), base_seed: int = 3):
    """`count` independent LTI instances of uneven size; instance i uses seed [base_seed, i]."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([base_seed, i])
        N_n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        N_n = max(N_n, 3)
        n_x = int(rng.choice(np.asarray(nx_choices)))
        A = lti_matrix(rng, n_x)
        x_a = rng.standard_normal(n_x)
        out.append(Instance(N_n=N_n, n_x=n_x, J=A, x_a=x_a, per_node=False))
    return out


def sparse_modes(seed, N: int, count: int = 64):
    """A random set of Chebyshev mode indices in [0, N] (always containing 0, 1, 2, N-1, N)
    with N(0, 1) amplitudes."""
    rng = np.random.default_rng(seed)
    fixed = {0, 1, 2, max(N - 1, 0), N}
    extra = max(count - len(fixed), 0)
    pool = rng.choice(np.arange(3, max(N - 1, 4)), size=min(extra, max(N - 4, 0)), replace=False) \
        if N > 4 else np.array([], dtype=np.int64)
    modes = np.array(sorted(fixed | set(int(k) for k in pool)), dtype=np.int64)
    modes = modes[modes <= N]
    alphas = rng.standard_normal(modes.shape[0])
    return modes, alphas


def sparse_series(seed, N: int, ncomp: int, count: int):
    """ncomp sparse Chebyshev series sampled on the N + 1 CGL nodes: component c takes the
    modes and amplitudes of sparse_modes([*seed, c, N], N, count) and its values
    v_j = sum_s alpha_s cos(pi k_s (N - j) / N) (the integer argument reduced exactly).
    Returns (values (ncomp, N + 1), [(modes, alphas) per component])."""
    seed = list(seed) if isinstance(seed, (list, tuple)) else [seed]
    j = np.arange(N + 1, dtype=np.int64)
    X = np.zeros((ncomp, N + 1))
    specs = []
    for c in range(ncomp):
        modes, alphas = sparse_modes([*seed, c, N], N, count=count)
        for k, a in zip(modes, alphas):
            X[c] += a * np.cos(np.pi * ((int(k) * (N - j)) % (2 * N)).astype(np.float64) / N)
        specs.append((modes, alphas))
    return X, specs


def node_sparse(seed, N: int, ncomp: int, per: int = 6):
    """ncomp vectors on N + 1 nodes, each with N(0, 1) values at `per` seeded nodes (the
    two end nodes among them) and zeros elsewhere.  Returns (values, [nodes per component])."""
    rng = np.random.default_rng(seed)
    G = np.zeros((ncomp, N + 1))
    nodes = []
    for c in range(ncomp):
        idx = np.unique(np.concatenate([[0, N], rng.integers(0, N + 1, per - 2)]))
        G[c, idx] = rng.standard_normal(idx.shape[0])
        nodes.append(idx)
    return G, nodes


def kepler_ivp(seed, N_n: int, e: float | None = None):
    """The nonlinear two-body initial value problem over one period of a seeded orbit.

    mu = a = 1, period 2 pi, time scale s = pi for tau in [-1, 1].  Returns a dict with
    the scale, mu, the initial state x_a (periapsis), the closed-form solution at the
    nodes (6, N_n) and the starting guess: the circular orbit of the same period in the
    same plane and phase.
    """
    rng = np.random.default_rng(seed)
    if e is None:
        e = float(rng.uniform(0.0, 0.2))
    R = _random_rotation(rng)
    period = 2.0 * math.pi
    tau = grid_times(N_n - 1)
    t = (tau + 1.0) * (0.5 * period)
    r, v, _ = kepler_orbit(t, e, R)
    r0, v0, _ = kepler_orbit(t, 0.0, R)
    X = np.concatenate([r, v])
    return {"scale": 0.5 * period, "mu": 1.0, "e": e, "x_a": X[:, 0].copy(), "exact": X,
            "guess": np.concatenate([r0, v0])}
