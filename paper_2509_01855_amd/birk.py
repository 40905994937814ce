"""Python binding of libbirk (the C ABI declared in include/birk.h).

Argument marshalling only: every computation runs in the HIP library.  The functions
keep the C names (birk_plan_create, birk_apply, ...).  Vectors are torch tensors on the
plan's GPU (contiguous, in the plan's storage dtype); PyTorch supplies device memory and
the stream, nothing else.  If the shared library has not been built, importing this
module raises ImportError: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbirk.so")

BIRK_OK = 0
BIRK_ERR_ARG = -1
BIRK_ERR_SIZE = -2
BIRK_ERR_DEVICE = -3
BIRK_ERR_NOMEM = -4
BIRK_ERR_SINGULAR = -5
BIRK_ERR_NOCONV = -6
BIRK_ERR_BREAKDOWN = -7
BIRK_ERR_NONFINITE = -8
BIRK_ERR_UNSUPPORTED = -9

BIRK_F64 = 0
BIRK_F32 = 1
BIRK_F32_REFINE_F64 = 2
BIRK_DF32 = 3

BIRK_J_CONSTANT = 0
BIRK_J_PER_NODE = 1

EXPORTED = [
    "birk_plan_create", "birk_plan_destroy", "birk_plan_length", "birk_plan_tune", "birk_plan_set_graphs",
    "birk_weights",
    "birk_apply", "birk_apply_T", "birk_apply_noalloc", "birk_apply_b", "birk_apply_bT", "birk_endpoint", "birk_precond",
    "birk_fast_ax",
    "birk_solve_opts_default", "birk_krylov_solve", "birk_kkt_solve", "birk_status_string",
    "birk_two_body", "birk_newton_opts_default", "birk_newton_ivp",
]

BIRK_MODEL_TWO_BODY = 0
BIRK_MODEL_CALLBACK = 1

# birk_rhs_fn: (ctx, X, F, J, hip_stream) -> birk_status
RHS_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p)


class birk_solve_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("use_precond", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("inner_rtol", ctypes.c_double)]


class birk_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.POINTER(ctypes.c_int32)),
                ("inner_iters", ctypes.POINTER(ctypes.c_int32)),
                ("outer_iters", ctypes.POINTER(ctypes.c_int32)),
                ("rel_resid_fp64", ctypes.POINTER(ctypes.c_double))]


class birk_ivp_model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("mu", ctypes.c_double), ("scale", ctypes.c_double),
                ("fn", RHS_FN), ("ctx", ctypes.c_void_p)]


class birk_newton_opts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int32), ("tol", ctypes.c_double), ("line_search", ctypes.c_int32),
                ("linear", birk_solve_opts)]


class birk_newton_info(ctypes.Structure):
    _fields_ = [("status", ctypes.POINTER(ctypes.c_int32)),
                ("newton_iters", ctypes.POINTER(ctypes.c_int32)),
                ("linear_iters", ctypes.POINTER(ctypes.c_int32)),
                ("rel_resid", ctypes.POINTER(ctypes.c_double))]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2509_01855_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.birk_plan_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i64), ctypes.POINTER(i32), i32, vp]
    lib.birk_plan_destroy.argtypes = [vp]
    lib.birk_plan_length.argtypes = [vp]
    lib.birk_plan_length.restype = i64
    lib.birk_plan_tune.argtypes = [vp, ctypes.c_char_p, i64]
    lib.birk_plan_set_graphs.argtypes = [vp, i32]
    lib.birk_weights.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    lib.birk_apply.argtypes = [vp, vp, vp]
    lib.birk_apply_T.argtypes = [vp, vp, vp]
    lib.birk_apply_noalloc.argtypes = [vp, vp, vp, i32]
    lib.birk_apply_b.argtypes = [vp, vp, vp]
    lib.birk_apply_bT.argtypes = [vp, vp, vp]
    lib.birk_endpoint.argtypes = [vp, vp, vp, vp]
    lib.birk_precond.argtypes = [vp, i32, vp, vp, vp, i32]
    lib.birk_fast_ax.argtypes = [vp, i32, vp, vp, vp]
    lib.birk_solve_opts_default.argtypes = [ctypes.POINTER(birk_solve_opts)]
    lib.birk_solve_opts_default.restype = None
    lib.birk_krylov_solve.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(birk_solve_opts),
                                      ctypes.POINTER(birk_solve_info)]
    lib.birk_kkt_solve.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(birk_solve_opts),
                                   ctypes.POINTER(birk_solve_info)]
    lib.birk_two_body.argtypes = [vp, dbl, dbl, vp, vp, vp]
    lib.birk_newton_opts_default.argtypes = [ctypes.POINTER(birk_newton_opts)]
    lib.birk_newton_opts_default.restype = None
    lib.birk_newton_ivp.argtypes = [vp, ctypes.POINTER(birk_ivp_model), vp, vp, ctypes.POINTER(birk_newton_opts),
                                    ctypes.POINTER(birk_newton_info)]
    lib.birk_status_string.argtypes = [i32]
    lib.birk_status_string.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("birk_plan_length", "birk_solve_opts_default", "birk_newton_opts_default",
                        "birk_status_string"):
            getattr(lib, name).restype = i32
    return lib


_lib = _load()


class BirkError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__(f"{where}: {birk_status_string(status)}")


def birk_status_string(status: int) -> str:
    return _lib.birk_status_string(int(status)).decode()


def _check(st: int, where: str) -> None:
    if st != BIRK_OK:
        raise BirkError(st, where)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


# ---- argument checks: every tensor handed to the library is checked for type, dtype,
# length and contiguity, then all of them for their device, then for overlaps, before the
# call; a wrong tensor is a Python error here and never an out-of-bounds access on the GPU.
def _spec_vec(plan: Plan, t, name: str):
    """A vector in the plan's storage type and layout (birk_plan_length elements; double-
    float plans store two floats per element)."""
    if plan.prec == BIRK_F64:
        return (t, name, "f64", plan.length, False)
    if plan.prec == BIRK_DF32:
        return (t, name, "f32", 2 * plan.length, False)
    return (t, name, "f32", plan.length, False)


def _spec_f64(plan: Plan, t, name: str, numel: int = None, allow_none: bool = False):
    """A double array: by default one value per element of the plan layout."""
    return (t, name, "f64", plan.length if numel is None else numel, allow_none)


def _jac_numel(plan: Plan, jac_kind: int) -> int:
    if jac_kind == BIRK_J_CONSTANT:
        return sum(nx * nx for nx in plan.n_x)
    if jac_kind == BIRK_J_PER_NODE:
        return sum(nx * nx * nn for nn, nx in zip(plan.n_nodes, plan.n_x))
    raise ValueError(f"jac_kind must be BIRK_J_CONSTANT or BIRK_J_PER_NODE, got {jac_kind}")


def _spec_jac(plan: Plan, J, jac_kind: int):
    return (J, "J", "f64", _jac_numel(plan, jac_kind), False)


def _validate(plan: Plan, *specs, disjoint=()) -> None:
    """specs: (tensor, name, dtype, numel, allow_none).  disjoint: pairs of names whose
    storage must not overlap."""
    import torch
    present = {}
    for t, name, dtype, numel, allow_none in specs:
        if t is None:
            if allow_none:
                continue
            raise ValueError(f"{name}: a tensor is required")
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
        want = {"f64": torch.float64, "f32": torch.float32}[dtype]
        if t.dtype != want:
            raise ValueError(f"{name}: dtype {t.dtype}, the plan needs {want}")
        if t.numel() != numel:
            raise ValueError(f"{name}: {t.numel()} elements, the plan needs {numel}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        present[name] = t
    for a, b in disjoint:
        if a in present and b in present:
            ta, tb = present[a], present[b]
            a0, b0 = ta.data_ptr(), tb.data_ptr()
            if a0 < b0 + tb.numel() * tb.element_size() and b0 < a0 + ta.numel() * ta.element_size():
                raise ValueError(f"{a} and {b} overlap")
    for name, t in present.items():
        if not t.is_cuda or t.device.index != plan.device:
            raise ValueError(f"{name}: must live on cuda:{plan.device} (got {t.device})")


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


@dataclass
class Plan:
    """Owning handle of a birk_plan, with the sizes the argument checks need."""
    handle: int
    n_nodes: tuple
    n_x: tuple
    prec: int
    device: int = 0

    @property
    def length(self) -> int:
        return sum(a * b for a, b in zip(self.n_nodes, self.n_x))

    @property
    def n_comp(self) -> int:
        return sum(self.n_x)

    def destroy(self) -> None:
        if self.handle:
            _lib.birk_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def birk_plan_create(n_nodes, n_x, prec: int = BIRK_F64, stream=None) -> Plan:
    n_nodes = [int(v) for v in n_nodes]
    n_x = [int(v) for v in n_x]
    if len(n_nodes) != len(n_x):
        raise ValueError("n_nodes and n_x must have the same length")
    b = len(n_nodes)
    nn = (ctypes.c_int64 * max(b, 1))(*n_nodes)
    nx = (ctypes.c_int32 * max(b, 1))(*n_x)
    h = ctypes.c_void_p()
    import torch
    dev = torch.cuda.current_device()
    st = _lib.birk_plan_create(ctypes.byref(h), b, nn, nx, int(prec), _stream_handle(stream))
    _check(st, "birk_plan_create")
    return Plan(h.value, tuple(n_nodes), tuple(n_x), int(prec), int(dev))


def birk_plan_destroy(plan: Plan) -> None:
    plan.destroy()


def birk_plan_length(plan: Plan) -> int:
    return int(_lib.birk_plan_length(plan.handle))


def birk_plan_tune(plan: Plan) -> str:
    """Run the autotuner of the product schedules (power-of-two groups, then the
    Bluestein two-step splits); returns its report."""
    buf = ctypes.create_string_buffer(16384)
    _check(_lib.birk_plan_tune(plan.handle, buf, len(buf)), "birk_plan_tune")
    return buf.value.decode()


def birk_plan_set_graphs(plan: Plan, enable: bool = True) -> None:
    """Replay birk_apply / birk_apply_T from recorded HIP graphs (see include/birk.h)."""
    _check(_lib.birk_plan_set_graphs(plan.handle, 1 if enable else 0), "birk_plan_set_graphs")


def birk_weights(plan: Plan, inst: int = 0):
    import numpy as np
    w = np.empty(plan.n_nodes[inst], dtype=np.float64)
    _check(_lib.birk_weights(plan.handle, int(inst), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "birk_weights")
    return w


def _product_args(plan: Plan, v, out, vname: str) -> None:
    _validate(plan, _spec_vec(plan, v, vname), _spec_vec(plan, out, "out"), disjoint=[(vname, "out")])


def birk_apply(plan: Plan, v, out) -> None:
    _product_args(plan, v, out, "v")
    _check(_lib.birk_apply(plan.handle, _ptr(v), _ptr(out)), "birk_apply")


def birk_apply_T(plan: Plan, g, out) -> None:
    _product_args(plan, g, out, "g")
    _check(_lib.birk_apply_T(plan.handle, _ptr(g), _ptr(out)), "birk_apply_T")


def birk_apply_noalloc(plan: Plan, v, out, transpose: bool = False) -> None:
    """birk_apply (or birk_apply_T) with the library's fixed device workspace; allocates nothing."""
    _product_args(plan, v, out, "v")
    _check(_lib.birk_apply_noalloc(plan.handle, _ptr(v), _ptr(out), int(bool(transpose))), "birk_apply_noalloc")


def birk_apply_b(plan: Plan, v, out) -> None:
    _product_args(plan, v, out, "v")
    _check(_lib.birk_apply_b(plan.handle, _ptr(v), _ptr(out)), "birk_apply_b")


def birk_apply_bT(plan: Plan, g, out) -> None:
    _product_args(plan, g, out, "g")
    _check(_lib.birk_apply_bT(plan.handle, _ptr(g), _ptr(out)), "birk_apply_bT")


def birk_endpoint(plan: Plan, xa, v, xb) -> None:
    """xb = xa + w^T v per component (device double arrays of one entry per component)."""
    _validate(plan, _spec_f64(plan, xa, "xa", plan.n_comp), _spec_vec(plan, v, "v"),
              _spec_f64(plan, xb, "xb", plan.n_comp), disjoint=[("xa", "v"), ("xb", "v")])
    _check(_lib.birk_endpoint(plan.handle, _ptr(xa), _ptr(v), _ptr(xb)), "birk_endpoint")


def birk_precond(plan: Plan, J, y, out, inverse, jac_kind: int = BIRK_J_PER_NODE) -> None:
    """inverse: 0 (or False) P y, 1 (or True) P^{-1} y, 2 P^{-T} y."""
    _validate(plan, _spec_jac(plan, J, jac_kind), _spec_vec(plan, y, "y"), _spec_vec(plan, out, "out"),
              disjoint=[("y", "out"), ("J", "out")])
    _check(_lib.birk_precond(plan.handle, int(jac_kind), _ptr(J), _ptr(y), _ptr(out), int(inverse)),
           "birk_precond")


def birk_fast_ax(plan: Plan, J, x, out, jac_kind: int = BIRK_J_PER_NODE) -> None:
    _validate(plan, _spec_jac(plan, J, jac_kind), _spec_f64(plan, x, "x"), _spec_f64(plan, out, "out"),
              disjoint=[("x", "out"), ("J", "out")])
    _check(_lib.birk_fast_ax(plan.handle, int(jac_kind), _ptr(J), _ptr(x), _ptr(out)), "birk_fast_ax")


def birk_solve_opts_default() -> birk_solve_opts:
    o = birk_solve_opts()
    _lib.birk_solve_opts_default(ctypes.byref(o))
    return o


def birk_krylov_solve(plan: Plan, J, beta, chi, jac_kind: int = BIRK_J_PER_NODE, raise_on_error: bool = True,
                      **opts):
    """Solve [I - B^a J] chi = beta; returns a dict with per-instance status, iteration counts
    and final double-precision relative residuals."""
    o = birk_solve_opts_default()
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    _validate(plan, _spec_jac(plan, J, jac_kind), _spec_f64(plan, beta, "beta"), _spec_f64(plan, chi, "chi"),
              disjoint=[("beta", "chi"), ("J", "chi")])
    b = len(plan.n_nodes)
    stv = (ctypes.c_int32 * b)()
    inner = (ctypes.c_int32 * b)()
    outer = (ctypes.c_int32 * b)()
    res = (ctypes.c_double * b)()
    info = birk_solve_info(stv, inner, outer, res)
    st = _lib.birk_krylov_solve(plan.handle, int(jac_kind), _ptr(J), _ptr(beta), _ptr(chi), ctypes.byref(o),
                                ctypes.byref(info))
    out = {"status": int(st), "inst_status": list(stv), "inner_iters": list(inner),
           "outer_iters": list(outer), "rel_resid": list(res)}
    if raise_on_error and st != BIRK_OK:
        raise BirkError(st, "birk_krylov_solve")
    return out


def birk_kkt_solve(plan: Plan, J, g, chi, lam=None, h=None, f=None, jac_kind: int = BIRK_J_PER_NODE,
                   raise_on_error: bool = True, **opts):
    """MINRES on [[diag(h), A^T], [A, 0]] [chi; lam] = [f; g] (h None: identity, f None: zero,
    lam None: the multipliers are not returned).  Returns a dict like birk_krylov_solve."""
    o = birk_solve_opts_default()
    o.method = 1
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    _validate(plan, _spec_jac(plan, J, jac_kind), _spec_f64(plan, g, "g"), _spec_f64(plan, chi, "chi"),
              _spec_f64(plan, lam, "lam", allow_none=True), _spec_f64(plan, h, "h", allow_none=True),
              _spec_f64(plan, f, "f", allow_none=True),
              disjoint=[(a, b) for a in ("chi", "lam") for b in ("J", "g", "h", "f")] + [("chi", "lam")])
    b = len(plan.n_nodes)
    stv = (ctypes.c_int32 * b)()
    inner = (ctypes.c_int32 * b)()
    outer = (ctypes.c_int32 * b)()
    res = (ctypes.c_double * b)()
    info = birk_solve_info(stv, inner, outer, res)
    st = _lib.birk_kkt_solve(plan.handle, int(jac_kind), _ptr(J), _ptr(h), _ptr(f), _ptr(g), _ptr(chi), _ptr(lam),
                             ctypes.byref(o), ctypes.byref(info))
    out = {"status": int(st), "inst_status": list(stv), "inner_iters": list(inner),
           "outer_iters": list(outer), "rel_resid": list(res)}
    if raise_on_error and st != BIRK_OK:
        raise BirkError(st, "birk_kkt_solve")
    return out


def birk_two_body(plan: Plan, X, F, J, mu: float = 1.0, scale: float = 1.0) -> None:
    """Two-body right-hand side F and per-node Jacobian J at X (F or J may be None)."""
    _validate(plan, _spec_f64(plan, X, "X"), _spec_f64(plan, F, "F", allow_none=True),
              _spec_f64(plan, J, "J", _jac_numel(plan, BIRK_J_PER_NODE), allow_none=True),
              disjoint=[("X", "F"), ("X", "J"), ("F", "J")])
    _check(_lib.birk_two_body(plan.handle, float(mu), float(scale), _ptr(X), _ptr(F), _ptr(J)), "birk_two_body")


def birk_newton_opts_default() -> birk_newton_opts:
    o = birk_newton_opts()
    _lib.birk_newton_opts_default(ctypes.byref(o))
    return o


def birk_newton_ivp(plan: Plan, xa, X, mu: float = 1.0, scale: float = 1.0, rhs=None, raise_on_error: bool = True,
                    linear=None, **opts):
    """Newton's method on X - x^a b - B^a f(X) = 0.  With rhs=None the built-in two-body model
    (mu, scale); otherwise rhs(X_ptr, F_ptr, J_ptr, stream_ptr) -> birk_status is called to
    evaluate f (and df/dx when J_ptr is not 0).  linear: dict of birk_solve_opts fields for the
    Newton systems.  Returns a dict with per-instance status, Newton and Krylov iteration
    counts and final ||G|| / ||X||."""
    o = birk_newton_opts_default()
    for k, v in opts.items():
        if k == "linear" or not hasattr(o, k):
            raise TypeError(f"unknown Newton option {k}")
        setattr(o, k, v)
    for k, v in (linear or {}).items():
        if not hasattr(o.linear, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o.linear, k, v)
    if rhs is None:
        model = birk_ivp_model(BIRK_MODEL_TWO_BODY, float(mu), float(scale), RHS_FN(), None)
        cb = None
    else:
        cb = RHS_FN(lambda ctx, x, f, j, stream: int(rhs(x or 0, f or 0, j or 0, stream or 0)))
        model = birk_ivp_model(BIRK_MODEL_CALLBACK, 0.0, 0.0, cb, None)
    _validate(plan, _spec_f64(plan, xa, "xa", plan.n_comp), _spec_f64(plan, X, "X"), disjoint=[("xa", "X")])
    b = len(plan.n_nodes)
    stv = (ctypes.c_int32 * b)()
    nit = (ctypes.c_int32 * b)()
    lit = (ctypes.c_int32 * b)()
    res = (ctypes.c_double * b)()
    info = birk_newton_info(stv, nit, lit, res)
    st = _lib.birk_newton_ivp(plan.handle, ctypes.byref(model), _ptr(xa), _ptr(X), ctypes.byref(o),
                              ctypes.byref(info))
    del cb
    out = {"status": int(st), "inst_status": list(stv), "newton_iters": list(nit), "linear_iters": list(lit),
           "rel_resid": list(res)}
    if raise_on_error and st != BIRK_OK:
        raise BirkError(st, "birk_newton_ivp")
    return out
