"""Host-only checks of the C-ABI library: it loads, exports every symbol that
include/birk.h declares, and rejects bad arguments on the host before any device work.
No compute call is made (no GPU is needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "birk.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef[^;]*;", "", text)   # function-pointer and struct typedefs
    return sorted(set(re.findall(r"\b(birk_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def birk():
    from paper_2509_01855_amd import birk as b
    return b


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("birk_apply", "birk_apply_T", "birk_precond", "birk_krylov_solve",
                     "birk_plan_create", "birk_plan_destroy", "birk_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(birk):
    lib = ctypes.CDLL(birk.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert sorted(birk.EXPORTED) == _declared_functions()


def test_status_strings_cover_every_code(birk):
    seen = set()
    for code in range(0, -10, -1):
        s = birk.birk_status_string(code)
        assert s.startswith("BIRK_") and s not in seen
        seen.add(s)
    assert birk.birk_status_string(12345) == "unknown birk_status"


def test_solve_opts_defaults(birk):
    o = birk.birk_solve_opts_default()
    assert (o.method, o.restart, o.max_iter, o.use_precond, o.use_x0) == (0, 30, 300, 1, 0)
    assert o.rtol == 1e-10 and o.inner_rtol == 1e-5 and o.max_refine == 8


def test_struct_layouts(birk):
    assert ctypes.sizeof(birk.birk_solve_opts) == 48
    assert ctypes.sizeof(birk.birk_solve_info) == 32


def test_struct_layouts_match_the_c_header(birk, tmp_path):
    """Sizes and field offsets of every struct in include/birk.h, from a C program compiled
    against the header with gcc, equal those of the ctypes mirrors."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"birk_solve_opts": birk.birk_solve_opts, "birk_solve_info": birk.birk_solve_info,
               "birk_ivp_model": birk.birk_ivp_model, "birk_newton_opts": birk.birk_newton_opts,
               "birk_newton_info": birk.birk_newton_info}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "birk.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'  printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{name}.{f[0]}"


@pytest.mark.parametrize("n_nodes,n_x,prec,expect", [
    ([2], [6], 0, -2),          # N_n < 3
    ([256], [0], 0, -2),        # n_x < 1
    ([256], [6], 7, -1),        # bad precision
    ([(1 << 23) + 2], [1], 0, -2),   # N = 2^23 + 1 is not a power of two and exceeds 2^22
    ([(1 << 24) + 1], [1], 0, -2),   # power of two beyond the limit
])
def test_plan_create_rejects_on_host(birk, n_nodes, n_x, prec, expect):
    h = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 1)(*n_nodes)
    nx = (ctypes.c_int32 * 1)(*n_x)
    assert birk._lib.birk_plan_create(ctypes.byref(h), 1, nn, nx, prec, None) == expect
    assert h.value is None


def test_null_arguments_are_rejected(birk):
    lib = birk._lib
    h = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 1)(256)
    nx = (ctypes.c_int32 * 1)(6)
    assert lib.birk_plan_create(None, 1, nn, nx, 0, None) == birk.BIRK_ERR_ARG
    assert lib.birk_plan_create(ctypes.byref(h), 1, None, nx, 0, None) == birk.BIRK_ERR_ARG
    assert lib.birk_plan_create(ctypes.byref(h), 0, nn, nx, 0, None) == birk.BIRK_ERR_SIZE
    assert lib.birk_apply(None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_apply_T(None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_apply_b(None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_apply_bT(None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_endpoint(None, None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_two_body(None, 1.0, 1.0, None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_newton_ivp(None, None, None, None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_precond(None, 0, None, None, None, 1) == birk.BIRK_ERR_ARG
    assert lib.birk_fast_ax(None, 0, None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_krylov_solve(None, 0, None, None, None, None, None) == birk.BIRK_ERR_ARG
    assert lib.birk_weights(None, 0, None) == birk.BIRK_ERR_ARG
    assert lib.birk_plan_tune(None, None, 0) == birk.BIRK_ERR_ARG
    assert lib.birk_plan_set_graphs(None, 1) == birk.BIRK_ERR_ARG
    assert lib.birk_plan_destroy(None) == birk.BIRK_OK
    assert lib.birk_plan_length(None) == 0


# ---- the binding checks every tensor before calling the library (no GPU needed: the
# checks run in Python and raise before any call; a tensor that passes them all still
# fails the device check here because it lives on the CPU)
def _fake_plan(birk, prec, n_nodes=(9, 5), n_x=(2, 3)):
    return birk.Plan(0, tuple(n_nodes), tuple(n_x), prec, 0)


@pytest.mark.parametrize("prec,dtype,factor", [(0, "float64", 1), (1, "float32", 1), (2, "float32", 1),
                                              (3, "float32", 2)])
def test_binding_rejects_bad_vectors(birk, prec, dtype, factor):
    import torch
    plan = _fake_plan(birk, prec)
    n = (9 * 2 + 5 * 3) * factor
    good = torch.zeros(n, dtype=getattr(torch, dtype))
    other = torch.float32 if dtype == "float64" else torch.float64
    for fn in (birk.birk_apply, birk.birk_apply_T, birk.birk_apply_b, birk.birk_apply_bT):
        with pytest.raises(ValueError, match="dtype"):
            fn(plan, good.to(other), good.clone())
        with pytest.raises(ValueError, match="elements"):
            fn(plan, good[:-1], good.clone())
        with pytest.raises(ValueError, match="elements"):
            fn(plan, good, torch.zeros(n + 1, dtype=good.dtype))
        with pytest.raises(ValueError, match="contiguous"):
            fn(plan, torch.zeros(2 * n, dtype=good.dtype)[::2], good.clone())
        with pytest.raises(ValueError, match="cuda"):
            fn(plan, good, good.clone())
        with pytest.raises(ValueError, match="required"):
            fn(plan, None, good)
    with pytest.raises(ValueError, match="Tensor"):
        birk.birk_apply(plan, [0.0] * n, good)


def test_binding_rejects_bad_jacobians_and_solve_arguments(birk):
    import torch
    plan = _fake_plan(birk, 0)
    n = 9 * 2 + 5 * 3
    v = torch.zeros(n, dtype=torch.float64)
    Jc = torch.zeros(2 * 2 + 3 * 3, dtype=torch.float64)
    Jn = torch.zeros(9 * 4 + 5 * 9, dtype=torch.float64)
    with pytest.raises(ValueError, match="J: .*elements"):
        birk.birk_precond(plan, Jc, v, v.clone(), True, birk.BIRK_J_PER_NODE)
    with pytest.raises(ValueError, match="J: .*elements"):
        birk.birk_precond(plan, Jn, v, v.clone(), True, birk.BIRK_J_CONSTANT)
    with pytest.raises(ValueError, match="jac_kind"):
        birk.birk_precond(plan, Jn, v, v.clone(), True, 5)
    with pytest.raises(ValueError, match="J: dtype"):
        birk.birk_fast_ax(plan, Jc.float(), v, v.clone(), birk.BIRK_J_CONSTANT)
    with pytest.raises(ValueError, match="beta: .*elements"):
        birk.birk_krylov_solve(plan, Jc, v[:-1], v.clone(), birk.BIRK_J_CONSTANT)
    with pytest.raises(ValueError, match="chi: dtype"):
        birk.birk_krylov_solve(plan, Jc, v, v.float(), birk.BIRK_J_CONSTANT)
    # a float plan still takes double beta / chi / J in the solve
    p32 = _fake_plan(birk, 2)
    with pytest.raises(ValueError, match="cuda"):
        birk.birk_krylov_solve(p32, Jc, v, v.clone(), birk.BIRK_J_CONSTANT)
    # endpoint: one double per component
    with pytest.raises(ValueError, match="xa: .*elements"):
        birk.birk_endpoint(plan, torch.zeros(4, dtype=torch.float64), v, torch.zeros(5, dtype=torch.float64))
    # two-body: J per node
    with pytest.raises(ValueError, match="J: .*elements"):
        birk.birk_two_body(plan, v, v.clone(), Jc)


def test_binding_rejects_overlapping_buffers(birk):
    import torch
    plan = _fake_plan(birk, 0)
    n = 9 * 2 + 5 * 3
    buf = torch.zeros(2 * n, dtype=torch.float64)
    with pytest.raises(ValueError, match="overlap"):
        birk.birk_apply(plan, buf[:n], buf[:n])
    with pytest.raises(ValueError, match="overlap"):
        birk.birk_apply(plan, buf[:n], buf[1:n + 1])
    # disjoint halves pass the overlap check and reach the device check
    with pytest.raises(ValueError, match="cuda"):
        birk.birk_apply(plan, buf[:n], buf[n:])
