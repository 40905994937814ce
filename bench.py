"""Benchmark of the Birkhoff hot path on one MI355X.

Headline workload: the million-point configuration -- N_n = 2^20 + 1 CGL nodes, n_x = 6
states, time-varying Jacobian of the two-body problem along a seeded Keplerian orbit
(a = 7000 km, e ~ U(0, 0.2), canonical units, one period), synthetic inputs.

One step is one pass of the whole hot path:
  * headline: B^a v (FastBV) in double, once per buffer of a rotation of R
    input/output pairs whose footprint exceeds the 256 MB Infinity Cache, so that every
    product reads its input from HBM; B^aT g in double (same rotation); B^a v in float;
    P^{-1} y (inverse-preconditioner scan) and P y in double; FastAX (x - B^a (J x)) in
    double; the preconditioned GMRES solve to relative residual 1e-10, once with float
    Krylov bulk inside double refinement (mixed) and once in double (FP64); the b-form
    products B^b v, B^bT g and the endpoint row x^b = x^a + w^T v in double; Newton's
    method on the nonlinear two-body IVP over one period (e = 0.15) from the circular
    orbit, to ||G|| <= 1e-13 ||X||; MINRES on the symmetric KKT form
    [[I, A^T], [A, 0]] [chi; lambda] = [0; beta] to 1e-10;
  * small workloads: N_n = 256 and 257, n_x = 6 (LTI, B^a, B^aT and the solve to 1e-12)
    and N_n = 2^16 + 1, n_x = 6 (LTI, B^a, B^aT and both solves to 1e-10);
  * batched uneven workload: 512 LTI instances (N_n log-uniform in [2^8, 2^16], n_x in
    {4, 6, 12}) in one plan: B^a v in double, and the mixed and FP64 solves to 1e-10;
  * many-RHS workload: 32 right-hand sides of N_n = 2^18 + 1, n_x = 6 in one plan:
    B^a v in compensated double-float (DF32), in double and in float.

value = Gpts/s of the headline double B^a product = n / (mean duration of one
birk_apply), timed with HIP events on the plan's stream over the timed region.

After the timed steps, untimed runs of the same plans on inputs with known exact
results (sparse Chebyshev series, node-sparse right-hand sides, closed-form solutions)
feed the oracle leg, which states the error of every result against the FP64 oracle and
times the oracle itself (cpu_baseline).  A CPU run of the paper's own fast method
(scipy's DCT-I and GMRES) is reported beside it as context (cpu_context).

`python bench.py --gpus N --steps K --warmup W`; N must be 1 (single-GPU build).
"""

from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Birkhoff matvec Gpts/s at N=2^20; solve time mixed vs FP64 at 1e-10 resid"
KERNEL_SOURCES = ["paper_2509_01855_amd/csrc/birk_fast.hip", "paper_2509_01855_amd/csrc/birk_dct.hip",
                  "paper_2509_01855_amd/csrc/birk_fft.h"]
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=20, help="N = 2^log2n (N_n = N + 1)")
    ap.add_argument("--rotation", type=int, default=6, help="input/output buffer pairs per product sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (timing and errors)")
    ap.add_argument("--no-cpu-context", action="store_true", help="skip the scipy run of the fast method")
    ap.add_argument("--no-tune", action="store_true", help="skip birk_plan_tune (default tile schedules)")
    ap.add_argument("--products-only", action="store_true", help="skip the solves (for profiling runs)")
    ap.add_argument("--headline-only", action="store_true", help="skip the small, batched and many-RHS workloads")
    ap.add_argument("--cpu-sample", type=int, default=800, help="rows of B^a the oracle computes at N = 2^20")
    ap.add_argument("--solve-only", choices=["fp64", "mixed"], default=None,
                    help="time only the headline solve in this precision (per-kernel profiles of one solve)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration under rocprofv3)")
    return ap.parse_args()


def calibrate_copy():
    """A plain 1 GiB device-to-device copy, three times, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 1 << 27  # doubles: 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_each": n * 8, "copies": 3}), flush=True)


def traffic_key(split, tb, xcd, narrow=0):
    from bench_traffic import schedule_key
    return schedule_key(split, tb, xcd, narrow)


def traffic_record(kernel_sources, schedule=None):
    """Measured HBM bytes per product from profiles/, if the kernels are unchanged since and
    the product runs the tile schedule the counters were taken with."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "apply_f64_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in kernel_sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    for r in rec.get("records", []):
        if schedule is None or r["schedule"] == schedule:
            return r
    return None


class Timer:
    """HIP-event timing of named regions on one stream; read after a synchronisation."""

    def __init__(self, stream):
        self.stream = stream
        self.pending = []
        self.rec = {}

    def region(self, name, fn):
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        fn()
        e1.record(self.stream)
        self.pending.append((name, e0, e1))

    def wall(self, name, fn):
        t0 = time.perf_counter()
        out = fn()
        self.rec.setdefault(name, []).append((time.perf_counter() - t0) * 1e3)
        return out

    def collect(self, keep: bool):
        for name, e0, e1 in self.pending:
            if keep:
                self.rec.setdefault(name, []).append(e0.elapsed_time(e1))
        self.pending = []

    def mean_ms(self, name):
        xs = self.rec.get(name, [])
        return float(sum(xs) / len(xs)) if xs else float("nan")

    def median_ms(self, name):
        xs = sorted(self.rec.get(name, []))
        return float(xs[len(xs) // 2]) if xs else float("nan")

    def min_ms(self, name):
        xs = self.rec.get(name, [])
        return float(min(xs)) if xs else float("nan")


def copy_ceiling_gbs(torch, stream, reps=5):
    """Measured HBM ceiling: a 1 GiB device-to-device copy (read + write counted), best of
    `reps`, timed with events on the bench stream."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return round(2.0 * n * 8 / best / 1e9, 1)


def graph_replay_timing(B, torch, reps=200):
    """B^a at N_n = 256, n_x = 6 (the small workload) on a side stream: eager launches vs
    replays of the recorded graph (birk_plan_set_graphs), mean per product."""
    side = torch.cuda.Stream()
    Nn, nx = 256, 6
    res = {"workload": "B^a, N_n = 256, n_x = 6 (Bluestein path), back-to-back products"}
    with torch.cuda.stream(side):
        v = torch.randn(Nn * nx, dtype=torch.float64, device="cuda")
        o = torch.empty_like(v)
        for mode in ("eager", "graph"):
            plan = B.birk_plan_create([Nn], [nx], B.BIRK_F64, side)
            if mode == "graph":
                B.birk_plan_set_graphs(plan)
            for _ in range(3):
                B.birk_apply(plan, v, o)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(reps):
                B.birk_apply(plan, v, o)
            e1.record(side)
            e1.synchronize()
            res[f"{mode}_us"] = round(e0.elapsed_time(e1) * 1e3 / reps, 2)
            plan.destroy()
    side.synchronize()
    return res


# ------------------------------------------------------------------ the oracle leg
def oracle_leg(a, acc, nproc):
    """The FP64 oracle on the host: (1) errors of every GPU result gathered in `acc`
    against oracle references (exact series, rows and columns of B^a, dense LU) or closed
    forms, (2) cpu_baseline: the oracle's own throughput on a bounded sample of the
    headline product, and the dense oracle (build + matvec + LU) at N_n = 256 and 4097."""
    import concurrent.futures as cf

    import numpy as np
    import scipy.linalg

    from oracle import birkhoff as bk
    from oracle import system as sy
    from paper_2509_01855_amd import workloads as wl

    def rel(got, ref):
        got = np.asarray(got, dtype=np.float64)
        ref = np.asarray(ref, dtype=np.float64)
        return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))

    err = {}
    # headline products: exact antiderivatives of the Chebyshev series (B^a), combinations of
    # O(N log N) rows for node-sparse right-hand sides (B^aT)
    N = acc["N"]
    ref = np.stack([bk.sparse_mode_exact(N, m, al) for m, al in acc["head_specs"]])
    err["apply_f64"] = rel(acc["head_apply_f64"], ref)
    err["apply_f32"] = rel(acc["head_apply_f32"], ref)
    refT = np.stack([sum(acc["head_G"][c, i] * bk.ba_row(N, int(i)) for i in idx)
                     for c, idx in enumerate(acc["head_nodes"])])
    err["apply_T_f64"] = rel(acc["head_apply_T_f64"], refT)
    if "head_solve" in acc:
        Z = acc["head_solve_exact"]
        err["solve_fp64_vs_closed_form"] = rel(acc["head_solve"]["fp64"], Z)
        err["solve_mixed_vs_closed_form"] = rel(acc["head_solve"]["mixed"], Z)
        err["solve_note"] = ("time-shift right-hand side Z(-1) of the headline Kepler system, exact "
                             "solution (v, a)(t) along the orbit; solved to 1e-10 like the timed solves")
        if "head_kkt_chi" in acc:
            err["kkt_minres_chi_vs_closed_form"] = rel(acc["head_kkt_chi"], Z)
    if "newton_err" in acc:
        err["newton_ivp_vs_kepler"] = acc["newton_err"]
    if "small" in acc:
        sm = acc["small"]
        for Nn, d in sm["c0"].items():
            inst = wl.lti_instance(0, Nn)
            Ba = bk.dense_Ba(Nn - 1)
            err[f"c0_{Nn}_apply_f64"] = rel(d["apply"], d["v"] @ Ba.T)
            err[f"c0_{Nn}_apply_T_f64"] = rel(d["apply_T"], d["v"] @ Ba)
            xs = sy.solve_dense(sy.dense_A(Nn - 1, inst.J, Ba), sy.beta_vector(inst.x_a, Nn))
            err[f"c0_{Nn}_solve_fp64_vs_dense_lu"] = rel(d["solve"], xs)
        d = sm["c1"]
        N1 = d["N"]
        err["c1_apply_f64"] = rel(d["apply"], np.stack([bk.sparse_mode_exact(N1, m, al) for m, al in d["specs"]]))
        inst = wl.lti_instance(1, N1 + 1)
        tau = bk.cgl_nodes(N1)
        idx = np.unique(np.linspace(0, N1, 257).astype(int))
        Xe = np.stack([scipy.linalg.expm(inst.J * (tau[k] + 1.0)) @ inst.x_a for k in idx], axis=1)
        for p in ("fp64", "mixed"):
            err[f"c1_solve_{p}_vs_expm"] = rel(d["solve"][p].reshape(6, N1 + 1)[:, idx], Xe)
    if "batched" in acc:
        bt = acc["batched"]
        for p in ("fp64", "mixed"):
            worst = 0.0
            o = 0
            for ins in bt["insts"]:
                n = ins.n_x * ins.N_n
                X = bt[p][o:o + n].reshape(ins.n_x, ins.N_n)
                tau = bk.cgl_nodes(ins.N_n - 1)
                idx = np.unique(np.linspace(0, ins.N_n - 1, 17).astype(int))
                Xe = np.stack([scipy.linalg.expm(ins.J * (tau[k] + 1.0)) @ ins.x_a for k in idx], axis=1)
                worst = max(worst, rel(X[:, idx], Xe))
                o += n
            err[f"batched_solve_{p}_worst_instance_vs_expm"] = worst
        err["batched_apply_f64"] = bt["apply_err"](bk)
    if "many_rhs" in acc:
        m = acc["many_rhs"]
        ref = np.stack([bk.sparse_mode_exact(m["N"], mm, al) for mm, al in m["specs"]])
        for p in ("df32", "f64", "f32"):
            got = m[p].reshape(-1, m["N"] + 1)
            err[f"many_rhs_apply_{p}"] = max(rel(got[c::len(m["specs"])], ref[c][None, :])
                                             for c in range(len(m["specs"])))

    # cpu_baseline: rows of B^a (oracle.birkhoff.ba_row, one O(N log N) row per output) on
    # the headline size, the rows spread over nproc threads
    rows = np.linspace(0, N, a.cpu_sample).astype(np.int64)
    v = acc["head_v0"]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=nproc) as ex:
        outs = list(ex.map(lambda i: float(bk.ba_row(N, int(i)) @ v), rows))
    dt = time.perf_counter() - t0
    base = {"value": a.cpu_sample / dt / 1e9, "unit": "Gpts/s", "cores": nproc, "kind": "oracle",
            "sample": f"{a.cpu_sample} outputs of B^a v (one component) at N_n={N + 1}, each one full row of B^a "
                      f"from oracle.birkhoff.ba_row (closed-form coefficients + scipy DCT-I), rows spread over "
                      f"{nproc} threads, {dt:.1f} s"}
    del outs
    # the dense oracle (build B^a and A, one dense matvec, dense LU solve), NumPy/LAPACK on all cores
    dense = {}
    for Nn, seed in ((256, 0), (4097, 1)):
        inst = wl.lti_instance(seed, Nn)
        t0 = time.perf_counter()
        Ba = bk.dense_Ba(Nn - 1)
        A = sy.dense_A(Nn - 1, inst.J, Ba)
        t1 = time.perf_counter()
        V = np.random.default_rng(Nn).standard_normal((6, Nn))
        t2 = time.perf_counter()
        _ = V @ Ba.T
        t3 = time.perf_counter()
        xs = sy.solve_dense(A, sy.beta_vector(inst.x_a, Nn))
        t4 = time.perf_counter()
        dense[f"N_n={Nn}"] = {"n": 6 * Nn, "build_s": round(t1 - t0, 3), "matvec_s": round(t3 - t2, 5),
                              "lu_solve_s": round(t4 - t3, 3),
                              "matvec_gpts": round(6 * Nn / (t3 - t2) / 1e9, 4)}
        del A, Ba, xs
    base["dense_oracle"] = dense
    base["dense_threads"] = nproc
    return err, base


# ------------------------------------------------------------------ the paper's method on the CPU (context)
def cpu_fastbv(V, workers):
    """B^a V along the last axis by FastBV with scipy's DCT-I: nodal values -> Chebyshev
    coefficients (DCT of the reversed values), the integration recurrence with the
    T_{N+1} alias, coefficients -> nodal values (second DCT), then the constant that
    makes the value at tau = -1 zero.  The paper's fast method run on the host CPU."""
    import numpy as np
    import scipy.fft
    N = V.shape[-1] - 1
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    a = scipy.fft.dct(V[..., ::-1], type=1, axis=-1, workers=workers) / (N * c)
    ch = np.zeros_like(a)
    k = np.arange(2, N)
    ch[..., 1] = a[..., 0] - a[..., 2] / 2.0
    ch[..., 2:N] = (a[..., 1:N - 1] - a[..., 3:N + 1]) / (2.0 * k)
    ch[..., N] = a[..., N - 1] / (2.0 * N)
    ch[..., N - 1] += a[..., N] / (2.0 * (N + 1))
    x = ch.copy()
    x[..., 1:N] *= 0.5
    y = scipy.fft.dct(x, type=1, axis=-1, workers=workers)[..., ::-1]
    return y - y[..., :1]


def cpu_solve(inst, workers, rtol):
    """Right-preconditioned GMRES (scipy) on [I - B^a J] chi = beta with the Birkhoff
    preconditioner applied by node-by-node forward substitution, products by cpu_fastbv."""
    import numpy as np
    import scipy.fft
    import scipy.sparse.linalg as spla
    Nn, nx = inst.N_n, inst.n_x
    N = Nn - 1
    # CC weights (the last row of B^a) from the moments of T_k with one DCT-I
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    k = np.arange(N + 1)
    mom = np.zeros(N + 1)
    mom[k % 2 == 0] = 2.0 / (1.0 - k[k % 2 == 0].astype(float) ** 2)
    x = mom / (N * c) * 2.0
    x[1:N] *= 0.5
    e = np.ones(N + 1)
    e[0] = e[N] = 0.5
    w = e * scipy.fft.dct(x, type=1, workers=workers)[::-1]
    J = inst.J if inst.per_node else np.repeat(inst.J[:, :, None], Nn, axis=2)
    Jn = np.ascontiguousarray(np.moveaxis(J, 2, 0))
    Minv = np.linalg.inv(np.eye(nx)[None] - 0.5 * w[:, None, None] * Jn)
    WJ = w[:, None, None] * Jn

    def pinv(y):
        Y = y.reshape(nx, Nn).T
        X = np.empty_like(Y)
        S = np.zeros(nx)
        for kk in range(Nn):
            xk = Minv[kk] @ (Y[kk] + S)
            X[kk] = xk
            S = S + WJ[kk] @ xk
        return X.T.reshape(-1)

    def amul(z):
        Z = z.reshape(nx, Nn)
        return (Z - cpu_fastbv(np.einsum("krc,ck->rk", Jn, Z), workers)).reshape(-1)

    beta = np.repeat(inst.x_a, Nn)
    n = nx * Nn
    op = spla.LinearOperator((n, n), matvec=lambda u: amul(pinv(u)))
    its = [0]

    def cb(_):
        its[0] += 1
    t0 = time.perf_counter()
    u, _ = spla.gmres(op, beta, rtol=rtol, restart=30, maxiter=10, callback=cb, callback_type="pr_norm")
    chi = pinv(u)
    dt = time.perf_counter() - t0
    return dt, its[0], float(np.linalg.norm(beta - amul(chi)) / np.linalg.norm(beta))


def cpu_context(nproc):
    """The paper's method on the host CPU (not the oracle): FastBV with scipy's DCT-I at
    N_n = 2^16 + 1 and 2^20 + 1 (six components), and the preconditioned GMRES solve of the
    LTI system (2^16 + 1) and the Kepler system (2^16 + 1 and 2^20 + 1) to 1e-10."""
    import numpy as np
    from paper_2509_01855_amd import workloads as wl
    out = {"kind": "the paper's method on the CPU (scipy DCT-I + GMRES), context only", "threads": nproc}
    for lg in (16, 20):
        V = np.random.default_rng(lg).standard_normal((6, (1 << lg) + 1))
        cpu_fastbv(V, nproc)
        reps = 5 if lg == 16 else 2
        t0 = time.perf_counter()
        for _ in range(reps):
            cpu_fastbv(V, nproc)
        dt = (time.perf_counter() - t0) / reps
        out[f"fastbv_N_n=2^{lg}+1"] = {"ms": round(dt * 1e3, 2), "gpts": round(V.size / dt / 1e9, 4)}
    for name, inst in (("lti_2^16+1", wl.lti_instance(1, (1 << 16) + 1)),
                       ("kepler_2^16+1", wl.kepler_instance(2, (1 << 16) + 1)),
                       ("kepler_2^20+1", wl.kepler_instance(2, (1 << 20) + 1))):
        dt, its, rr = cpu_solve(inst, nproc, 1e-10)
        out[f"solve_{name}"] = {"s": round(dt, 2), "gmres_iters": its, "rel_resid": rr}
    return out


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {a.gpus}); "
              "the multi-GPU sharding is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2509_01855_amd import birk as B
    from paper_2509_01855_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    tm = Timer(stream)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    nproc = min(os.cpu_count() or 1, 16)
    D64 = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")  # noqa: E731
    host = lambda t: t.detach().cpu().numpy()  # noqa: E731

    # ---- headline workload
    N = 1 << a.log2n
    Nn = N + 1
    nx = 6
    n = Nn * nx
    print(f"[bench] building inputs N_n={Nn} n_x={nx}", file=sys.stderr, flush=True)
    inst = wl.kepler_instance(2, Nn)
    plan64 = B.birk_plan_create([Nn], [nx], B.BIRK_F64, stream)
    planmx = B.birk_plan_create([Nn], [nx], B.BIRK_F32_REFINE_F64, stream)
    J = torch.from_numpy(inst.J.ravel()).to("cuda")
    R = max(1, a.rotation)
    vin = [torch.randn(n, dtype=torch.float64, device="cuda", generator=gen) for _ in range(R)]
    vout = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(R)]
    v32 = [x.float() for x in vin[:2]]
    o32 = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(2)]
    beta = torch.from_numpy(np.repeat(inst.x_a, Nn)).to("cuda")
    chi = torch.zeros(n, dtype=torch.float64, device="cuda")
    solve_info = {}
    # nonlinear IVP: one period of a Kepler orbit (e = 0.15) by Newton from the circular orbit
    ivp = wl.kepler_ivp(44, Nn, 0.15)
    ivp_guess = torch.from_numpy(ivp["guess"].ravel()).to("cuda")
    ivp_xa = torch.from_numpy(ivp["x_a"]).to("cuda")
    ivp_X = torch.empty_like(ivp_guess)
    ivp_info = {}

    extra = not a.headline_only and not a.solve_only
    if extra:
        # ---- small workloads (N_n = 256, 257 with n_x = 6; N_n = 2^16 + 1 with n_x = 6)
        print("[bench] building the small workloads", file=sys.stderr, flush=True)
        small = {}
        for Nn0 in (256, 257):
            i0 = wl.lti_instance(0, Nn0)
            small[Nn0] = {"plan": B.birk_plan_create([Nn0], [6], B.BIRK_F64, stream), "inst": i0,
                          "v": D64(wl.random_vectors([5, Nn0], (6, Nn0))[0].ravel()),
                          "J": D64(i0.J.ravel()), "beta": D64(np.repeat(i0.x_a, Nn0)),
                          "chi": torch.zeros(6 * Nn0, dtype=torch.float64, device="cuda")}
            small[Nn0]["out"] = torch.empty_like(small[Nn0]["v"])
        N1 = 1 << 16
        i1 = wl.lti_instance(1, N1 + 1)
        c1 = {"plan": B.birk_plan_create([N1 + 1], [6], B.BIRK_F64, stream),
              "planmx": B.birk_plan_create([N1 + 1], [6], B.BIRK_F32_REFINE_F64, stream),
              "v": D64(wl.random_vectors([6, N1], (6 * (N1 + 1),))[0]), "J": D64(i1.J.ravel()),
              "beta": D64(np.repeat(i1.x_a, N1 + 1)), "chi": torch.zeros(6 * (N1 + 1), dtype=torch.float64,
                                                                         device="cuda")}
        c1["out"] = torch.empty_like(c1["v"])
        # ---- batched uneven workload
        print("[bench] building the 512-instance batch", file=sys.stderr, flush=True)
        binst = wl.batched_instances(count=512)
        bNn = [i.N_n for i in binst]
        bnx = [i.n_x for i in binst]
        bn = sum(p * q for p, q in zip(bNn, bnx))
        bplan64 = B.birk_plan_create(bNn, bnx, B.BIRK_F64, stream)
        bplanmx = B.birk_plan_create(bNn, bnx, B.BIRK_F32_REFINE_F64, stream)
        bJ = torch.from_numpy(np.concatenate([i.J.ravel() for i in binst])).to("cuda")
        bbeta = torch.from_numpy(np.concatenate([np.repeat(i.x_a, i.N_n) for i in binst])).to("cuda")
        bchi = torch.zeros(bn, dtype=torch.float64, device="cuda")
        bv = torch.randn(bn, dtype=torch.float64, device="cuda", generator=gen)
        bo = torch.empty_like(bv)
        bsol = {}
        # ---- many-RHS workload
        print("[bench] building the 32-RHS workload", file=sys.stderr, flush=True)
        mNn, mnx, mR = (1 << 18) + 1, 6, 32
        mn = mNn * mnx * mR
        mplans = {p: B.birk_plan_create([mNn] * mR, [mnx] * mR, p, stream)
                  for p in (B.BIRK_F64, B.BIRK_F32, B.BIRK_DF32)}
        mv = torch.randn(mn, dtype=torch.float64, device="cuda", generator=gen)
        mo = torch.empty_like(mv)
        mv32 = mv.float()
        mo32 = torch.empty_like(mv32)
        hi = mv.float()
        lo = (mv - hi.double()).float()
        mvdf = torch.stack([hi, lo], dim=1).reshape(-1).contiguous()
        modf = torch.empty_like(mvdf)
    torch.cuda.synchronize()

    kkt_lam = torch.zeros(n, dtype=torch.float64, device="cuda")
    xa_end = torch.zeros(nx, dtype=torch.float64, device="cuda")
    xb_end = torch.empty_like(xa_end)

    # autotuner of the power-of-two product path (plan setup, outside the timed region)
    tuned = {}
    head_sched = traffic_key(int(os.environ.get("BIRK_FAST_SPLIT", "0")), int(os.environ.get("BIRK_FAST_TB", "0")),
                             int(os.environ.get("BIRK_FAST_XCD", "1")), int(os.environ.get("BIRK_FAST_NARROW", "1")))
    if not a.no_tune:
        print("[bench] autotuning the power-of-two plans", file=sys.stderr, flush=True)
        tplans = {"headline_f64": plan64, "headline_f32": planmx}
        if extra:
            tplans.update({"c1_f64": c1["plan"], "batched_f64": bplan64, "batched_f32": bplanmx,
                           "many_rhs_f64": mplans[B.BIRK_F64],
                           "many_rhs_f32": mplans[B.BIRK_F32], "many_rhs_df32": mplans[B.BIRK_DF32]})
        for name, plan in tplans.items():
            rep = B.birk_plan_tune(plan)
            tuned[name] = [ln.split(" chosen ")[0].split(":")[0] + ": " + ln.split(" chosen ")[1]
                           for ln in rep.splitlines() if " chosen " in ln]
            if name == "headline_f64":
                m = re.search(r"chosen \[split (\d+), tb (\d+), xcd (\d+), streams \d+, narrow (\d+)\]", rep)
                head_sched = traffic_key(int(m.group(1)), int(m.group(2)), int(m.group(3)), int(m.group(4)))
        torch.cuda.synchronize()

    def step(timed: bool):
        if a.solve_only:
            plan = plan64 if a.solve_only == "fp64" else planmx
            solve_info[a.solve_only] = tm.wall(a.solve_only if timed else "_warm",
                                               lambda: B.birk_krylov_solve(plan, J, beta, chi, B.BIRK_J_PER_NODE,
                                                                           rtol=1e-10))
            return
        for i in range(R):
            tm.region("apply", lambda i=i: B.birk_apply(plan64, vin[i], vout[i]))
        for i in range(R):
            tm.region("apply_T", lambda i=i: B.birk_apply_T(plan64, vin[i], vout[(i + 1) % R]))
        for i in range(2):
            tm.region("apply_f32", lambda i=i: B.birk_apply(planmx, v32[i], o32[i]))
        tm.region("pinv", lambda: B.birk_precond(plan64, J, vin[0], vout[1], 1, B.BIRK_J_PER_NODE))
        tm.region("fast_ax", lambda: B.birk_fast_ax(plan64, J, vin[0], vout[0], B.BIRK_J_PER_NODE))
        tm.region("pfwd", lambda: B.birk_precond(plan64, J, vin[1], vout[1], 0, B.BIRK_J_PER_NODE))
        tm.region("apply_b", lambda: B.birk_apply_b(plan64, vin[1], vout[0]))
        tm.region("apply_bT", lambda: B.birk_apply_bT(plan64, vin[0], vout[1]))
        tm.region("endpoint", lambda: B.birk_endpoint(plan64, xa_end, vin[1], xb_end))
        if extra:
            for Nn0, d in small.items():
                tm.region(f"c0_{Nn0}_apply", lambda d=d: B.birk_apply(d["plan"], d["v"], d["out"]))
                tm.region(f"c0_{Nn0}_apply_T", lambda d=d: B.birk_apply_T(d["plan"], d["v"], d["out"]))
            tm.region("c1_apply", lambda: B.birk_apply(c1["plan"], c1["v"], c1["out"]))
            tm.region("c1_apply_T", lambda: B.birk_apply_T(c1["plan"], c1["v"], c1["out"]))
            tm.region("b_apply", lambda: B.birk_apply(bplan64, bv, bo))
            tm.region("m_apply_f64", lambda: B.birk_apply(mplans[B.BIRK_F64], mv, mo))
            tm.region("m_apply_f32", lambda: B.birk_apply(mplans[B.BIRK_F32], mv32, mo32))
            tm.region("m_apply_df32", lambda: B.birk_apply(mplans[B.BIRK_DF32], mvdf, modf))
        torch.cuda.synchronize()
        tm.collect(timed)
        if not a.products_only:
            solves = [("mixed", planmx, J, beta, chi, B.BIRK_J_PER_NODE, 1e-10),
                      ("fp64", plan64, J, beta, chi, B.BIRK_J_PER_NODE, 1e-10)]
            if extra:
                for Nn0, d in small.items():
                    solves.append((f"c0_{Nn0}_fp64", d["plan"], d["J"], d["beta"], d["chi"], B.BIRK_J_CONSTANT,
                                   1e-12))
                solves += [("c1_mixed", c1["planmx"], c1["J"], c1["beta"], c1["chi"], B.BIRK_J_CONSTANT, 1e-10),
                           ("c1_fp64", c1["plan"], c1["J"], c1["beta"], c1["chi"], B.BIRK_J_CONSTANT, 1e-10),
                           ("b_mixed", bplanmx, bJ, bbeta, bchi, B.BIRK_J_CONSTANT, 1e-10),
                           ("b_fp64", bplan64, bJ, bbeta, bchi, B.BIRK_J_CONSTANT, 1e-10)]
            for name, plan, Jm, bt, ch, jk, rtol in solves:
                info = tm.wall(name if timed else "_warm",
                               lambda: B.birk_krylov_solve(plan, Jm, bt, ch, jk, rtol=rtol))
                solve_info[name] = info
                if extra and name in ("b_mixed", "b_fp64"):
                    bsol[name[2:]] = ch.clone()
                if extra and name == "c1_mixed":
                    c1["sol_mixed"] = ch.clone()

            def newton():
                ivp_X.copy_(ivp_guess)
                ivp_info.update(B.birk_newton_ivp(plan64, ivp_xa, ivp_X, mu=ivp["mu"], scale=ivp["scale"]))
            tm.wall("newton" if timed else "_warm", newton)
            # MINRES on the KKT form with H = I, f = 0 (chi = A^{-1} beta, lambda = -A^{-T} chi)
            solve_info["kkt"] = tm.wall("kkt" if timed else "_warm",
                                        lambda: B.birk_kkt_solve(plan64, J, beta, chi, kkt_lam,
                                                                 jac_kind=B.BIRK_J_PER_NODE, rtol=1e-10))

    for _ in range(a.warmup):
        step(False)
    torch.cuda.synchronize()
    print(f"[bench] warmup done; timing {a.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(True)
        print(f"[bench] step {k + 1}/{a.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    if a.solve_only:
        info = solve_info[a.solve_only]
        print(json.dumps({"solve_only": a.solve_only, "workload": "headline Kepler system, rtol 1e-10",
                          "ms": round(tm.mean_ms(a.solve_only), 3), "inner_iters": info["inner_iters"],
                          "outer_iters": info["outer_iters"], "rel_resid": info["rel_resid"]}), flush=True)
        return
    t_apply = tm.mean_ms("apply") * 1e-3
    gpts = n / t_apply / 1e9
    bytes_alg = 2.0 * n * 8.0
    achieved = bytes_alg / t_apply / 1e9
    us = lambda name: round(tm.mean_ms(name) * 1e3, 2)  # noqa: E731
    out = {
        "metric": METRIC,
        "value": round(gpts, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "million-point Kepler-linearised Birkhoff system: B^a / B^aT products, "
                               "P^{-1}, preconditioned GMRES to 1e-10",
                   "N_n": Nn, "n_x": nx, "n": n, "rotation_buffers": R,
                   "products_per_step": {"apply_f64": R, "apply_T_f64": R, "apply_f32": 2, "precond_inverse": 1,
                                         "precond_forward": 1, "fast_ax_f64": 1,
                                         "apply_b_f64": 1, "apply_bT_f64": 1, "endpoint_f64": 1,
                                         "solves": 0 if a.products_only else 2}},
        "roofline": {"bound": "hbm", "kernel": "birk_apply (FastBV, three-pass, double)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": bytes_alg, "avg_launch_us": round(t_apply * 1e6, 2)},
        "autotune": tuned if tuned else None,
        "secondary": {
            "apply_f64_us": us("apply"),
            "apply_f64_us_median": round(tm.median_ms("apply") * 1e3, 2),
            "apply_f64_us_min": round(tm.min_ms("apply") * 1e3, 2),
            "apply_T_f64_us": us("apply_T"),
            "apply_f32_us": us("apply_f32"),
            "apply_f32_gpts": round(n / (tm.mean_ms("apply_f32") * 1e-3) / 1e9, 3),
            "precond_inverse_f64_us": us("pinv"),
            "precond_forward_f64_us": us("pfwd"),
            "fast_ax_f64_us": us("fast_ax"),
            "apply_b_f64_us": us("apply_b"),
            "apply_bT_f64_us": us("apply_bT"),
            "endpoint_f64_us": us("endpoint"),
            "endpoint_f64_GBs": round(n * 8.0 / (tm.mean_ms("endpoint") * 1e-3) / 1e9, 1),
        },
    }
    out["roofline"]["measured_copy_GBs"] = copy_ceiling_gbs(torch, stream)
    out["roofline"]["frac_of_copy"] = round(achieved / out["roofline"]["measured_copy_GBs"], 4)
    tr = traffic_record(KERNEL_SOURCES, head_sched)
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes_per_product"]
        out["roofline"]["traffic_source"] = "profiles/apply_f64_traffic.json"
    if not a.products_only:
        mx, f64 = tm.mean_ms("mixed"), tm.mean_ms("fp64")
        out["solve"] = {
            "rtol": 1e-10,
            "mixed_ms": round(mx, 3), "fp64_ms": round(f64, 3), "speedup_mixed_vs_fp64": round(f64 / mx, 3),
            "mixed": {k: solve_info["mixed"][k] for k in ("inner_iters", "outer_iters", "rel_resid")},
            "fp64": {k: solve_info["fp64"][k] for k in ("inner_iters", "outer_iters", "rel_resid")},
        }
        ki = solve_info["kkt"]
        out["kkt_minres"] = {
            "workload": "MINRES on [[I, A^T], [A, 0]] [chi; lambda] = [0; beta], headline Kepler system, "
                        "preconditioner blockdiag(I, P P^T)^{-1}, rtol 1e-10",
            "ms": round(tm.mean_ms("kkt"), 3), "minres_iters": ki["inner_iters"][0],
            "restarts": ki["outer_iters"][0], "rel_resid": ki["rel_resid"][0]}
        err = float(np.max(np.abs(ivp_X.cpu().numpy().reshape(6, Nn) - ivp["exact"])))
        out["newton_ivp"] = {
            "workload": "two-body IVP over one period (e = 0.15), N_n = 2^20 + 1, Newton from the circular orbit",
            "ms": round(tm.mean_ms("newton"), 3), "newton_iters": ivp_info["newton_iters"][0],
            "linear_iters": ivp_info["linear_iters"][0], "rel_resid": ivp_info["rel_resid"][0],
            "max_abs_err_vs_kepler": err}
    if extra:
        sm_out = {}
        for Nn0 in small:
            sm_out[f"N_n={Nn0}"] = {"apply_f64_us": us(f"c0_{Nn0}_apply"), "apply_T_f64_us": us(f"c0_{Nn0}_apply_T")}
            if not a.products_only:
                sm_out[f"N_n={Nn0}"]["solve_fp64_ms_rtol_1e-12"] = round(tm.mean_ms(f"c0_{Nn0}_fp64"), 3)
                sm_out[f"N_n={Nn0}"]["gmres_iters"] = solve_info[f"c0_{Nn0}_fp64"]["inner_iters"][0]
        sm_out["N_n=65537"] = {"apply_f64_us": us("c1_apply"), "apply_T_f64_us": us("c1_apply_T"),
                               "apply_f64_gpts": round(6 * (N1 + 1) / (tm.mean_ms("c1_apply") * 1e-3) / 1e9, 3)}
        if not a.products_only:
            sm_out["N_n=65537"].update({
                "solve_fp64_ms": round(tm.mean_ms("c1_fp64"), 3), "solve_mixed_ms": round(tm.mean_ms("c1_mixed"), 3),
                "gmres_iters_fp64": solve_info["c1_fp64"]["inner_iters"][0],
                "gmres_iters_mixed": solve_info["c1_mixed"]["inner_iters"][0]})
        out["small"] = {"workload": "LTI, n_x = 6: N_n = 256 and 257 (solve to 1e-12), N_n = 2^16 + 1 "
                                    "(solves to 1e-10); latency-bound sizes, times not %HBM", **sm_out}
        bt = tm.mean_ms("b_apply") * 1e-3
        out["batched"] = {"workload": "512 LTI instances, N_n log-uniform in [2^8, 2^16], n_x in {4, 6, 12}",
                          "n": bn, "apply_f64_us": us("b_apply"), "apply_f64_gpts": round(bn / bt / 1e9, 3)}
        if not a.products_only:
            bmx, b64 = tm.mean_ms("b_mixed"), tm.mean_ms("b_fp64")
            summ = lambda info: {"inner_iters": [min(info["inner_iters"]), max(info["inner_iters"])],  # noqa: E731
                                 "outer_iters": [min(info["outer_iters"]), max(info["outer_iters"])],
                                 "worst_rel_resid": max(info["rel_resid"]), "status": info["status"]}
            out["batched"].update({"rtol": 1e-10, "mixed_ms": round(bmx, 3), "fp64_ms": round(b64, 3),
                                   "speedup_mixed_vs_fp64": round(b64 / bmx, 3),
                                   "mixed": summ(solve_info["b_mixed"]), "fp64": summ(solve_info["b_fp64"])})
        out["many_rhs"] = {
            "workload": "32 RHS x n_x = 6 at N_n = 2^18 + 1 in one plan (192 components)", "n": mn,
            "apply_df32_us": us("m_apply_df32"), "apply_f64_us": us("m_apply_f64"), "apply_f32_us": us("m_apply_f32"),
            "apply_df32_gpts": round(mn / (tm.mean_ms("m_apply_df32") * 1e-3) / 1e9, 3),
            "apply_f64_gpts": round(mn / (tm.mean_ms("m_apply_f64") * 1e-3) / 1e9, 3),
            "apply_f32_gpts": round(mn / (tm.mean_ms("m_apply_f32") * 1e-3) / 1e9, 3),
        }
        out["graphs"] = graph_replay_timing(B, torch)

    if not a.no_cpu_baseline:
        # untimed runs on inputs with known exact results, for the oracle leg
        print("[bench] accuracy runs", file=sys.stderr, flush=True)
        acc = {"N": N, "head_v0": host(vin[0][:Nn])}
        Xs, specs = wl.sparse_series(101, N, nx, 16)
        acc["head_specs"] = specs
        vs = D64(Xs.ravel())
        os_ = torch.empty_like(vs)
        B.birk_apply(plan64, vs, os_)
        acc["head_apply_f64"] = host(os_).reshape(nx, Nn)
        vs32 = vs.float()
        os32 = torch.empty_like(vs32)
        B.birk_apply(planmx, vs32, os32)
        acc["head_apply_f32"] = host(os32).reshape(nx, Nn)
        Gs, nodes = wl.node_sparse(102, N, nx)
        B.birk_apply_T(plan64, D64(Gs.ravel()), os_)
        acc["head_apply_T_f64"] = host(os_).reshape(nx, Nn)
        acc["head_G"], acc["head_nodes"] = Gs, nodes
        if not a.products_only:
            Z = np.concatenate([inst.extra["v"], inst.extra["acc"]])
            bz = D64(np.repeat(Z[:, 0], Nn))
            acc["head_solve"] = {}
            for p, plan in (("fp64", plan64), ("mixed", planmx)):
                xz = torch.zeros_like(bz)
                B.birk_krylov_solve(plan, J, bz, xz, B.BIRK_J_PER_NODE, rtol=1e-10)
                acc["head_solve"][p] = host(xz).reshape(6, Nn)
            acc["head_solve_exact"] = Z
            xk = torch.zeros_like(bz)
            lk = torch.zeros_like(bz)
            B.birk_kkt_solve(plan64, J, bz, xk, lk, jac_kind=B.BIRK_J_PER_NODE, rtol=1e-10)
            acc["head_kkt_chi"] = host(xk).reshape(6, Nn)
            acc["newton_err"] = out["newton_ivp"]["max_abs_err_vs_kepler"] / float(np.max(np.abs(ivp["exact"])))
        if extra:
            c0d = {}
            for Nn0, d in small.items():
                B.birk_apply(d["plan"], d["v"], d["out"])
                ap = host(d["out"]).reshape(6, Nn0)
                B.birk_apply_T(d["plan"], d["v"], d["out"])
                apT = host(d["out"]).reshape(6, Nn0)
                c0d[Nn0] = {"v": host(d["v"]).reshape(6, Nn0), "apply": ap, "apply_T": apT,
                            "solve": host(d["chi"])}
            X1, sp1 = wl.sparse_series(103, N1, 6, 16)
            v1 = D64(X1.ravel())
            o1 = torch.empty_like(v1)
            B.birk_apply(c1["plan"], v1, o1)
            acc["small"] = {"c0": c0d, "c1": {"N": N1, "specs": sp1, "apply": host(o1).reshape(6, N1 + 1),
                                              "solve": {"fp64": host(c1["chi"]),
                                                        "mixed": host(c1.get("sol_mixed", c1["chi"]))}}}
            # batch: exact series on every component of every instance, and the solves
            bX, bref_specs = [], []
            for i, ins in enumerate(binst):
                Xi, si = wl.sparse_series([104, i], ins.N_n - 1, ins.n_x, 8)
                bX.append(Xi.ravel())
                bref_specs.append(si)
            bvs = D64(np.concatenate(bX))
            B.birk_apply(bplan64, bvs, bo)
            bres = host(bo)

            def batched_apply_err(bk, bres=bres, bref_specs=bref_specs):
                worst = 0.0
                o = 0
                for ins, si in zip(binst, bref_specs):
                    n0 = ins.n_x * ins.N_n
                    ref = np.stack([bk.sparse_mode_exact(ins.N_n - 1, m, al) for m, al in si])
                    got = bres[o:o + n0].reshape(ins.n_x, ins.N_n)
                    worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
                    o += n0
                return worst
            acc["batched"] = {"insts": binst, "apply_err": batched_apply_err,
                              "fp64": host(bsol["fp64"]) if "fp64" in bsol else host(bchi),
                              "mixed": host(bsol["mixed"]) if "mixed" in bsol else host(bchi)}
            if a.products_only:
                del acc["batched"]["fp64"], acc["batched"]["mixed"]
            # many RHS: six exact series repeated over the 192 components
            mX, msp = wl.sparse_series(105, mNn - 1, 6, 16)
            mvv = np.tile(mX, (mR, 1)).ravel()
            mres = {}
            for p, key in ((B.BIRK_F64, "f64"), (B.BIRK_F32, "f32"), (B.BIRK_DF32, "df32")):
                if key == "f64":
                    vin_m, out_m = D64(mvv), mo
                elif key == "f32":
                    vin_m, out_m = D64(mvv).float(), mo32
                else:
                    t = D64(mvv)
                    h_ = t.float()
                    l_ = (t - h_.double()).float()
                    vin_m, out_m = torch.stack([h_, l_], dim=1).reshape(-1).contiguous(), modf
                B.birk_apply(mplans[p], vin_m, out_m)
                r = host(out_m)
                if key == "df32":
                    r = r.reshape(-1, 2)
                    r = r[:, 0].astype(np.float64) + r[:, 1].astype(np.float64)
                mres[key] = r.astype(np.float64)
            acc["many_rhs"] = {"N": mNn - 1, "specs": msp, **mres}
        torch.cuda.synchronize()
        print("[bench] oracle leg: errors and the oracle's own timing", file=sys.stderr, flush=True)
        err, base = oracle_leg(a, acc, nproc)
        out["err_vs_oracle"] = err
        out["cpu_baseline"] = base
    if not a.no_cpu_context and not a.headline_only:
        print("[bench] CPU context: the fast method with scipy", file=sys.stderr, flush=True)
        out["cpu_context"] = cpu_context(nproc)
    plans = [plan64, planmx]
    if extra:
        plans += [bplan64, bplanmx, c1["plan"], c1["planmx"]] + list(mplans.values()) + [d["plan"] for d in small.values()]
    for p in plans:
        p.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
