"""Benchmark of the Birkhoff hot path on one MI355X.

Headline workload: the million-point configuration -- N_n = 2^20 + 1 CGL nodes, n_x = 6
states, time-varying Jacobian of the two-body problem along a seeded Keplerian orbit
(a = 7000 km, e ~ U(0, 0.2), canonical units, one period), synthetic inputs.

One step is one pass of the whole hot path:
  * headline: B^a v (FastBV) in double, once per buffer of a rotation of R
    input/output pairs whose footprint exceeds the 256 MB Infinity Cache, so that every
    product reads its input from HBM; B^aT g in double (same rotation); B^a v in float;
    P^{-1} y (inverse-preconditioner scan) and P y in double; FastAX (x - B^a (J x)) in
    double; the preconditioned GMRES solve to
    relative residual 1e-10, once with float Krylov bulk inside double refinement
    (mixed) and once in double (FP64); the b-form products B^b v, B^bT g and the
    endpoint row x^b = x^a + w^T v in double; Newton's method on the nonlinear two-body
    IVP over one period (e = 0.15) from the circular orbit, to ||G|| <= 1e-13 ||X||;
  * batched uneven workload: 512 LTI instances (N_n log-uniform in [2^8, 2^16], n_x in
    {4, 6, 12}) in one plan: B^a v in double, and the mixed and FP64 solves to 1e-10;
  * many-RHS workload: 32 right-hand sides of N_n = 2^18 + 1, n_x = 6 in one plan:
    B^a v in compensated double-float (DF32), in double and in float.

value = Gpts/s of the headline double B^a product = n / (mean duration of one
birk_apply), timed with HIP events on the plan's stream over the timed region.  The other
rows are reported under "secondary", "solve", "newton_ivp", "batched" and "many_rhs".

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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip birk_plan_tune (default tile schedules)")
    ap.add_argument("--products-only", action="store_true", help="skip the solves (for profiling runs)")
    ap.add_argument("--headline-only", action="store_true", help="skip the batched and many-RHS workloads")
    ap.add_argument("--cpu-sample", type=int, default=400, help="rows of B^a the oracle computes")
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
    from paper_2509_01855_amd.traffic import schedule_key
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


def cpu_baseline(N: int, sample_rows: int, v):
    """Time the FP64 oracle on a bounded sample of the same product: `sample_rows` outputs of
    B^a v at N_n = N + 1, each from one O(N log N) row of B^a (oracle.birkhoff.ba_row)."""
    import numpy as np
    from oracle import birkhoff as bk
    rows = np.linspace(0, N, sample_rows).astype(np.int64)
    t0 = time.perf_counter()
    acc = 0.0
    for i in rows:
        acc += float(bk.ba_row(N, int(i)) @ v)
    dt = time.perf_counter() - t0
    return {"value": sample_rows / dt / 1e9, "unit": "Gpts/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample_rows} outputs of B^a v (one component) at N_n={N + 1}, each a full row of "
                      f"B^a from oracle.birkhoff.ba_row (closed-form coefficients + scipy DCT-I, "
                      f"single thread), {dt:.1f} s"}


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

    # ---- batched uneven workload
    extra = not a.headline_only
    if extra:
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

    xa_end = torch.zeros(nx, dtype=torch.float64, device="cuda")
    xb_end = torch.empty_like(xa_end)

    # autotuner of the power-of-two product path (plan setup, outside the timed region)
    tuned = {}
    # the double plan's default schedule unless the tuner picks another
    head_sched = traffic_key(int(os.environ.get("BIRK_FAST_SPLIT", "0")), int(os.environ.get("BIRK_FAST_TB", "0")),
                             int(os.environ.get("BIRK_FAST_XCD", "1")), int(os.environ.get("BIRK_FAST_NARROW", "1")))
    if not a.no_tune:
        print("[bench] autotuning the power-of-two plans", file=sys.stderr, flush=True)
        tplans = {"headline_f64": plan64, "headline_f32": planmx}
        if extra:
            tplans.update({"many_rhs_f64": mplans[B.BIRK_F64], "many_rhs_f32": mplans[B.BIRK_F32],
                           "many_rhs_df32": mplans[B.BIRK_DF32]})
        for name, plan in tplans.items():
            rep = B.birk_plan_tune(plan)
            tuned[name] = [ln.split(" chosen ")[0].split(":")[0] + ": " + ln.split(" chosen ")[1]
                           for ln in rep.splitlines() if " chosen " in ln]
            if name == "headline_f64":
                m = re.search(r"chosen \[split (\d+), tb (\d+), xcd (\d+), streams \d+, narrow (\d+)\]", rep)
                head_sched = traffic_key(int(m.group(1)), int(m.group(2)), int(m.group(3)), int(m.group(4)))
        torch.cuda.synchronize()

    def step(timed: bool):
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
            tm.region("b_apply", lambda: B.birk_apply(bplan64, bv, bo))
            tm.region("m_apply_f64", lambda: B.birk_apply(mplans[B.BIRK_F64], mv, mo))
            tm.region("m_apply_f32", lambda: B.birk_apply(mplans[B.BIRK_F32], mv32, mo32))
            tm.region("m_apply_df32", lambda: B.birk_apply(mplans[B.BIRK_DF32], mvdf, modf))
        torch.cuda.synchronize()
        tm.collect(timed)
        if not a.products_only:
            solves = [("mixed", planmx, J, beta, chi, B.BIRK_J_PER_NODE),
                      ("fp64", plan64, J, beta, chi, B.BIRK_J_PER_NODE)]
            if extra:
                solves += [("b_mixed", bplanmx, bJ, bbeta, bchi, B.BIRK_J_CONSTANT),
                           ("b_fp64", bplan64, bJ, bbeta, bchi, B.BIRK_J_CONSTANT)]
            for name, plan, Jm, bt, ch, jk in solves:
                info = tm.wall(name if timed else "_warm",
                               lambda: B.birk_krylov_solve(plan, Jm, bt, ch, jk, rtol=1e-10))
                solve_info[name] = info

            def newton():
                ivp_X.copy_(ivp_guess)
                ivp_info.update(B.birk_newton_ivp(plan64, ivp_xa, ivp_X, mu=ivp["mu"], scale=ivp["scale"]))
            tm.wall("newton" if timed else "_warm", newton)

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
    if not a.products_only:
        err = float(np.max(np.abs(ivp_X.cpu().numpy().reshape(6, Nn) - ivp["exact"])))
        out["newton_ivp"] = {
            "workload": "two-body IVP over one period (e = 0.15), N_n = 2^20 + 1, Newton from the circular orbit",
            "ms": round(tm.mean_ms("newton"), 3), "newton_iters": ivp_info["newton_iters"][0],
            "linear_iters": ivp_info["linear_iters"][0], "rel_resid": ivp_info["rel_resid"][0],
            "max_abs_err_vs_kepler": err}
    if extra:
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
        # deviation of the double-float and float products from the double product
        hi_lo = modf.view(-1, 2).double()
        dfv = hi_lo[:, 0] + hi_lo[:, 1]
        scale = float(mo.abs().max())
        dev_df = float((dfv - mo).abs().max()) / scale
        dev_32 = float((mo32.double() - mo).abs().max()) / scale
        out["many_rhs"] = {
            "workload": "32 RHS x n_x = 6 at N_n = 2^18 + 1 in one plan (192 components)", "n": mn,
            "apply_df32_us": us("m_apply_df32"), "apply_f64_us": us("m_apply_f64"), "apply_f32_us": us("m_apply_f32"),
            "apply_df32_gpts": round(mn / (tm.mean_ms("m_apply_df32") * 1e-3) / 1e9, 3),
            "apply_f64_gpts": round(mn / (tm.mean_ms("m_apply_f64") * 1e-3) / 1e9, 3),
            "apply_f32_gpts": round(mn / (tm.mean_ms("m_apply_f32") * 1e-3) / 1e9, 3),
            "max_dev_vs_f64": {"df32": dev_df, "f32": dev_32},
        }
    if extra:
        out["graphs"] = graph_replay_timing(B, torch)
    if not a.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(N, a.cpu_sample, vin[0][:Nn].cpu().numpy())
    for p in [plan64, planmx] + ([bplan64, bplanmx] + list(mplans.values()) if extra else []):
        p.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
