"""Benchmark of the Birkhoff hot path on one MI355X.

Workload: the million-point configuration -- N_n = 2^20 + 1 CGL nodes, n_x = 6 states,
time-varying Jacobian of the two-body problem along a seeded Keplerian orbit
(a = 7000 km, e ~ U(0, 0.2), canonical units, one period), synthetic inputs.

One step is one pass of the whole hot path on that batch:
  * B^a v (FastBV) in double, once per buffer of a rotation of R input/output pairs
    whose footprint exceeds the 256 MB Infinity Cache, so that every product reads its
    input from HBM;
  * B^aT g in double (same rotation);
  * B^a v in float;
  * P^{-1} y (preconditioner inverse scan) in double;
  * the preconditioned GMRES solve to relative residual 1e-10, once with float Krylov
    bulk inside double refinement (mixed) and once in double (FP64).

value = Gpts/s of the double B^a product = n / (mean duration of one birk_apply), timed
with HIP events on the plan's stream over the timed region.  The solve times (mixed vs
FP64 at the same 1e-10 residual) are reported in "solve".

`python bench.py --gpus N --steps K --warmup W`; N must be 1 (single-GPU build).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Birkhoff matvec Gpts/s at N=2^20; solve time mixed vs FP64 at 1e-10 resid"
KERNEL_SOURCES = ["paper_2509_01855_amd/csrc/birk_fast.hip", "paper_2509_01855_amd/csrc/birk_dct.hip"]
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=20, help="N = 2^log2n (N_n = N + 1)")
    ap.add_argument("--rotation", type=int, default=6, help="input/output buffer pairs per product sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--products-only", action="store_true", help="skip the solves (for profiling runs)")
    ap.add_argument("--cpu-sample", type=int, default=200, help="rows of B^a the oracle computes")
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


def traffic_record(kernel_sources):
    """Measured HBM bytes per product from profiles/, if the kernels are unchanged since."""
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
    return rec


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
    N = 1 << a.log2n
    Nn = N + 1
    nx = 6
    n = Nn * nx
    print(f"[bench] building inputs N_n={Nn} n_x={nx}", file=sys.stderr, flush=True)
    inst = wl.kepler_instance(2, Nn)
    stream = torch.cuda.current_stream()
    plan64 = B.birk_plan_create([Nn], [nx], B.BIRK_F64, stream)
    planmx = B.birk_plan_create([Nn], [nx], B.BIRK_F32_REFINE_F64, stream)
    J = torch.from_numpy(inst.J.ravel()).to("cuda")
    R = max(1, a.rotation)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    vin = [torch.randn(n, dtype=torch.float64, device="cuda", generator=gen) for _ in range(R)]
    vout = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(R)]
    v32 = [x.float() for x in vin[:2]]
    o32 = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(2)]
    ex = inst.extra
    Z = np.concatenate([ex["v"], ex["acc"]])
    beta_np = np.repeat(inst.x_a, Nn)
    beta = torch.from_numpy(beta_np).to("cuda")
    chi = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rec = {"apply": [], "apply_T": [], "apply_f32": [], "pinv": [], "mixed": [], "fp64": []}
    solve_info = {}

    def step(timed: bool):
        pairs = []
        for i in range(R):
            e0, e1 = ev(), ev()
            e0.record(stream)
            B.birk_apply(plan64, vin[i], vout[i])
            e1.record(stream)
            pairs.append(("apply", e0, e1))
        for i in range(R):
            e0, e1 = ev(), ev()
            e0.record(stream)
            B.birk_apply_T(plan64, vin[i], vout[(i + 1) % R])
            e1.record(stream)
            pairs.append(("apply_T", e0, e1))
        for i in range(2):
            e0, e1 = ev(), ev()
            e0.record(stream)
            B.birk_apply(planmx, v32[i], o32[i])
            e1.record(stream)
            pairs.append(("apply_f32", e0, e1))
        e0, e1 = ev(), ev()
        e0.record(stream)
        B.birk_precond(plan64, J, vin[0], vout[1], 1, B.BIRK_J_PER_NODE)
        e1.record(stream)
        pairs.append(("pinv", e0, e1))
        if not a.products_only:
            for name, plan in (("mixed", planmx), ("fp64", plan64)):
                t0 = time.perf_counter()
                info = B.birk_krylov_solve(plan, J, beta, chi, B.BIRK_J_PER_NODE, rtol=1e-10)
                dt = (time.perf_counter() - t0) * 1e3
                if timed:
                    rec[name].append(dt)
                    solve_info[name] = info
        torch.cuda.synchronize()
        if timed:
            for name, e0, e1 in pairs:
                rec[name].append(e0.elapsed_time(e1))

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

    mean = lambda xs: float(sum(xs) / len(xs)) if xs else float("nan")  # noqa: E731
    t_apply = mean(rec["apply"]) * 1e-3
    gpts = n / t_apply / 1e9
    bytes_alg = 2.0 * n * 8.0
    achieved = bytes_alg / t_apply / 1e9
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
                                         "solves": 0 if a.products_only else 2}},
        "roofline": {"bound": "hbm", "kernel": "birk_apply (FastBV, three-pass, double)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": bytes_alg, "avg_launch_us": round(t_apply * 1e6, 2)},
        "secondary": {
            "apply_f64_us": round(mean(rec["apply"]) * 1e3, 2),
            "apply_T_f64_us": round(mean(rec["apply_T"]) * 1e3, 2),
            "apply_f32_us": round(mean(rec["apply_f32"]) * 1e3, 2),
            "apply_f32_gpts": round(n / (mean(rec["apply_f32"]) * 1e-3) / 1e9, 3),
            "precond_inverse_f64_us": round(mean(rec["pinv"]) * 1e3, 2),
        },
    }
    tr = traffic_record(KERNEL_SOURCES)
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes_per_product"]
        out["roofline"]["traffic_source"] = "profiles/apply_f64_traffic.json"
    if not a.products_only:
        mx, f64 = mean(rec["mixed"]), mean(rec["fp64"])
        out["solve"] = {
            "rtol": 1e-10,
            "mixed_ms": round(mx, 3), "fp64_ms": round(f64, 3), "speedup_mixed_vs_fp64": round(f64 / mx, 3),
            "mixed": {k: solve_info["mixed"][k] for k in ("inner_iters", "outer_iters", "rel_resid")},
            "fp64": {k: solve_info["fp64"][k] for k in ("inner_iters", "outer_iters", "rel_resid")},
        }
    if not a.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(N, a.cpu_sample, vin[0][:Nn].cpu().numpy())
    plan64.destroy()
    planmx.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
