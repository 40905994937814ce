"""Turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs into HBM bytes per B^a product.

The record of one tile schedule (taken from the BIRK_FAST_SPLIT / BIRK_FAST_TB /
BIRK_FAST_XCD / BIRK_FAST_NARROW environment of the counter runs, defaults 0 / 0 / 1 / 1
for a double plan)
is merged into
<out.json>, which keeps one record per schedule for the current kernel sources.

Usage (after the four counter runs described in profiles/README.md):
    python bench_traffic.py <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir> <out.json>

Each counter is scaled by what it reads for a plain 1 GiB copy (bench.py --calibrate-copy):
scale = known bytes / counter value, separately for FETCH_SIZE and WRITE_SIZE.  The
product's bytes are the per-dispatch means of its three kernels (passes A, B, C of the
double forward product) summed.
"""

from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["paper_2509_01855_amd/csrc/birk_fast.hip", "paper_2509_01855_amd/csrc/birk_dct.hip",
           "paper_2509_01855_amd/csrc/birk_fft.h"]


def schedule_key(split, tb, xcd, narrow=0):
    """What fixes the kernels of the double product at N = 2^20: the split of 2N = L1 L2,
    the rows per pass-B tile of the register kernel (4 when asked for, else 2), the tile
    order and the column tiles of passes A and C (4 with narrow where L1 = 2^10, else 8).
    (The multi-stream schedules run the same kernels.)"""
    narrow_applies = bool(narrow) and not split     # L1 = 2^10 only with split 0 at N = 2^20
    return {"split": 1 if split else 0, "rows_b": 4 if tb == 4 else 2, "xcd": 1 if xcd else 0,
            "cols_ac": 4 if narrow_applies else 8}


def _schedule():
    """Tile schedule of the counter runs (bench.py --no-tune with the environment defaults)."""
    return schedule_key(int(os.environ.get("BIRK_FAST_SPLIT", "0")),
                        max(0, min(14, int(os.environ.get("BIRK_FAST_TB", "0")))) & ~1,
                        int(os.environ.get("BIRK_FAST_XCD", "1")),
                        int(os.environ.get("BIRK_FAST_NARROW", "1")))
import re

# forward double product: pass A, pass B (TRANS = 0), pass C (TRANS = 0); the
# fixed-length kernels (suffix 2) are used where they apply
PASSES = (r"k_fastA2?<double", r"k_fastB[23]<double, 0,|k_fastB<double, \d+, 0>", r"k_fastC2?<double, 0")


def _rows(d):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(f[0])))


def _mean_by_kernel(d, counter):
    acc = {}
    for r in _rows(d):
        if r["Counter_Name"] != counter:
            continue
        acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _copy_value(d, counter):
    vals = [v for k, v in _mean_by_kernel(d, counter).items() if "copy" in k.lower() or "elementwise" in k.lower()]
    return max(vals)


def main():
    fetch_dir, write_dir, cf_dir, cw_dir, out = sys.argv[1:6]
    copy_bytes = float(1 << 30)
    sf = copy_bytes / _copy_value(cf_dir, "FETCH_SIZE")
    sw = copy_bytes / _copy_value(cw_dir, "WRITE_SIZE")
    fetch = _mean_by_kernel(fetch_dir, "FETCH_SIZE")
    write = _mean_by_kernel(write_dir, "WRITE_SIZE")
    per = {}
    for key in PASSES:
        names = [k for k in fetch if re.search(key, k)]
        if not names:
            raise SystemExit(f"no kernel matching {key} in the counter runs")
        name = names[0]
        per[name] = {"fetch_bytes": fetch[name] * sf, "write_bytes": write[name] * sw}
    total = sum(v["fetch_bytes"] + v["write_bytes"] for v in per.values())
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    rec = {"schedule": _schedule(), "bytes_per_product": total, "per_kernel": per, "fetch_scale": sf,
           "write_scale": sw}
    doc = {"source_sha256": h.hexdigest(), "records": []}
    if os.path.exists(out):
        old = json.load(open(out))
        if old.get("source_sha256") == doc["source_sha256"]:
            doc["records"] = [r for r in old.get("records", []) if r["schedule"] != rec["schedule"]]
    doc["records"].append(rec)
    json.dump(doc, open(out, "w"), indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
