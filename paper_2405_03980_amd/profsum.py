"""Summary of rocprofv3 output (rocpd SQLite databases) for the committed profiles.

Reads one sub-directory per rocprofv3 run under a root folder:

* ``trace``  -- ``--kernel-trace --stats``: per-kernel call count, mean duration, share;
* ``fetch`` / ``write`` -- ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` of the benchmark;
* ``copyf`` / ``copyw`` -- the same two counters over a plain 1 GiB device copy, which
  fix the factor between each counter and true bytes;
* ``sq`` -- one pass of SQ_* counters.

Prints a text summary and, with a second argument, writes the per-kernel HBM traffic
(KiB per dispatch plus the copy calibration) as JSON, stamped with a hash of the kernel
sources so that a reader can tell when the figures are stale.

    python -m paper_2405_03980_amd.profsum gpurun_out/prof profiles/counters.json
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_MIB = 1024
KERNEL_GROUPS = {"k_keys<float>": "keys", "k_scatter": "scatter", "k_reorder<float>": "reorder",
                 "k_density_cand<true>": "density", "k_force_cand<true>": "force",
                 "k_density_brick<true>": "density", "k_force_brick<true>": "force"}


def source_sha() -> str:
    """Hash of the device sources (the same one bench.py compares against)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "sph_device.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return name.replace("sph::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def _counters(db: str):
    con = sqlite3.connect(db)
    out = defaultdict(lambda: defaultdict(list))
    for name, cname, val in con.execute(
            "select kernel_name, counter_name, value from counters_collection"):
        out[_short(name)][cname].append(val)
    return out


def _avg(c, kernel, counter):
    v = c.get(kernel, {}).get(counter, [])
    return sum(v) / len(v) if v else None


def summarize(root: str, out_json: str | None = None, workload: str = "") -> dict:
    allc = {}
    for sub in sorted(os.listdir(root)):
        dbs = glob.glob(os.path.join(root, sub, "**", "*.db"), recursive=True)
        if not dbs:
            continue
        print(f"== {sub}")
        if sub == "trace":
            con = sqlite3.connect(dbs[0])
            for r in con.execute("select name, total_calls, average, percentage from top_kernels"):
                print(f"  {_short(r[0]):28s} calls={r[1]:4d} avg_us={r[2]:10.1f}"
                      f" share={r[3]:5.1f}%")
            continue
        c = _counters(dbs[0])
        allc[sub] = c
        for k, d in c.items():
            vals = ", ".join(f"{cn}={sum(v) / len(v):.4g}" for cn, v in sorted(d.items()))
            print(f"  {k:28s} n={len(next(iter(d.values())))} {vals}")
    res = {}
    if all(k in allc for k in ("fetch", "write", "copyf", "copyw")):
        kib = COPY_MIB * 1024
        cf = _avg(allc["copyf"], "__amd_rocclr_copyBuffer", "FETCH_SIZE")
        cw = _avg(allc["copyw"], "__amd_rocclr_copyBuffer", "WRITE_SIZE")
        kern = {}
        for kname, group in KERNEL_GROUPS.items():
            f = _avg(allc["fetch"], kname, "FETCH_SIZE")
            w = _avg(allc["write"], kname, "WRITE_SIZE")
            if f is not None and w is not None and group not in kern:
                kern[group] = {"kernel": kname, "FETCH_SIZE_KiB": f, "WRITE_SIZE_KiB": w}
        sq = {}
        for kname, group in KERNEL_GROUPS.items():
            if kname in allc.get("sq", {}) and group not in sq:
                sq[group] = {cn: sum(v) / len(v) for cn, v in allc["sq"][kname].items()}
        res = {"source_sha": source_sha(), "fetch_scale": kib / cf, "write_scale": kib / cw,
               "copy_MiB": COPY_MIB, "copy_FETCH_SIZE_KiB": cf, "copy_WRITE_SIZE_KiB": cw,
               "kernels": kern, "sq": sq, "workload": workload}
        if out_json:
            with open(out_json, "w") as fh:
                json.dump(res, fh, indent=1)
            print("wrote", out_json)
    return res


if __name__ == "__main__":
    summarize(sys.argv[1] if len(sys.argv) > 1 else "gpurun_out/prof",
              sys.argv[2] if len(sys.argv) > 2 else None,
              "cylinder nz=184 (19,567,296 particles), FP32-mixed, tuned launch")
