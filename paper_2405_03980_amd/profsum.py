"""Summary of rocprofv3 output (rocpd SQLite databases) for the committed profiles.

Reads one sub-directory per rocprofv3 run under a root folder:

* ``trace``  -- ``--kernel-trace --stats``: per-kernel call count, mean duration, share;
* ``fetch`` / ``write`` -- ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` of the benchmark;
* ``copyf`` / ``copyw`` -- the same two counters over a plain 1 GiB device copy, which
  fix the factor between each counter and true bytes;
* ``sq`` -- one pass of SQ_* instruction counters;
* ``sq2`` -- one pass of SQ_* wait counters (where a kernel's waves spend their cycles).

Prints a text summary; with a second argument writes the per-kernel HBM traffic (KiB per
dispatch plus the copy calibration) as JSON, stamped with a hash of the kernel sources so
that a reader can tell when the figures are stale; with a third writes the same figures as
a markdown summary that lists the commands behind them (COMMANDS).

    python -m paper_2405_03980_amd.profsum gpurun_out/prof profiles/counters.json \
        profiles/sweeps_cylinder_19.57M.md
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
BENCH = ("python3 bench.py --steps 5 --warmup 2 --runs 1 --no-cpu-baseline --no-configs "
         "--fp64-steps 0 --batch-steps 0 --f1-steps 3")
COPY = "python3 bench.py --copy-calibration 1024"
SQ = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
      "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VALU")
SQ2 = ("SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_INSTS_VMEM_RD "
       "SQ_INST_CYCLES_VMEM_RD SQ_LDS_IDX_ACTIVE")
# One rocprofv3 run per sub-directory, from the repository root, with TMPDIR=/tmp.
COMMANDS = [
    ("trace", f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof/trace -o run -- {BENCH}"),
    ("fetch", f"rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/fetch -o run -- {BENCH}"),
    ("write", f"rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/write -o run -- {BENCH}"),
    ("copyf", f"rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/copyf -o run -- {COPY}"),
    ("copyw", f"rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/copyw -o run -- {COPY}"),
    ("sq", f"rocprofv3 --pmc {SQ} -d gpurun_out/prof/sq -o run -- {BENCH}"),
    ("sq2", f"rocprofv3 --pmc {SQ2} -d gpurun_out/prof/sq2 -o run -- {BENCH}"),
]
# VALU instruction issue capacity: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles
# on a 16-lane SIMD, at 2.4 GHz.
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
COPY_MIB = 1024
KERNEL_GROUPS = {"k_keys<float>": "keys", "k_scatter": "scatter", "k_reorder<float>": "reorder",
                 "k_density_cand<true, false, 32>": "density", "k_force_cand<true>": "force",
                 "k_density_cand<true, true, 32>": "density_flagging",
                 "k_filter_cand<true>": "filter", "k_collide": "collide"}


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


def summarize(root: str, out_json: str | None = None, workload: str = "",
              out_md: str | None = None) -> dict:
    allc = {}
    trace = []
    for sub in sorted(os.listdir(root)):
        dbs = glob.glob(os.path.join(root, sub, "**", "*.db"), recursive=True)
        if not dbs:
            continue
        print(f"== {sub}")
        if sub == "trace":
            con = sqlite3.connect(dbs[0])
            for r in con.execute("select name, total_calls, average, percentage from top_kernels"):
                trace.append((_short(r[0]), int(r[1]), float(r[2]), float(r[3])))
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
            if kname in allc.get("sq2", {}) and group in sq:
                sq[group].update({f"{cn}@2": sum(v) / len(v) for cn, v in allc["sq2"][kname].items()})
        res = {"source_sha": source_sha(), "fetch_scale": kib / cf, "write_scale": kib / cw,
               "copy_MiB": COPY_MIB, "copy_FETCH_SIZE_KiB": cf, "copy_WRITE_SIZE_KiB": cw,
               "kernels": kern, "sq": sq, "workload": workload}
        if out_json:
            with open(out_json, "w") as fh:
                json.dump(res, fh, indent=1)
            print("wrote", out_json)
        if out_md:
            with open(out_md, "w") as fh:
                fh.write(_markdown(res, trace))
            print("wrote", out_md)
    return res


def _markdown(res: dict, trace: list) -> str:
    avg_us = {name: us for name, _, us, _ in trace}
    out = [f"# rocprofv3: {res['workload']}", "",
           f"Kernel sources: `{res['source_sha']}` (sha256 prefix of `csrc/kernels.hip` + "
           "`csrc/sph_device.h`).", "",
           "Commands (repository root, `TMPDIR=/tmp`, one run each):", "", "```"]
    out += [c for _, c in COMMANDS]
    out += ["python3 -m paper_2405_03980_amd.profsum gpurun_out/prof profiles/counters.json "
            "profiles/<this file>", "```", "",
            "## Kernel trace (`--kernel-trace --stats`)", "",
            "| kernel | calls | mean us | share |", "|---|---|---|---|"]
    out += [f"| `{n}` | {c} | {us:.1f} | {sh:.1f}% |" for n, c, us, sh in trace]
    out += ["", "## HBM traffic per launch", "",
            f"Copy calibration: a {res['copy_MiB']} MiB device copy reads FETCH_SIZE = "
            f"{res['copy_FETCH_SIZE_KiB']:.0f} KiB and WRITE_SIZE = "
            f"{res['copy_WRITE_SIZE_KiB']:.0f} KiB, so the factors are "
            f"{res['fetch_scale']:.4f} (fetch) and {res['write_scale']:.4f} (write).", "",
            "| group | kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled GB | GB/s at mean time |",
            "|---|---|---|---|---|---|"]
    for g, k in res["kernels"].items():
        gb = 1024.0 * (k["FETCH_SIZE_KiB"] * res["fetch_scale"]
                       + k["WRITE_SIZE_KiB"] * res["write_scale"]) / 1e9
        us = avg_us.get(k["kernel"])
        bw = f"{gb / (us * 1e-6):.0f}" if us else "-"
        out.append(f"| {g} | `{k['kernel']}` | {k['FETCH_SIZE_KiB']:.0f} | "
                   f"{k['WRITE_SIZE_KiB']:.0f} | {gb:.2f} | {bw} |")
    out += ["", "## SQ counters per launch", "",
            "VALU issue = SQ_INSTS_VALU / (mean time x "
            f"{VALU_ISSUE_PER_S:.3e} wave64 instructions/s).", "",
            "| group | VALU insts | SALU insts | LDS insts | LDS bank-conflict cycles | "
            "VALU issue |", "|---|---|---|---|---|---|"]
    for g, c in res["sq"].items():
        us = avg_us.get(res["kernels"].get(g, {}).get("kernel", ""))
        util = f"{100 * c['SQ_INSTS_VALU'] / (us * 1e-6 * VALU_ISSUE_PER_S):.0f}%" if us else "-"
        out.append(f"| {g} | {c['SQ_INSTS_VALU']:.3e} | {c['SQ_INSTS_SALU']:.3e} | "
                   f"{c['SQ_INSTS_LDS']:.3e} | {c['SQ_LDS_BANK_CONFLICT']:.3e} | {util} |")
    waits = {g: c for g, c in res["sq"].items() if "SQ_WAVE_CYCLES@2" in c}
    if waits:
        out += ["", "## Where the waves wait (second SQ pass)", "",
                "Fractions of SQ_WAVE_CYCLES (summed over waves) spent waiting on anything, "
                "waiting to issue, and waiting on LDS instructions; vector memory reads per "
                "wave.", "",
                "| group | wait any | wait inst any | wait inst LDS | VMEM reads per wave |",
                "|---|---|---|---|---|"]
        for g, c in waits.items():
            wc = c["SQ_WAVE_CYCLES@2"] or 1.0
            out.append(f"| {g} | {c['SQ_WAIT_ANY@2'] / wc:.2f} | {c['SQ_WAIT_INST_ANY@2'] / wc:.2f} | "
                       f"{c['SQ_WAIT_INST_LDS@2'] / wc:.2f} | "
                       f"{c['SQ_INSTS_VMEM_RD@2'] / max(c['SQ_WAVES@2'], 1.0):.1f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    summarize(sys.argv[1] if len(sys.argv) > 1 else "gpurun_out/prof",
              sys.argv[2] if len(sys.argv) > 2 else None,
              "cylinder nz=184 (19,567,296 particles), FP32-mixed, tuned launch",
              sys.argv[3] if len(sys.argv) > 3 else None)
