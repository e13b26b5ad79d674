#!/usr/bin/env python
"""Throughput of the two-fluid SPH step on one MI355X.

Workload: the 19.57M-particle rotating cylinder (R = H = 1, dx = 1/184, Wendland C2,
h = 1.3 dx, 70/30 inviscid/viscous fluid, three wall layers turning at Omega = 1, fluid at
rest plus N(0, 1e-3) noise), FP32-mixed path, dt = 1e-4.  A step is one velocity-Verlet
step of every particle: kick/drift, cell list, density/EOS, forces/torques.

Prints ONE JSON line: particle-updates/s (walls included, as the paper counts particles),
the per-kernel roofline of the dominant kernel from HIP events recorded on the library's
stream during the timed steps, the FP64 GPU path's step time, and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic work per fluid particle and step, FP32-mixed path:
# 80 neighbours on the lattice (r < 2h = 2.6 dx); flops of one evaluation of the pair
# formula averaged over the species mix (unlike pairs 42 %, viscous-viscous 9 %).
NEIGHBOURS = 80
FORCE_FLOPS_PER_PAIR = 52
DENSITY_FLOPS_PER_PAIR = 19
# Compulsory HBM bytes per particle of each kernel group (mixed precision).
BYTES_PER_PARTICLE = {
    "keys": 24 + 24 + 12 + 1 + 4 + 4,          # x, v, acc, sk -> key, slot
    "scan": 0.0,                                # per cell, counted below
    "scatter": 4 + 4 + 4 + 4,                   # key, slot, start -> tmp
    "reorder": 4 + 4 + 4 + 72 + 24 + 1 + 72 + 4 + 1 + 4,  # tmp, key, id, state -> state, pcell
    "density": 24 + 1 + 4 + 4 + 16 + 8,         # x, sk, pcell, cell_xyz -> aux, rho/P
    "force": 72 + 16 + 1 + 4 + 4 + 24,          # x, v, w, aux, sk, pcell, cell -> acc, alpha
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nz", type=int, default=184, help="cylinder resolution (184: 19.57M)")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2405_03980_amd", "tuned.json"))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device-to-device copy of this size (5 times), to "
                         "calibrate the HBM traffic counters, and exit")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    """Plain copy kernel of known size: FETCH_SIZE and WRITE_SIZE of these dispatches
    should each read `mib` MiB; their ratio to that is the counters' scale factor."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_MiB": mib, "bytes_per_copy": 4 * n}), flush=True)


def load_tuning(path, name):
    try:
        with open(path) as f:
            return json.load(f).get(name, {})
    except (OSError, ValueError):
        return {}


def cpu_baseline(nz: int, steps: int) -> dict:
    """The FP64 oracle on an 8-layer z-slab of the same cylinder (same dx, kernel, species
    mix and wall layers, z periodic over the slab): its per-particle cost is the full
    workload's; the rate is particle-updates per second of wall time on the host."""
    from oracle import oracle as O
    from paper_2405_03980_amd import inputs as I
    layers = 8
    w = I.make_cylinder(layers, H=layers / nz, seed=(3980, 3))
    s = O.State.from_workload(w)
    t0 = time.perf_counter()
    s.step(1e-4, 1.0, steps)
    dt = time.perf_counter() - t0
    return {"value": w.n * steps / dt, "unit": "particle-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of an {layers}-layer z-slab ({w.n} particles) of the "
                      f"nz={nz} cylinder, FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch
    from paper_2405_03980_amd import _lib as L
    from paper_2405_03980_amd import inputs as I
    from paper_2405_03980_amd import sim as S

    w = I.make_cylinder(args.nz, seed=(3980, 3))
    name = f"cylinder_nz{args.nz}"
    n, nf = w.n, w.n_fluid
    print(f"[bench] {name}: {n} particles ({nf} fluid)", file=sys.stderr, flush=True)

    def run(precision, steps, warmup, tuning):
        s = S.simulation_from(w, precision=precision)
        if tuning:
            s.set_tuning(**tuning)
        s.step(1e-4, w.Omega, warmup)
        s.sync()
        torch.cuda.synchronize()
        s.profile_begin()
        t0 = time.perf_counter()
        s.step(1e-4, w.Omega, steps)
        ms, nsteps = s.profile_end()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        s.sync()
        s.close()
        del s
        torch.cuda.empty_cache()
        return elapsed, ms, nsteps

    tuning = load_tuning(args.tuning, name)
    elapsed, ms, nsteps = run(L.FP32_MIXED, args.steps, args.warmup, tuning)
    assert nsteps == args.steps
    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    per = {k: v / nsteps for k, v in ms.items()}
    print(f"[bench] mixed: {ms_step:.3f} ms/step; per kernel (ms): "
          + ", ".join(f"{k}={v:.3f}" for k, v in per.items()), file=sys.stderr, flush=True)

    # Roofline of the dominant kernel (force sweep), from the events of the timed steps.
    dom = max(per, key=per.get)
    t_dom = per[dom] * 1e-3
    if dom in ("force", "density"):
        fpp = FORCE_FLOPS_PER_PAIR if dom == "force" else DENSITY_FLOPS_PER_PAIR
        units = nf if dom == "force" else n
        flops = units * NEIGHBOURS * fpp
        alu = flops / t_dom / 1e12
    else:
        alu = 0.0
    hbm = n * BYTES_PER_PARTICLE[dom] / t_dom / 1e9
    alu_frac, hbm_frac = alu / VALU_PEAK_TFLOPS, hbm / HBM_PEAK_GBS
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(alu, 3), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    roof.update({"kernel": dom, "avg_ms": round(per[dom], 4), "traffic": None,
                 "hbm_GBs": round(hbm, 1), "hbm_frac": round(hbm_frac, 4)})

    fp64 = None
    if args.fp64_steps > 0:
        e64, ms64, n64 = run(L.FP64, args.fp64_steps, 2, tuning)
        fp64 = {"ms_per_step": round(1e3 * e64 / args.fp64_steps, 3),
                "speedup_mixed_vs_fp64": round((e64 / args.fp64_steps) / (elapsed / args.steps), 3)}
        print(f"[bench] fp64: {fp64['ms_per_step']} ms/step", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.nz, args.cpu_steps)
    line = {
        "metric": "particle-updates/sec @19.6M particles, FP32-mixed vs FP64 at stated error",
        "value": value, "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"rotating cylinder, {n} particles ({nf} fluid), dx=1/{args.nz}, "
                               "Wendland C2, FP32-mixed, dt=1e-4",
                   "particles": n, "precision": "fp32_mixed", "tuning": tuning or "default"},
        "kernel_ms": {k: round(v, 4) for k, v in per.items()},
        "roofline": roof,
        "fp64_gpu": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
