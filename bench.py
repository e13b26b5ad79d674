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
    "scatter": 4 + 4 + 4 + 4 + 4 + 4,           # key, slot, start, id -> tmp, idt
    "reorder": 4 + 4 + 4 + 72 + 24 + 1 + 72 + 4 + 1 + 4,  # tmp, key, id, state -> state, pcell
    "density": 24 + 1 + 4 + 4 + 16 + 8,         # x, sk, pcell, cell_xyz -> aux, rho/P
    "force": 72 + 16 + 1 + 4 + 4 + 24,          # x, v, w, aux, sk, pcell, cell -> acc, alpha
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nz", type=int, default=184, help="cylinder resolution (184: 19.57M)")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2405_03980_amd", "tuned.json"))
    ap.add_argument("--f1-steps", type=int, default=20,
                    help="timed steps with the pressure filter and the collision step on (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the batched 64-instance ensemble (0: skip)")
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


TUNING_KEYS = ("block_density", "block_force", "block_stream", "use_graph", "sweep")


def load_tuning(path, name):
    """Tuned settings of a workload: (launch tuning for sph_tuning, cell factor)."""
    try:
        with open(path) as f:
            t = json.load(f).get(name, {})
    except (OSError, ValueError):
        t = {}
    return {k: v for k, v in t.items() if k in TUNING_KEYS}, int(t.get("cell_factor", 1))


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


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "sph_device.h"):
        with open(os.path.join(ROOT, "paper_2405_03980_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration), or None when the
    kernel source has changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_sha") != kernel_source_sha() or kernel not in c.get("kernels", {}):
        return None
    k = c["kernels"][kernel]
    return 1024.0 * (k["FETCH_SIZE_KiB"] * c["fetch_scale"] + k["WRITE_SIZE_KiB"] * c["write_scale"])


def batch_bench(steps: int, tuning_path: str) -> dict:
    """The 64-instance ensemble (20k-300k particles each, viscous fraction 0.05-0.5,
    Omega 0.5-2), FP32-mixed: all instances in shared launches replayed from a hipGraph,
    against the same instances stepped one after another."""
    import torch
    from paper_2405_03980_amd import inputs as I
    from paper_2405_03980_amd import sim as S
    ws = I.make_batch(64)
    tun, cf = load_tuning(tuning_path, "batch64")
    for w in ws:
        w.params = dict(w.params, cell_factor=cf)
    Om = [w.Omega for w in ws]
    N = sum(w.n for w in ws)
    b = S.batch_from(ws)
    if tun:
        b.set_tuning(**tun)
    b.step(1e-4, Om, 4)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(1e-4, Om, steps)
    b.sync()
    el = time.perf_counter() - t0
    b.close()
    del b
    seq_steps = max(2, steps // 4)
    sims = [S.simulation_from(w) for w in ws]
    for s_, w in zip(sims, ws):
        s_.step(1e-4, w.Omega, 2)
    for s_ in sims:
        s_.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(seq_steps):
        for s_, w in zip(sims, ws):
            s_.step(1e-4, w.Omega, 1)
    for s_ in sims:
        s_.sync()
    el_seq = time.perf_counter() - t0
    for s_ in sims:
        s_.close()
    del sims
    torch.cuda.empty_cache()
    ms = 1e3 * el / steps
    ms_seq = 1e3 * el_seq / seq_steps
    return {"value": N * steps / el, "unit": "particle-updates/s", "n_inst": len(ws),
            "tuning": tun or "default", "cell_factor": cf,
            "particles": N, "ms_per_step": round(ms, 3), "sequential_ms_per_step": round(ms_seq, 3),
            "speedup_vs_sequential": round(ms_seq / ms, 2)}


def field_errors(a: dict, b: dict, fluid) -> dict:
    """Normwise relative difference of a against b over fluid particles."""
    out = {}
    for k in ("rho", "P", "v", "omega", "acc"):
        x, y = a[k][..., fluid], b[k][..., fluid]
        if x.ndim == 2:
            d, r = np.sqrt(((x - y) ** 2).sum(0)), np.sqrt((y * y).sum(0))
        else:
            d, r = np.abs(x - y), np.abs(y)
        out[k] = float(d.max() / max(r.max(), 1e-300))
    return out


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

    def run(precision, steps, warmup, tuning, vortex=False, extra=None):
        tun, cf = tuning
        s = S.Simulation(dict(w.params, cell_factor=cf, **(extra or {})), w.n, precision=precision)
        if tun:
            s.set_tuning(**tun)
        s.init(w.x, w.v, w.omega, w.species, w.kind)
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
        fields = s.read(("rho", "P", "v", "omega", "acc"))
        if vortex:
            # the vortex diagnostic of the z = 0 section on the state just stepped
            s.vortex_image(0.0, 0.5, 3, to_numpy=False)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            cnt, img, _ = s.vortex_image(0.0, 0.5, 3, to_numpy=False)
            torch.cuda.synchronize()
            fields["vortex"] = {"ms": round(1e3 * (time.perf_counter() - t1), 3), "z0": 0.0,
                                "theta": 0.5, "min_pixels": 3, "count": cnt,
                                "image": [int(img.shape[0]), int(img.shape[1])]}
        s.close()
        del s
        torch.cuda.empty_cache()
        return elapsed, ms, nsteps, fields

    tuning = load_tuning(args.tuning, name)
    elapsed, ms, nsteps, f_mixed = run(L.FP32_MIXED, args.steps, args.warmup, tuning, vortex=True)
    vortex = f_mixed.pop("vortex")
    print(f"[bench] vortex diagnostic: {vortex}", file=sys.stderr, flush=True)
    assert nsteps == args.steps
    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    per = {k: v / nsteps for k, v in ms.items() if k not in ("collide", "filter")}
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
    traffic = measured_traffic(dom)
    roof.update({"kernel": dom, "avg_ms": round(per[dom], 4),
                 "traffic": None if traffic is None else round(traffic / 1e9, 3),
                 "traffic_unit": "GB per launch",
                 "hbm_GBs": round(hbm, 1), "hbm_frac": round(hbm_frac, 4)})

    fp64 = None
    if args.fp64_steps > 0:
        # the FP64 path runs the same warmup + timed step count, so that the fields of
        # both paths are compared after the same trajectory length
        n64 = args.fp64_steps
        e64, ms64, _, f64 = run(L.FP64, n64, args.warmup + args.steps - n64, tuning)
        fp64 = {"ms_per_step": round(1e3 * e64 / n64, 3),
                "speedup_mixed_vs_fp64": round((e64 / n64) / (elapsed / args.steps), 3),
                "mixed_error_vs_fp64": field_errors(f_mixed, f64, w.kind == I.FLUID),
                "after_steps": args.warmup + args.steps}
        print(f"[bench] fp64: {fp64['ms_per_step']} ms/step; mixed vs fp64 "
              f"{fp64['mixed_error_vs_fp64']}", file=sys.stderr, flush=True)
    f1 = None
    if args.f1_steps > 0:
        # the same workload with Algorithm 1's pressure filter and collision step switched
        # on (the lattice keeps every pair beyond the collision distance, so the collision
        # step costs its search only)
        f1p = dict(pressure_filter=1, coll_alpha=0.8, coll_e=0.3)
        e1, ms1, n1, _ = run(L.FP32_MIXED, args.f1_steps, args.warmup, tuning, extra=f1p)
        f1 = dict(f1p, steps=args.f1_steps, ms_per_step=round(1e3 * e1 / args.f1_steps, 3),
                  value=n * args.f1_steps / e1,
                  kernel_ms={k: round(v / n1, 4) for k, v in ms1.items()})
        print(f"[bench] with filter and collisions: {f1}", file=sys.stderr, flush=True)
    batch = batch_bench(args.batch_steps, args.tuning) if args.batch_steps > 0 else None
    if batch:
        print(f"[bench] batch: {batch}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.nz, args.cpu_steps)
    line = {
        "metric": "particle-updates/sec @19.6M particles, FP32-mixed vs FP64 at stated error",
        "value": value, "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"rotating cylinder, {n} particles ({nf} fluid), dx=1/{args.nz}, "
                               "Wendland C2, FP32-mixed, dt=1e-4",
                   "particles": n, "precision": "fp32_mixed",
                   "tuning": tuning[0] or "default", "cell_factor": tuning[1]},
        "kernel_ms": {k: round(v, 4) for k, v in per.items()},
        "roofline": roof,
        "fp64_gpu": fp64,
        "batch64": batch,
        "vortex_diag": vortex,
        "filter_collide": f1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
