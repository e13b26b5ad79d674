#!/usr/bin/env python
"""Throughput of the two-fluid SPH step on one MI355X.

Headline workload: the 19.57M-particle rotating cylinder (R = H = 1, dx = 1/184, Wendland
C2, h = 1.3 dx, 70/30 inviscid/viscous fluid, three wall layers turning at Omega = 1, fluid
at rest plus N(0, 1e-3) noise), FP32-mixed path, dt = 1e-4.  A step is one velocity-Verlet
step of every particle: kick/drift, cell list, density/EOS, forces/torques.

Prints ONE JSON line: particle-updates/s (walls included, as the paper counts particles;
median of three timed runs of --steps steps), the roofline of the dominant kernel (the
force sweep) from HIP events recorded on the library's stream during a further profiled
run, the whole step's HBM fraction, every configuration of the measurement plan timed on
the GPU (FP64 and FP32-mixed, median of three runs), and the FP64 CPU oracle timed on the
host (one step of the headline workload; configurations 0 and 1 beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X published FP32 vector peak (packed FP32) and the rate without packed FP32
# instructions, which this build does not emit: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Compulsory HBM bytes per particle-update of the FP32-mixed step (the algorithmic count of
# the measurement plan): the force sweep reads x, v, w (72), rho, P, S (12), species (1),
# its cell index (4) and writes a, alpha (24); the whole step moves about 350 B.
FORCE_BYTES_PER_PU = 113
STEP_BYTES_PER_PU = 350
# Algorithmic flops of the force sweep per particle-update: about 84 per unique pair
# (distance 9, pair terms 75 averaged over the species mix) over 40 unique pairs.
FORCE_FLOPS_PER_PU = 84 * 40
# Our own per-kernel counts of compulsory bytes per particle (mixed precision), for the
# per-kernel table.
KERNEL_BYTES_PER_PARTICLE = {
    "keys": 24 + 24 + 12 + 1 + 4 + 4,          # x, v, acc, sk -> key, slot
    "scatter": 4 + 4 + 4 + 4 + 4 + 4,           # key, slot, start, id -> tmp, idt
    "reorder": 4 + 4 + 4 + 72 + 24 + 1 + 72 + 4 + 1 + 4,  # tmp, key, id, state -> state, pcell
    "density": 24 + 1 + 4 + 4 + 16 + 8,         # x, sk, pcell, cell_xyz -> aux, rho/P
    "force": FORCE_BYTES_PER_PU,
}
GOLD100 = os.path.join(ROOT, "tests", "golden", "cylinder_2p45M_100steps.npz")
TUNING_KEYS = ("block_density", "block_force", "block_stream", "use_graph", "sweep", "xcd_run",
        "list_targets")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--runs", type=int, default=3, help="timed runs per figure (median)")
    ap.add_argument("--nz", type=int, default=184, help="cylinder resolution (184: 19.57M)")
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the smaller configurations (0-2) of the measurement plan")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2405_03980_amd", "tuned.json"))
    ap.add_argument("--f1-steps", type=int, default=20,
                    help="timed steps with the pressure filter and the collision step on (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="steps of the batched 64-instance ensemble (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device-to-device copy of this size (5 times), to "
                         "calibrate the HBM traffic counters, and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    """Tuned settings of a workload: (launch tuning for sph_tuning, cell factor)."""
    try:
        with open(path) as f:
            t = json.load(f).get(name, {})
    except (OSError, ValueError):
        t = {}
    return {k: v for k, v in t.items() if k in TUNING_KEYS}, int(t.get("cell_factor", 1))


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


def _sync_all(obj):
    import torch
    obj.sync()
    torch.cuda.synchronize()


def time_runs(obj, Om, steps: int, runs: int) -> list[float]:
    """Seconds of `runs` timed runs of `steps` steps each, every run bracketed by a stream
    and device synchronisation."""
    out = []
    for _ in range(runs):
        _sync_all(obj)
        t0 = time.perf_counter()
        obj.step(1e-4, Om, steps)
        _sync_all(obj)
        out.append(time.perf_counter() - t0)
    return out


def profile_run(obj, Om, steps: int) -> dict:
    """Per-kernel milliseconds per step from HIP events on the library's stream."""
    _sync_all(obj)
    obj.profile_begin()
    obj.step(1e-4, Om, steps)
    ms, n = obj.profile_end()
    _sync_all(obj)
    return {k: v / n for k, v in ms.items() if v}


def simulation(w, precision, tuning, extra=None):
    from paper_2405_03980_amd import sim as S
    tun, cf = tuning
    s = S.Simulation(dict(w.params, cell_factor=cf, **(extra or {})), w.n, precision=precision)
    if tun:
        s.set_tuning(**tun)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    return s


def timed_config(w, precision, steps, warmup, runs, tuning, profile=False, fields=None):
    """ms/step (median of `runs`), PU/s, optional per-kernel ms and fields read after the
    first run (warmup + steps steps from the initial state)."""
    import torch
    s = simulation(w, precision, tuning)
    s.step(1e-4, w.Omega, warmup)
    t = time_runs(s, w.Omega, steps, 1)
    got = s.read(fields) if fields else None
    t += time_runs(s, w.Omega, steps, runs - 1)
    med = statistics.median(t)
    out = {"ms_per_step": round(1e3 * med / steps, 4), "value": w.n * steps / med,
           "runs_ms_per_step": [round(1e3 * x / steps, 4) for x in t], "steps": steps,
           "warmup": warmup}
    if profile:
        out["kernel_ms"] = {k: round(v, 4) for k, v in profile_run(s, w.Omega, steps).items()}
    s.close()
    del s
    torch.cuda.empty_cache()
    return out, got


def field_errors(a: dict, b: dict, fluid, B) -> dict:
    """Normwise relative difference of a against b over fluid particles (P over B)."""
    out = {}
    for k in ("rho", "P", "v", "omega", "acc"):
        x, y = a[k][..., fluid], b[k][..., fluid]
        if k == "P":
            out[k] = float(np.abs(x - y).max() / B)
            continue
        if x.ndim == 2:
            d, r = np.sqrt(((x - y) ** 2).sum(0)), np.sqrt((y * y).sum(0))
        else:
            d, r = np.abs(x - y), np.abs(y)
        out[k] = float(d.max() / max(r.max(), 1e-300))
    return out


def golden_errors(out: dict, w) -> dict:
    """Errors against the stored FP64 oracle sample of the 2.45M cylinder after 100 steps
    (5,000 fluid particles, normwise over the oracle's whole-field maxima)."""
    g = np.load(GOLD100, allow_pickle=False)
    ids = g["ids"]
    p = w.params
    B = p["rho0"] * p["c0"] ** 2 / 7.0
    nrm = lambda a: np.sqrt((a * a).sum(axis=0))
    e = {"rho": float(np.abs(out["rho"][ids] - g["rho"]).max() / g["rho_max"]),
         "P": float(np.abs(out["P"][ids] - g["P"]).max() / B)}
    for k in ("v", "omega", "acc"):
        e[k] = float(nrm(out[k][:, ids] - g[k]).max() / g[k + "_max"])
    return e


def batch_bench(steps: int, runs: int, tuning_path: str) -> dict:
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
    t = time_runs(b, Om, steps, runs)
    kms = profile_run(b, Om, max(10, steps // 5))
    b.close()
    del b
    seq_steps = max(2, steps // 10)
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
    med = statistics.median(t)
    ms = 1e3 * med / steps
    ms_seq = 1e3 * el_seq / seq_steps
    return {"value": N * steps / med, "unit": "particle-updates/s", "n_inst": len(ws),
            "tuning": tun or "default", "cell_factor": cf, "particles": N, "steps": steps,
            "ms_per_step": round(ms, 4), "runs_ms_per_step": [round(1e3 * x / steps, 4) for x in t],
            "kernel_ms": {k: round(v, 4) for k, v in kms.items()},
            "sequential_ms_per_step": round(ms_seq, 3),
            "speedup_vs_sequential": round(ms_seq / ms, 2)}


def oracle_rate(w, steps: int) -> dict:
    """The FP64 oracle as it stands on the host's threads: particle-updates per second of
    `steps` steps (its evaluation at load excluded)."""
    from oracle import oracle as O
    s = O.State.from_workload(w)
    t0 = time.perf_counter()
    s.step(1e-4, w.Omega, steps)
    dt = time.perf_counter() - t0
    return {"value": w.n * steps / dt, "unit": "particle-updates/s", "cores": O.num_threads(),
            "kind": "oracle", "steps": steps, "seconds": round(dt, 2), "particles": w.n}


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

    w = I.make_cylinder(args.nz, seed=(3980, 3))
    name = f"cylinder_nz{args.nz}"
    n, nf = w.n, w.n_fluid
    B3 = w.params["rho0"] * w.params["c0"] ** 2 / 7.0
    log(f"{name}: {n} particles ({nf} fluid)")
    tuning = load_tuning(args.tuning, name)

    # Headline: FP32-mixed, median of `runs` timed runs, then one profiled run.
    s = simulation(w, L.FP32_MIXED, tuning)
    s.step(1e-4, w.Omega, args.warmup)
    t = time_runs(s, w.Omega, args.steps, args.runs)
    elapsed = statistics.median(t)
    per = {k: v for k, v in profile_run(s, w.Omega, args.steps).items()
           if k not in ("collide", "filter")}
    # the vortex diagnostic of the z = 0 section on the state just stepped
    s.vortex_image(0.0, 0.5, 3, to_numpy=False)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cnt, img, _ = s.vortex_image(0.0, 0.5, 3, to_numpy=False)
    torch.cuda.synchronize()
    vortex = {"ms": round(1e3 * (time.perf_counter() - t1), 3), "z0": 0.0, "theta": 0.5,
              "min_pixels": 3, "count": cnt, "image": [int(img.shape[0]), int(img.shape[1])]}
    s.close()
    del s
    torch.cuda.empty_cache()
    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    log(f"mixed: {ms_step:.3f} ms/step (runs {[round(1e3 * x / args.steps, 3) for x in t]}); "
        "per kernel (ms): " + ", ".join(f"{k}={v:.3f}" for k, v in per.items()))

    # Roofline of the dominant kernel (the force sweep) and of the whole step: algorithmic
    # bytes per particle-update over the measured time, against the HBM peak.
    dom = max(per, key=per.get)
    t_dom = per[dom] * 1e-3
    hbm = n * KERNEL_BYTES_PER_PARTICLE.get(dom, 0) / t_dom / 1e9
    traffic = measured_traffic(dom)
    roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 3),
            "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": dom, "avg_ms": round(per[dom], 4), "units": n,
            "alg_bytes_per_unit": KERNEL_BYTES_PER_PARTICLE.get(dom)}
    step_gbs = n * STEP_BYTES_PER_PU / (ms_step * 1e-3) / 1e9
    roof["step"] = {"alg_bytes_per_unit": STEP_BYTES_PER_PU, "achieved": round(step_gbs, 1),
                    "frac": round(step_gbs / HBM_PEAK_GBS, 4), "ms_per_step": round(ms_step, 4)}
    if dom == "force":
        tf = nf * FORCE_FLOPS_PER_PU / t_dom / 1e12
        roof["alu"] = {"achieved": round(tf, 3), "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS,
                       "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                       "nonpacked_ceiling": round(FP32_NONPACKED_TFLOPS, 1),
                       "frac_of_nonpacked": round(tf / FP32_NONPACKED_TFLOPS, 4),
                       "alg_flops_per_unit": FORCE_FLOPS_PER_PU, "units": nf,
                       "binding": "VALU instruction issue (rocprofv3 SQ counters)"}

    configs = {}
    # Configuration 3 on the FP64 path, and both paths after the same 25 steps.
    e25 = None
    if args.fp64_steps > 0:
        # both paths compared after the same trajectory: warmup + the first timed run
        fx = ("rho", "P", "v", "omega", "acc")
        _, fm = timed_config(w, L.FP32_MIXED, args.fp64_steps, args.warmup, 1, tuning, fields=fx)
        r64, f64 = timed_config(w, L.FP64, args.fp64_steps, args.warmup, args.runs, tuning,
                                fields=fx)
        e25 = field_errors(fm, f64, w.kind == I.FLUID, B3)
        configs["3_fp64"] = dict(r64, workload=name, precision="fp64")
        log(f"fp64: {r64['ms_per_step']} ms/step; mixed vs fp64 after "
            f"{args.warmup + args.fp64_steps} steps {e25}")
    configs["3_mixed"] = {"ms_per_step": round(ms_step, 4), "value": value, "steps": args.steps,
                          "runs_ms_per_step": [round(1e3 * x / args.steps, 4) for x in t],
                          "workload": name, "precision": "fp32_mixed"}

    if not args.no_configs:
        w0 = I.config(0)
        r, _ = timed_config(w0, L.FP64, 20, 5, args.runs, ({}, 1))
        configs["0_fp64"] = dict(r, workload="box4096_cubic", precision="fp64")
        r, _ = timed_config(w0, L.FP32_MIXED, 20, 5, args.runs, ({}, 1))
        configs["0_mixed"] = dict(r, workload="box4096_cubic", precision="fp32_mixed")
        w1 = I.config(1)
        t92 = load_tuning(args.tuning, "cylinder_nz92")
        r, _ = timed_config(w1, L.FP64, 100, 0, args.runs, t92)
        configs["1_fp64"] = dict(r, workload="cylinder_2.45M", precision="fp64")
        fx = ("rho", "P", "v", "omega", "acc")
        r, f2 = timed_config(w1, L.FP32_MIXED, 100, 0, args.runs, t92, profile=True, fields=fx)
        configs["2_mixed"] = dict(r, workload="cylinder_2.45M", precision="fp32_mixed",
                                  error_vs_oracle_100_steps=golden_errors(f2, w1))
        for k, v in configs.items():
            log(f"config {k}: {v['ms_per_step']} ms/step, {v['value']:.4g} PU/s")

    f1 = None
    if args.f1_steps > 0:
        # the same workload with Algorithm 1's pressure filter and collision step switched
        # on (the lattice keeps every pair beyond the collision distance, so the collision
        # step costs its search only)
        f1p = dict(pressure_filter=1, coll_alpha=0.8, coll_e=0.3)
        sf = simulation(w, L.FP32_MIXED, tuning, extra=f1p)
        sf.step(1e-4, w.Omega, args.warmup)
        tf1 = time_runs(sf, w.Omega, args.f1_steps, 1)[0]
        kms = profile_run(sf, w.Omega, args.f1_steps)
        sf.close()
        del sf
        torch.cuda.empty_cache()
        f1 = dict(f1p, steps=args.f1_steps, ms_per_step=round(1e3 * tf1 / args.f1_steps, 3),
                  value=n * args.f1_steps / tf1, kernel_ms={k: round(v, 4) for k, v in kms.items()})
        log(f"with filter and collisions: {f1}")
    batch = None
    if args.batch_steps > 0:
        batch = batch_bench(args.batch_steps, args.runs, args.tuning)
        configs["4_mixed_batch64"] = {k: batch[k] for k in ("ms_per_step", "value", "steps",
                                                            "runs_ms_per_step")}
        log(f"batch: {batch}")

    cpu = None
    oracle_configs = None
    if not args.no_cpu_baseline:
        # the oracle on the headline workload itself: one step of all 19.57M particles
        cpu = oracle_rate(w, 1)
        cpu["sample"] = (f"1 step of the whole {name} workload ({n} particles), FP64, "
                         f"{cpu['seconds']} s")
        log(f"oracle: {cpu}")
        if not args.no_configs:
            oracle_configs = {"0": oracle_rate(I.config(0), 20), "1": oracle_rate(I.config(1), 5)}
            log(f"oracle configs: {oracle_configs}")

    line = {
        "metric": "particle-updates/sec @19.6M particles, FP32-mixed vs FP64 at stated error",
        "value": value, "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"rotating cylinder, {n} particles ({nf} fluid), dx=1/{args.nz}, "
                               "Wendland C2, FP32-mixed, dt=1e-4",
                   "particles": n, "precision": "fp32_mixed", "timing": f"median of {args.runs} runs",
                   "tuning": tuning[0] or "default", "cell_factor": tuning[1]},
        "kernel_ms": {k: round(v, 4) for k, v in per.items()},
        "roofline": roof,
        "fp64_gpu": None if e25 is None else {
            "ms_per_step": configs["3_fp64"]["ms_per_step"],
            "speedup_mixed_vs_fp64": round(configs["3_fp64"]["ms_per_step"] / ms_step, 3),
            "mixed_error_vs_fp64": e25, "after_steps": args.warmup + args.fp64_steps},
        "configs": configs,
        "batch64": batch,
        "vortex_diag": vortex,
        "filter_collide": f1,
        "cpu_baseline": cpu,
        "cpu_oracle_configs": oracle_configs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
