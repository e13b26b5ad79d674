"""Autotuner of the launch shape: sweep implementation, cells per interaction radius,
brick-sweep tiling (bricks per XCD run, targets per density round), block sizes and graph
replay, picked by timing a few steps of the real workload.

Results are cached as JSON ({workload name: settings}) and read by bench.py.  The
settings change performance only: every candidate computes the same method (the cell
factor changes the summation order, hence rounding, not the neighbour sets).

    python -m paper_2405_03980_amd.tune --workload cylinder --nz 184 --out tuned.json
    python -m paper_2405_03980_amd.tune --workload batch --out tuned.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

from . import _lib as L
from . import inputs as I


def candidates(batch: bool):
    """Settings to try: the brick sweeps (cell factor 1) over the bricks given to each XCD in
    a run, the targets per density round, streaming block sizes and graph replay; and the
    per-particle sweeps for cell factors 1 and 2 over block sizes."""
    out = []
    for run, lt, bs in itertools.product((4, 8, 16, 32, 64), (16, 32), (256, 512)):
        for graph in ((1,) if batch else (0, 1)):
            out.append(dict(cell_factor=1, sweep=3, xcd_run=run, list_targets=lt, block_stream=bs,
                            use_graph=graph))
    for cf, bd, bf in itertools.product((1, 2), (128, 256), (128, 256)):
        out.append(dict(cell_factor=cf, sweep=1, block_density=bd, block_force=bf,
                        block_stream=256, use_graph=1))
    return out


def _time_single(w, cand, steps):
    from . import sim as S
    params = dict(w.params, cell_factor=cand["cell_factor"])
    s = S.Simulation(params, w.n, precision=L.FP32_MIXED)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    s.set_tuning(**{k: v for k, v in cand.items() if k != "cell_factor"})
    dt = _timed(s, w.Omega, steps)
    s.close()
    return dt


def _timed(obj, Om, steps):
    """Seconds per step: warm-up calls that also capture the step graphs of both buffer
    parities, then the better of two timed calls of `steps` steps."""
    import torch
    for _ in range(2):
        obj.step(1e-4, Om, 3)
    best = float("inf")
    for _ in range(2):
        obj.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj.step(1e-4, Om, steps)
        obj.sync()
        best = min(best, (time.perf_counter() - t0) / steps)
    return best


def _time_batch(ws, cand, steps):
    from . import sim as S
    import numpy as np
    params = [dict(w.params, cell_factor=cand["cell_factor"]) for w in ws]
    b = S.Batch(params, [w.n for w in ws], precision=L.FP32_MIXED)
    b.init(np.concatenate([w.x for w in ws], axis=1), np.concatenate([w.v for w in ws], axis=1),
           np.concatenate([w.omega for w in ws], axis=1), np.concatenate([w.species for w in ws]),
           np.concatenate([w.kind for w in ws]))
    b.set_tuning(**{k: v for k, v in cand.items() if k != "cell_factor"})
    dt = _timed(b, [w.Omega for w in ws], steps)
    b.close()
    return dt


def tune(kind: str, nz: int = 184, steps: int = 6, log=sys.stderr) -> tuple[str, dict, list]:
    if kind == "batch":
        ws = I.make_batch(64)
        name = "batch64"
        timer = lambda c: _time_batch(ws, c, steps)
    else:
        w = I.make_cylinder(nz, seed=(3980, 3))
        name = f"cylinder_nz{nz}"
        timer = lambda c: _time_single(w, c, steps)
    results = []
    for c in candidates(kind == "batch"):
        try:
            t = timer(c)
        except L.SphError as e:
            print(f"[tune] {name} {c}: {e}", file=log, flush=True)
            continue
        results.append((t, c))
        print(f"[tune] {name} {c}: {1e3 * t:.3f} ms/step", file=log, flush=True)
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    best["ms_per_step"] = round(1e3 * results[0][0], 4)
    return name, best, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("cylinder", "batch"), default="cylinder")
    ap.add_argument("--nz", type=int, default=184)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "tuned.json"))
    a = ap.parse_args()
    name, best, _ = tune(a.workload, a.nz, a.steps)
    cache = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            cache = json.load(f)
    cache[name] = best
    with open(a.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print(json.dumps({name: best}))


if __name__ == "__main__":
    main()
