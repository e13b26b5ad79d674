"""Writes cylinder_2p45M_100steps.npz: the FP64 oracle's state of the 2.45M-particle
cylinder (dx = 1/92, Wendland C2) after 100 steps of dt = 1e-4, for a seeded sample of
fluid particles, plus the whole-field normalisers of the normwise errors.

Calls only the oracle and the seeded input generator (no HIP code):

    python tests/golden/make_cylinder_2p45M_100.py        # a few minutes on 8 cores
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2405_03980_amd import inputs as I  # noqa: E402

STEPS, DT = 100, 1e-4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cylinder_2p45M_100steps.npz")


def sample_ids(w, n_random=3000, n_wall=2000, seed=2405):
    """Fluid particles: n_random anywhere, n_wall within six dx of the wall layer."""
    rng = np.random.default_rng(seed)
    fluid = np.nonzero(w.kind == I.FLUID)[0]
    r = np.hypot(w.x[0, fluid], w.x[1, fluid])
    near = fluid[r > 1.0 - 9 * w.params["dx"]]
    ids = np.concatenate([rng.choice(fluid, n_random, replace=False),
                          rng.choice(near, n_wall, replace=False)])
    return np.unique(ids)


def main():
    w = I.config(1)
    ids = sample_ids(w)
    ref = O.State.from_workload(w)
    t0 = time.time()
    ref.step(DT, w.Omega, STEPS)
    print(f"oracle: {w.n} particles x {STEPS} steps in {time.time() - t0:.0f} s", flush=True)
    f = w.kind == I.FLUID
    disp = ref.x - w.x
    H = w.params["hi"][2] - w.params["lo"][2]
    disp[2] -= H * np.round(disp[2] / H)  # z is periodic: minimum image
    norm = lambda a: np.sqrt((a * a).sum(axis=0))
    np.savez_compressed(
        OUT, ids=ids.astype(np.int64), steps=np.int64(STEPS), dt=np.float64(DT),
        x=ref.x[:, ids], v=ref.v[:, ids], omega=ref.omega[:, ids], rho=ref.rho[ids],
        P=ref.P[ids], acc=ref.acc[:, ids], alpha=ref.alpha[:, ids],
        disp_max=norm(disp[:, f]).max(), v_max=norm(ref.v[:, f]).max(),
        omega_max=norm(ref.omega[:, f]).max(), acc_max=norm(ref.acc[:, f]).max(),
        alpha_max=norm(ref.alpha[:, f]).max(), rho_max=np.abs(ref.rho[f]).max())
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
