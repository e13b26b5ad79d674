"""Parity at the full sizes of the measured workloads, in the launch configuration the
benchmark times (the tuned settings of paper_2405_03980_amd/tuned.json).

2.45M-particle cylinder: every fluid particle against the oracle after one and two steps,
and a stored sample of the oracle's state after 100 steps.  19.57M-particle cylinder:
sampled particles against the oracle evaluated one by one, one full step of every
particle, and 100 steps of the FP32-mixed path against the FP64 path.  64-instance batch:
every instance against its own single-instance run.
"""
import copy
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_03980_amd import _lib as L
from paper_2405_03980_amd import inputs as I
from tests._parity import field_errors, positions_ok

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = ("block_density", "block_force", "block_stream", "use_graph", "sweep", "xcd_run",
        "list_targets")


def _tuned(name):
    with open(os.path.join(ROOT, "paper_2405_03980_amd", "tuned.json")) as f:
        t = json.load(f).get(name, {})
    return {k: v for k, v in t.items() if k in KEYS}, int(t.get("cell_factor", 1))


def _sim(w, prec, name):
    from paper_2405_03980_amd import sim as S
    tun, cf = _tuned(name)
    s = S.Simulation(dict(w.params, cell_factor=cf), w.n, precision=prec)
    if tun:
        s.set_tuning(**tun)  # before init, so that the first evaluation uses it too
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    return s


@pytest.fixture(scope="module")
def cyl245():
    w = I.config(1)
    print(f"[full] cylinder 2.45M: n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    init = {k: getattr(ref, k).copy() for k in ("rho", "P", "acc", "alpha")}
    ref.step(1e-4, w.Omega, 1)
    one = {k: getattr(ref, k).copy() for k in ("x", "v", "omega", "rho", "P", "acc", "alpha")}
    ref.step(1e-4, w.Omega, 1)
    return w, init, one, ref


class _Snap:
    def __init__(self, d):
        self.__dict__.update(d)


def test_cylinder_2p45M_fp64_two_steps(cyl245):
    w, init, one, ref2 = cyl245
    s = _sim(w, L.FP64, "cylinder_nz92")
    out0 = s.read(("rho", "P", "acc", "alpha"))
    for k in ("rho", "acc", "alpha"):
        f = w.kind == I.FLUID
        e = np.abs(out0[k][..., f] - init[k][..., f]).max() / np.abs(init[k][..., f]).max()
        assert e < 1e-12, (k, e)
    s.step(1e-4, w.Omega, 2)
    e = field_errors(s.read(), ref2, w)
    print("2.45M fp64 2 steps", e, flush=True)
    assert positions_ok(e, 1e-12, 2), e
    for k in ("v", "omega", "rho", "P", "acc", "alpha"):
        assert e[k] < 1e-12, (k, e[k])
    s.close()


def test_cylinder_2p45M_mixed_one_step(cyl245):
    w, init, one, _ = cyl245
    s = _sim(w, L.FP32_MIXED, "cylinder_nz92")
    s.step(1e-4, w.Omega, 1)
    e = field_errors(s.read(), _Snap(one), w)
    print("2.45M mixed 1 step", e, flush=True)
    assert positions_ok(e, 1e-5, 1), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])
    s.close()


@pytest.fixture(scope="module")
def cyl1957():
    w = I.config(3)
    print(f"[full] cylinder 19.57M: n={w.n}", flush=True)
    return w


def test_cylinder_19p57M_vortex_image(cyl1957):
    """The vortex diagnostic of the z = 0 section at full size, in the benchmarked launch
    configuration, with random spins on the fluid: the oracle evaluates the density of the
    particles within dx + 2h of the section, then the section's intensities (any density
    read outside that slab is NaN and would show), the image and its components."""
    from oracle import vortex as V
    w = cyl1957
    omega = w.omega + np.random.default_rng(12).normal(size=w.omega.shape) * (w.kind == I.FLUID)
    theta, min_pixels = 0.5, 3
    wv = copy.copy(w)
    wv.omega = omega
    s = _sim(wv, L.FP32_MIXED, "cylinder_nz184")
    cnt, img, lab = s.vortex_image(0.0, theta, min_pixels)
    s.close()
    p = w.params
    dz = w.x[2] - 1.0 * np.floor(w.x[2] + 0.5)
    near = np.flatnonzero(np.abs(dz) < p["dx"] + 2.0 * p["h"] + 1e-12)
    rho_near = O.eval_subset(p, w.x, w.v, omega, w.species, w.kind, near)[0]
    rho = np.full(w.n, np.nan)
    rho[near] = rho_near
    sel = V.section_mask(p, w.x, w.kind, 0.0)
    inten = O.rot_intensity(p, w.x, omega, w.species, w.kind, rho, mask=sel)
    oimg = V.plane_image(p, w.x, w.kind, inten, 0.0)
    vmax = oimg.max()
    err = np.abs(img - oimg).max() / vmax
    print(f"19.57M vortex image: {img.shape}, section {sel.sum()} particles, err {err:.2e}, "
          f"components {cnt}", flush=True)
    assert np.isfinite(oimg).all() and err < 1e-5
    on = lab >= 0
    clear = np.abs(oimg - theta * vmax) > 2e-5 * vmax
    assert np.array_equal(on[clear], V.threshold(oimg, theta)[clear])
    assert np.array_equal(lab, V.components(on))
    assert cnt == V.count(lab, min_pixels) and cnt > 0


def test_cylinder_19p57M_sampled_initial_fields(cyl1957):
    """The benchmarked configuration: sampled particles against the oracle's one-by-one
    evaluation (density of the sample and its neighbours, then their forces)."""
    w = cyl1957
    rng = np.random.default_rng(11)
    fluid = np.nonzero(w.kind == I.FLUID)[0]
    near_wall = fluid[np.hypot(w.x[0, fluid], w.x[1, fluid]) > 1.0 - 6 * w.params["dx"]]
    idx = np.unique(np.concatenate([rng.choice(fluid, 2000, replace=False),
                                    rng.choice(near_wall, 1000, replace=False)]))
    rho, P, S_, acc, alpha = O.eval_subset(w.params, w.x, w.v, w.omega, w.species, w.kind, idx)
    B = w.params["rho0"] * w.params["c0"] ** 2 / 7.0
    for prec, tol in ((L.FP32_MIXED, 1e-5), (L.FP64, 1e-12)):
        s = _sim(w, prec, "cylinder_nz184")
        out = s.read(("rho", "P", "acc", "alpha"))
        s.close()
        del s
        e_rho = np.abs(out["rho"][idx] - rho).max() / np.abs(rho).max()
        e_P = np.abs(out["P"][idx] - P).max() / B
        na = np.sqrt((acc ** 2).sum(0)).max()
        e_acc = np.sqrt(((out["acc"][:, idx] - acc) ** 2).sum(0)).max() / na
        nl = np.sqrt((alpha ** 2).sum(0)).max()
        e_al = np.sqrt(((out["alpha"][:, idx] - alpha) ** 2).sum(0)).max() / nl
        print(f"19.57M sampled prec={prec}: rho {e_rho:.2e} P {e_P:.2e} acc {e_acc:.2e} alpha {e_al:.2e}",
              flush=True)
        assert max(e_rho, e_P, e_acc, e_al) < tol


def test_cylinder_19p57M_mixed_one_step(cyl1957):
    w = cyl1957
    s = _sim(w, L.FP32_MIXED, "cylinder_nz184")
    s.step(1e-4, w.Omega, 1)
    out = s.read(("x", "v", "omega", "rho", "P"))
    s.close()
    del s
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 1)
    e = field_errors(out, ref, w)
    print("19.57M mixed 1 step", e, flush=True)
    assert positions_ok(e, 1e-5, 1), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])


F1 = dict(pressure_filter=1, coll_alpha=0.8, coll_e=0.3)


def test_cylinder_19p57M_filtered_initial_fields(cyl1957):
    """The benchmarked workload with the pressure filter and the collision step on (the
    configuration of the benchmark's filter-and-collision leg): sampled particles against
    the oracle's one-by-one evaluation (densities of two rings around the sample, filtered
    pressures of one, then the sample's forces)."""
    w = copy.copy(cyl1957)
    w.params = dict(w.params, **F1)
    rng = np.random.default_rng(13)
    fluid = np.nonzero(w.kind == I.FLUID)[0]
    near_wall = fluid[np.hypot(w.x[0, fluid], w.x[1, fluid]) > 1.0 - 6 * w.params["dx"]]
    idx = np.unique(np.concatenate([rng.choice(fluid, 1500, replace=False),
                                    rng.choice(near_wall, 500, replace=False)]))
    rho, P, S_, acc, alpha = O.eval_subset(w.params, w.x, w.v, w.omega, w.species, w.kind, idx)
    B = w.params["rho0"] * w.params["c0"] ** 2 / 7.0
    s = _sim(w, L.FP32_MIXED, "cylinder_nz184")
    out = s.read(("rho", "P", "acc", "alpha"))
    s.close()
    del s
    e_P = np.abs(out["P"][idx] - P).max() / B
    na = np.sqrt((acc ** 2).sum(0)).max()
    e_acc = np.sqrt(((out["acc"][:, idx] - acc) ** 2).sum(0)).max() / na
    print(f"19.57M filtered sampled: P {e_P:.2e} acc {e_acc:.2e}", flush=True)
    assert max(e_P, e_acc) < 1e-5


def test_cylinder_19p57M_jittered_step_with_collisions(cyl1957):
    """Every particle after one step of the 19.57M cylinder with its fluid jittered by up
    to 0.3 dx, so that millions of pairs come within the collision distance, against the
    oracle's step, in the benchmarked launch configuration."""
    w = copy.copy(cyl1957)
    rng = np.random.default_rng([3980, 77])
    f = w.kind == I.FLUID
    x = w.x.copy()
    x[:, f] += rng.uniform(-0.3, 0.3, size=(3, int(f.sum()))) * w.params["dx"]
    x[2] = np.mod(x[2], 1.0)
    v = w.v.copy()
    v[:, f] += rng.normal(0.0, 0.05, size=(3, int(f.sum())))
    w.x, w.v = x, v
    w.params = dict(w.params, **F1)
    s = _sim(w, L.FP32_MIXED, "cylinder_nz184")
    s.step(1e-4, w.Omega, 1)
    out = s.read(("x", "v", "omega", "rho", "P"))
    s.close()
    del s
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 1)
    e = field_errors(out, ref, w)
    print("19.57M jittered, filter + collisions, 1 step", e, flush=True)
    assert positions_ok(e, 1e-5, 1), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])


def test_batch64_equals_single_instances():
    """The 64-instance ensemble (5.9M particles) in its tuned launch configuration equals,
    bit for bit, each instance run on its own with the same settings."""
    from paper_2405_03980_amd import sim as S
    ws = I.make_batch(64)
    tun, cf = _tuned("batch64")
    for w in ws:
        w.params = dict(w.params, cell_factor=cf)
    b = S.batch_from(ws)
    if tun:
        b.set_tuning(**tun)
    Om = [w.Omega for w in ws]
    b.step(1e-4, Om, 4)
    out = b.read(("x", "v", "omega", "rho"))
    b.close()
    del b
    for i in (0, 7, 23, 63):
        w = ws[i]
        s = S.simulation_from(w)
        if tun:
            s.set_tuning(**tun)
        s.step(1e-4, w.Omega, 4)
        o = s.read(("x", "v", "omega", "rho"))
        s.close()
        lo = sum(x.n for x in ws[:i])
        for k in o:
            assert np.array_equal(out[k][..., lo:lo + w.n], o[k]), (i, k)
    # and two instances against the oracle
    for i in (3, 40):
        w = ws[i]
        ref = O.State.from_workload(w)
        ref.step(1e-4, w.Omega, 4)
        lo = sum(x.n for x in ws[:i])
        part = {k: out[k][..., lo:lo + w.n] for k in out}
        e = field_errors(part, ref, w)
        print(f"batch instance {i} n={w.n}", e, flush=True)
        assert positions_ok(e, 1e-5, 4), e
        for k in ("v", "omega", "rho"):
            assert e[k] < 1e-5, (i, k, e[k])


GOLD100 = os.path.join(ROOT, "tests", "golden", "cylinder_2p45M_100steps.npz")


def _norm(a):
    return np.sqrt((a * a).sum(axis=0)) if a.ndim == 2 else np.abs(a)


@pytest.mark.parametrize("prec,tol", [(L.FP64, 1e-12), (L.FP32_MIXED, 1e-3)])
def test_cylinder_2p45M_100_steps_vs_oracle(prec, tol):
    """100 steps of the 2.45M cylinder against the oracle's state after 100 steps: a seeded
    sample of 5,000 fluid particles (3,000 anywhere, 2,000 next to the wall) stored by
    tests/golden/make_cylinder_2p45M_100.py, normwise errors over the oracle's whole-field
    maxima.  FP64 path within 1e-12 on every field, FP32-mixed within 1e-3."""
    g = np.load(GOLD100, allow_pickle=False)
    w = I.config(1)
    steps = int(g["steps"])
    print(f"[full] cylinder 2.45M, {steps} steps, prec={prec}", flush=True)
    s = _sim(w, prec, "cylinder_nz92")
    s.step(float(g["dt"]), w.Omega, steps)
    out = s.read(("x", "v", "omega", "rho", "P", "acc", "alpha"))
    s.close()
    del s
    ids = g["ids"]
    p = w.params
    B = p["rho0"] * p["c0"] ** 2 / 7.0
    H = p["hi"][2] - p["lo"][2]
    dx = out["x"][:, ids] - g["x"]
    dx[2] -= H * np.round(dx[2] / H)
    e = {"x": float(_norm(dx).max() / g["disp_max"]),
         "x_ulp": float((np.abs(dx) / np.spacing(np.abs(g["x"]))).max()),
         "rho": float(np.abs(out["rho"][ids] - g["rho"]).max() / g["rho_max"]),
         "P": float(np.abs(out["P"][ids] - g["P"]).max() / B)}
    for k in ("v", "omega", "acc", "alpha"):
        e[k] = float(_norm(out[k][:, ids] - g[k]).max() / g[k + "_max"])
    print(f"2.45M {steps} steps prec={prec}", e, flush=True)
    assert positions_ok(e, tol, steps), e
    fields = ("v", "omega", "rho", "P", "acc", "alpha") if prec == L.FP64 else ("v", "omega", "rho", "P")
    for k in fields:
        assert e[k] < tol, (k, e[k])


def test_cylinder_19p57M_mixed_vs_fp64_100_steps(cyl1957):
    """The benchmarked workload over 100 steps: the FP32-mixed path against the FP64 GPU path
    (which the tests above tie to the oracle), within 1e-3 on positions, velocities, spins,
    density and pressure."""
    w = cyl1957
    outs = {}
    for prec in (L.FP64, L.FP32_MIXED):
        print(f"[full] cylinder 19.57M, 100 steps, prec={prec}", flush=True)
        s = _sim(w, prec, "cylinder_nz184")
        s.step(1e-4, w.Omega, 100)
        outs[prec] = s.read(("x", "v", "omega", "rho", "P", "acc", "alpha"))
        s.close()
        del s
    e = field_errors(outs[L.FP32_MIXED], _Snap(outs[L.FP64]), w)
    print("19.57M mixed vs fp64, 100 steps", e, flush=True)
    assert positions_ok(e, 1e-3, 100), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-3, (k, e[k])
