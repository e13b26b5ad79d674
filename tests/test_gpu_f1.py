"""Parity of the pressure filter and the collision step (Algorithm 1) on the HIP path,
through the C ABI, against the FP64 oracle.

Workloads: jittered periodic boxes with random velocities, where hundreds of pairs come
closer than the collision distance and the pressure varies strongly from particle to
particle, and a rotating cylinder with jittered fluid, where the filter meets the walls
and fluid particles collide with wall particles.  Tolerances as for the rest of the
step: FP64 1e-12 per field, FP32-mixed 1e-5 after one step.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_03980_amd import _lib as L
from paper_2405_03980_amd import inputs as I
from tests._parity import field_errors, positions_ok

pytestmark = pytest.mark.gpu

FP64, MIXED = L.FP64, L.FP32_MIXED
F1 = dict(pressure_filter=1, coll_alpha=0.8, coll_e=0.3)


def _sim(w, prec, **tune):
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(w.params, w.n, precision=prec)
    if tune:
        s.set_tuning(**tune)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    return s


def _crowd(n=12, seed=3, amp=0.3, vs=0.3, kernel=I.KERNEL_WENDLAND_C2, f1=F1):
    """Periodic box, lattice jittered by up to amp dx per axis, N(0, vs) velocities."""
    w = I.make_box(n, kernel=kernel, rigid=False, seed=(3980, 40 + seed))
    rng = np.random.default_rng([3980, 300 + seed])
    dx = w.params["dx"]
    w.x = np.mod(w.x + rng.uniform(-amp, amp, size=w.x.shape) * dx, 1.0)
    w.v = rng.normal(0.0, vs, size=w.x.shape)
    w.omega = rng.normal(0.0, 1.0, size=w.x.shape)
    c0 = 10.0 * float(np.sqrt((w.v * w.v).sum(axis=0)).max())
    w.params = dict(w.params, c0=c0, sigma_T=0.05 * c0 * c0 / 7.0, **f1)
    return w


def _cylinder(nz=16, amp=0.3, seed=5):
    """Rotating cylinder with its fluid jittered by up to amp dx per axis (walls exact)."""
    w = I.make_cylinder(nz, seed=(3980, 60 + seed))
    rng = np.random.default_rng([3980, 400 + seed])
    f = w.kind == I.FLUID
    w.x[:, f] += rng.uniform(-amp, amp, size=(3, int(f.sum()))) * w.params["dx"]
    w.x[2] = np.mod(w.x[2], 1.0)
    w.v[:, f] += rng.normal(0.0, 0.1, size=(3, int(f.sum())))
    w.params = dict(w.params, **F1)
    return w


CASES = {"crowd": _crowd, "crowd_cubic": lambda: _crowd(13, seed=4, kernel=I.KERNEL_CUBIC),
         "cylinder": _cylinder}


def _assert_fields(e, tol, steps, keys=("v", "omega", "rho", "P", "acc", "alpha")):
    assert positions_ok(e, tol, steps), e
    for k in keys:
        assert e[k] < tol, (k, e[k])


@pytest.mark.parametrize("prec,sweep,tol", [(FP64, None, 1e-12), (MIXED, 1, 1e-5), (MIXED, 3, 1e-5)])
@pytest.mark.parametrize("case", list(CASES))
def test_filtered_initial_fields(case, prec, sweep, tol):
    """The evaluation at load already uses the filtered pressure (no collision step)."""
    w = CASES[case]()
    print(f"[f1 init] {case} prec={prec} sweep={sweep} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, prec, **({"sweep": sweep} if sweep else {}))
    out = s.read()
    s.close()
    e = field_errors(out, ref, w)
    print(e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < tol, (k, e[k])
    # the filter matters here: the unfiltered pressure is far from the filtered one
    rho, P, _ = O.density(w.params, w.x, w.species, w.kind)
    B = w.params["rho0"] * w.params["c0"] ** 2 / 7.0
    assert np.abs(P - ref.P)[w.kind == I.FLUID].max() / B > 1e3 * tol


@pytest.mark.parametrize("prec,sweep,steps,tol", [(FP64, None, 5, 1e-12), (MIXED, 1, 1, 1e-5),
                                                  (MIXED, 3, 1, 1e-5)])
@pytest.mark.parametrize("case", list(CASES))
def test_steps_with_filter_and_collisions(case, prec, sweep, steps, tol):
    w = CASES[case]()
    print(f"[f1 steps] {case} prec={prec} sweep={sweep} steps={steps} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, steps)
    s = _sim(w, prec, **({"sweep": sweep} if sweep else {}))
    s.step(1e-4, w.Omega, steps)
    out = s.read()
    s.close()
    e = field_errors(out, ref, w)
    print(e, flush=True)
    _assert_fields(e, tol, steps)
    # the collision step matters here: without it the velocities are far off
    nocoll = O.State(dict(w.params, coll_alpha=0.0), w.x, w.v, w.omega, w.species, w.kind)
    nocoll.step(1e-4, w.Omega, steps)
    f = w.kind == I.FLUID
    assert np.abs(nocoll.v - ref.v)[:, f].max() > 1e3 * tol * np.abs(ref.v[:, f]).max()


def test_graph_replay_equals_single_steps():
    """Seven steps in one call (captured and replayed as a graph) equal seven calls of one
    step bit for bit: the collision step's scratch use of the spare velocity buffer is the
    same in both."""
    w = _crowd(12, seed=6)
    a = _sim(w, MIXED, sweep=3)
    a.step(1e-4, 0.0, 7)
    oa = a.read()
    a.close()
    b = _sim(w, MIXED, sweep=3, use_graph=0)
    for _ in range(7):
        b.step(1e-4, 0.0, 1)
    ob = b.read()
    b.close()
    for k in ("x", "v", "omega", "rho", "P", "acc", "alpha"):
        assert np.array_equal(oa[k], ob[k]), k


def test_batch_mixing_f1_settings():
    """An ensemble whose instances switch the filter and the collision step on and off
    independently: each equals its own single run bit for bit."""
    from paper_2405_03980_amd import sim as S
    ws = [_crowd(11, seed=7), _crowd(12, seed=8, f1=dict(pressure_filter=0, coll_alpha=0.0)),
          _crowd(10, seed=9, f1=dict(pressure_filter=1)), _cylinder(12, seed=6)]
    ws[3].params = dict(ws[3].params, pressure_filter=0)
    print("[f1 batch] sizes", [w.n for w in ws], flush=True)
    for prec in (MIXED, FP64):
        b = S.batch_from(ws, precision=prec)
        if prec == MIXED:
            b.set_tuning(sweep=3)
        b.step(1e-4, [w.Omega for w in ws], 3)
        out = b.read()
        b.close()
        for i, w in enumerate(ws):
            s = _sim(w, prec, **({"sweep": 3} if prec == MIXED else {}))
            s.step(1e-4, w.Omega, 3)
            o = s.read()
            s.close()
            lo, hi = b.offsets[i], b.offsets[i + 1]
            for k in ("x", "v", "omega", "rho", "P", "acc"):
                assert np.array_equal(out[k][..., lo:hi], o[k]), (prec, i, k)


def test_f1_parameters_are_checked():
    from paper_2405_03980_amd import sim as S
    w = _crowd(8)
    for bad in (dict(pressure_filter=2), dict(coll_alpha=-0.5), dict(coll_e=1.5),
                dict(coll_alpha=2.0 * 1.3 + 1e-9), dict(coll_e=float("nan"))):
        with pytest.raises(L.SphError):
            S.Simulation(dict(w.params, **bad), w.n, precision=MIXED)


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (MIXED, 1e-5)])
def test_free_cluster_conserves_momentum(prec, tol):
    """Open geometry, crowded free cluster: ten steps with the filter and collisions against
    the oracle, and sum m v and sum (m x × v + I omega) unchanged on the GPU (FP64 sums of
    the GPU state, to the accuracy of the path)."""
    w = I.make_cluster(9, jitter=0.35, noise=0.3)
    w.params = dict(w.params, **F1)
    steps = 10 if prec == FP64 else 1
    ref = O.State.from_workload(w)
    ref.step(1e-4, 0.0, steps)
    s = _sim(w, prec)
    P0, J0, _ = s.diagnostics()
    s.step(1e-4, 0.0, steps)
    out = s.read()
    P1, J1, _ = s.diagnostics()
    s.close()
    e = field_errors(out, ref, w)
    print("[f1 cluster]", prec, e, flush=True)
    _assert_fields(e, tol, steps)
    m = O.default_mass(w.params)[0]
    scale = m * w.n * np.abs(w.v).max()
    ctol = 1e-13 if prec == FP64 else 1e-6
    assert np.abs(P1 - P0).max() < ctol * scale
    assert np.abs(J1 - J0).max() < ctol * scale


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_lone_particle(prec):
    """One particle: its filtered pressure is its own, and nothing collides."""
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, 0.05, [0, 0, 0], [1, 1, 1], 1.0)
    p = dict(p, **F1)
    x = np.array([[0.5], [0.5], [0.5]])
    v = np.array([[0.3], [-0.1], [0.2]])
    w = I.Workload("lone", p, x, v, np.zeros((3, 1)), np.zeros(1, np.uint8), np.zeros(1, np.uint8))
    ref = O.State.from_workload(w)
    ref.step(1e-3, 0.0, 3)
    s = _sim(w, prec)
    s.step(1e-3, 0.0, 3)
    out = s.read()
    s.close()
    B = p["rho0"] * p["c0"] ** 2 / 7.0
    assert abs(out["P"][0] - ref.P[0]) <= (1e-12 if prec == FP64 else 1e-6) * B
    assert np.allclose(out["x"], ref.x, rtol=0, atol=1e-14)
    assert np.array_equal(out["v"], v)


@pytest.mark.parametrize("alpha", [1.5, 2.5])
def test_long_collision_distance(alpha):
    """Collision distances that defeat the density sweep's near lists: at 1.5 dx every
    particle has more near neighbours than a list holds, at 2.5 dx (close to 2h) none is
    listed; both take the cell walk, and match the oracle."""
    w = _crowd(12, seed=11, f1=dict(pressure_filter=1, coll_alpha=alpha, coll_e=0.5))
    ref = O.State.from_workload(w)
    ref.step(1e-4, 0.0, 1)
    s = _sim(w, MIXED, sweep=3)
    s.step(1e-4, 0.0, 1)
    out = s.read()
    s.close()
    e = field_errors(out, ref, w)
    print(f"[f1 alpha={alpha}]", e, flush=True)
    _assert_fields(e, 1e-5, 1)
