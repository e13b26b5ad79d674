"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 path 1e-12 per field; FP32-mixed path 1e-5 after one step and 1e-3
after 100 steps (normwise relative, fluid particles; positions as displacement, pressure
over the Tait stiffness B).  Cell lists and neighbour sets must match bit for bit when
both sides see the same positions.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_03980_amd import _lib as L
from paper_2405_03980_amd import inputs as I
from tests._parity import field_errors, mixed_tol, positions_ok

pytestmark = pytest.mark.gpu

FP64, MIXED = L.FP64, L.FP32_MIXED


def _sim(w, prec, **tune):
    """A simulation of w whose first evaluation (at init) already uses the given tuning."""
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(w.params, w.n, precision=prec)
    if tune:
        s.set_tuning(**tune)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    return s


def _jitter_box(n=12, seed=1, amp=0.3, kernel=I.KERNEL_WENDLAND_C2, **kw):
    w = I.make_box(n, kernel=kernel, **kw)
    rng = np.random.default_rng(seed)
    w.x = np.mod(w.x + rng.uniform(-amp, amp, size=w.x.shape) / n, 1.0)
    w.v = w.v + rng.normal(0, 0.05, size=w.v.shape)
    w.omega = rng.normal(0, 1.0, size=w.omega.shape)
    return w


CELL_CASES = {
    "box4096": lambda: I.config(0),
    "cylinder": lambda: I.make_cylinder(14),
    "cluster": lambda: I.make_cluster(9),
    "box_cf2": lambda: I.make_box(14, cell_factor=2),
    "jitter": lambda: _jitter_box(13),
}


@pytest.mark.parametrize("case", list(CELL_CASES))
def test_cells_bit_exact(case):
    w = CELL_CASES[case]()
    print(f"[cells] {case} n={w.n}", flush=True)
    s = _sim(w, FP64)
    key, perm, cs = s.debug_cells()
    okey, operm, ocs = O.cells(w.params, w.x)
    assert np.array_equal(key, okey)
    assert np.array_equal(perm, operm)
    assert np.array_equal(cs, ocs)
    s.close()


@pytest.mark.parametrize("case", ["box4096", "cylinder", "jitter", "box_cf2"])
def test_neighbors_bit_exact(case):
    w = CELL_CASES[case]()
    print(f"[nbr] {case} n={w.n}", flush=True)
    s = _sim(w, MIXED)
    row, cols = s.debug_neighbors()
    orow, ocols = O.neighbors(w.params, w.x)
    assert np.array_equal(row, orow)
    assert np.array_equal(cols, ocols)
    s.close()


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (MIXED, 1e-5)])
@pytest.mark.parametrize("case", ["box4096", "cylinder", "jitter"])
def test_initial_fields(case, prec, tol):
    w = CELL_CASES[case]()
    print(f"[init] {case} prec={prec} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, prec)
    out = s.read()
    e = field_errors(out, ref, w)
    print(e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < tol, (k, e[k])
    assert np.array_equal(out["x"], w.x)
    s.close()


def test_box4096_fp64_20_steps():
    w = I.config(0)
    ref = O.State.from_workload(w)
    ref.step(w.dt, w.Omega, w.steps)
    s = _sim(w, FP64)
    s.step(w.dt, w.Omega, w.steps)
    e = field_errors(s.read(), ref, w)
    print("box4096 fp64 20 steps", e, flush=True)
    assert positions_ok(e, 1e-12, w.steps)
    assert max(v for k, v in e.items() if not k.startswith("x")) < 1e-12
    s.close()


@pytest.mark.parametrize("prec,steps,tol", [(FP64, 100, 1e-12), (MIXED, 1, 1e-5), (MIXED, 100, 1e-3)])
def test_cylinder_steps(prec, steps, tol):
    w = I.make_cylinder(16, seed=(3980, 1))
    print(f"[cyl] prec={prec} steps={steps} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, steps)
    s = _sim(w, prec)
    s.step(1e-4, w.Omega, steps)
    e = field_errors(s.read(), ref, w)
    print(e, flush=True)
    assert positions_ok(e, tol, steps), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < tol, (k, e[k])
    s.close()


TERMS = {
    "pressure": dict(eta=0.0, sigma_T=0.0, C_l=0.0),
    "interfacial": dict(eta=0.0, sigma_T=3.0, C_l=0.0, c0=0.0),
    "viscous": dict(eta=0.2, sigma_T=0.0, C_l=0.0, c0=0.0),
    "friction": dict(eta=0.0, sigma_T=0.0, C_l=5.0, c0=0.0),
}


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (MIXED, 1e-5)])
@pytest.mark.parametrize("term", list(TERMS))
def test_term_isolation(term, prec, tol):
    """Each pair term alone with O(1) coefficients, so a small term cannot hide under
    the tolerance of the others."""
    w = _jitter_box(12, seed=7)
    w.params = dict(w.params, **TERMS[term])
    if w.params["c0"] == 0.0:
        w.params["c0"] = 1e-9
    ref = O.State.from_workload(w)
    s = _sim(w, prec)
    e = field_errors(s.read(), ref, w)
    print(term, prec, e, flush=True)
    assert e["acc"] < tol and e["alpha"] < tol
    s.close()


def test_conservation_on_gpu():
    w = I.make_cluster(10)
    s = _sim(w, FP64)
    P0, J0, E0 = s.diagnostics()
    oP, oJ, oE = O.State.from_workload(w).diagnostics()
    assert np.allclose(P0, oP, rtol=1e-13, atol=1e-18) and np.allclose(J0, oJ, rtol=1e-13, atol=1e-18)
    s.step(1e-4, 0.0, 40)
    P1, J1, E1 = s.diagnostics()
    m = O.default_mass(w.params)[0]
    scale = m * w.n * 0.05
    assert np.abs(P1 - P0).max() < 1e-13 * scale
    assert np.abs(J1 - J0).max() < 1e-13 * scale
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_batch_equals_single(prec):
    ws = I.make_batch(5, scale=0.05)
    print("[batch] sizes", [w.n for w in ws], flush=True)
    from paper_2405_03980_amd import sim as S
    b = S.batch_from(ws, precision=prec)
    Om = [w.Omega for w in ws]
    b.step(1e-4, Om, 7)
    out = b.read()
    for i, w in enumerate(ws):
        s = _sim(w, prec)
        s.step(1e-4, w.Omega, 7)
        o = s.read()
        lo, hi = b.offsets[i], b.offsets[i + 1]
        for k in ("x", "v", "omega", "rho", "P", "acc"):
            assert np.array_equal(out[k][..., lo:hi], o[k]), (i, k)
        s.close()
    d = b.diagnostics()
    assert d.shape == (5, 7)
    b.close()


def test_batch_mixing_kernels_and_geometries():
    """One ensemble holding a cubic-spline periodic box, a jittered Wendland box and two
    Wendland cylinders: the brick sweeps choose their compiled copy per brick, and every
    instance equals its own single run bit for bit and the oracle within 1e-5."""
    from paper_2405_03980_amd import sim as S
    ws = [I.config(0), _jitter_box(11, seed=5), I.make_cylinder(12), I.make_cylinder(15, seed=(3980, 9))]
    print("[batch mix] sizes", [w.n for w in ws], flush=True)
    b = S.batch_from(ws, precision=MIXED)
    b.set_tuning(sweep=3)
    b.step(1e-4, [w.Omega for w in ws], 3)
    out = b.read()
    b.close()
    for i, w in enumerate(ws):
        s = _sim(w, MIXED, sweep=3)
        s.step(1e-4, w.Omega, 3)
        o = s.read()
        s.close()
        lo, hi = b.offsets[i], b.offsets[i + 1]
        for k in ("x", "v", "omega", "rho", "P", "acc"):
            assert np.array_equal(out[k][..., lo:hi], o[k]), (i, k)
        ref = O.State.from_workload(w)
        ref.step(1e-4, w.Omega, 3)
        e = field_errors({k: v[..., lo:hi] for k, v in out.items()}, ref, w)
        assert positions_ok(e, 1e-5, 3), (i, e)
        for k in ("v", "omega", "rho", "P"):
            assert e[k] < 1e-5, (i, k, e[k])


@pytest.mark.parametrize("prec,sweep,tol", [(FP64, None, 1e-12), (MIXED, 1, 1e-5), (MIXED, 3, 1e-5)])
def test_unequal_species_masses(prec, sweep, tol):
    """Per-species masses (the viscous species 5% heavier, so its lattice density sits 5%
    above rho0): every sweep takes its unequal-mass form of the mass-dependent pair factors,
    from the first evaluation on."""
    w = _jitter_box(12, seed=11)
    m = float(O.default_mass(w.params)[0])
    w.params = dict(w.params, mass=[m, 1.05 * m])
    print(f"[masses] prec={prec} sweep={sweep} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, prec, sweep=sweep) if sweep else _sim(w, prec)
    e = field_errors(s.read(), ref, w)
    print("unequal masses, first evaluation", e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < tol, (k, e[k])
    ref.step(1e-4, w.Omega, 3)
    s.step(1e-4, w.Omega, 3)
    e = field_errors(s.read(), ref, w)
    print("unequal masses, 3 steps", e, flush=True)
    assert positions_ok(e, tol, 3), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < tol, (k, e[k])
    s.close()


def test_three_cell_periodic_box():
    """A periodic box only three cells wide: each brick's 4x4x4 neighbourhood wraps onto
    itself (one cell staged twice, under two image shifts) and must still give each target
    every neighbour exactly once."""
    w = _jitter_box(8, seed=3, amp=0.2, h_factor=1.3)
    from oracle import oracle as O_
    dims, _ = O_.grid_dims(w.params)
    assert list(dims) == [3, 3, 3], dims
    ref = O.State.from_workload(w)
    s = _sim(w, MIXED, sweep=3)
    e = field_errors(s.read(), ref, w)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < 1e-5, (k, e[k])
    ref.step(1e-4, w.Omega, 2)
    s.step(1e-4, w.Omega, 2)
    e = field_errors(s.read(), ref, w)
    print("3-cell box", e, flush=True)
    assert positions_ok(e, 1e-5, 2), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_graph_replay_equals_eager(prec):
    w = I.make_cylinder(12)
    a = _sim(w, prec, use_graph=1)
    b = _sim(w, prec, use_graph=0)
    for it in range(3):
        a.step(1e-4, 1.0, 6)
        b.step(1e-4, 1.0, 6)
        oa, ob = a.read(), b.read()
        for k in oa:
            assert np.array_equal(oa[k], ob[k]), (it, k)
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_runs_are_bitwise_reproducible(prec):
    """Two independent simulations of the same input give identical bits: every summation
    order is fixed (cell order by id, fixed group trees, no floating-point atomics)."""
    w = I.make_cylinder(40, seed=(3980, 2))
    print(f"[repro] prec={prec} n={w.n}", flush=True)
    outs = []
    for _ in range(2):
        s = _sim(w, prec)
        s.step(1e-4, w.Omega, 5)
        outs.append(s.read())
        s.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_resume_from_checkpoint():
    """read_fields -> init_particles round trip: the fields come back unchanged, and a
    resumed run tracks the oracle resumed from its own checkpoint.  (Resuming is not
    bit-identical to continuing: velocity Verlet evaluates velocity-dependent forces at
    the half-step velocity, the restart at the full-step one.)"""
    from paper_2405_03980_amd import sim as S
    # rigidly rotating box: positions move ~1e-3, far above their rounding (a resting
    # cylinder moves ~1e-6, where one ulp of x is already 1e-10 of the displacement)
    w = I.config(0)
    half = _sim(w, FP64)
    half.step(1e-4, 1.0, 10)
    ck = half.read()
    res = S.Simulation(w.params, w.n, precision=FP64)
    res.init(ck["x"], ck["v"], ck["omega"], w.species, w.kind)
    again = res.read()
    for k in ("x", "v", "omega"):
        assert np.array_equal(again[k], ck[k]), k
    res.step(1e-4, 1.0, 10)
    out = res.read()
    ref = O.State.from_workload(w)
    ref.step(1e-4, 1.0, 10)
    ref = O.State(w.params, ref.x, ref.v, ref.omega, w.species, w.kind)
    ref.step(1e-4, 1.0, 10)
    e = field_errors(out, ref, w)
    print("resume", e, flush=True)
    assert positions_ok(e, 1e-12, 20), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-12, (k, e[k])
    for s in (half, res):
        s.close()


def test_nonfinite_input_is_reported():
    w = I.make_cylinder(10)
    w.v[0, 5] = np.nan
    s = _sim(w, MIXED)
    with pytest.raises(L.SphError) as e:
        s.sync()
    assert e.value.status == L.E_NONFINITE
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_nonfinite_spin_of_a_lone_particle_is_reported(prec):
    """A particle without neighbours never reaches the pair sweeps, so a NaN spin can only
    be caught where the state is stored (the reorder check)."""
    x = np.array([[0.2, 0.7], [0.5, 0.5], [0.5, 0.5]])
    om = np.array([[0.0, np.nan], [0.0, 0.0], [0.0, 0.0]])
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, 0.05, [0, 0, 0], [1, 1, 1], 1.0)
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(p, 2, precision=prec)
    s.init(x, np.zeros((3, 2)), om, np.zeros(2, np.uint8), np.zeros(2, np.uint8))
    with pytest.raises(L.SphError) as e:
        s.sync()
    assert e.value.status == L.E_NONFINITE
    s.close()


def test_domain_exit_is_reported():
    w = I.make_cluster(5)
    w.v[0, 0] = 1e4  # leaves the open grid in one step
    s = _sim(w, FP64)
    s.step(1e-4, 0.0, 1)
    with pytest.raises(L.SphError) as e:
        s.read()
    assert e.value.status == L.E_DOMAIN
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_leaving_the_cylinder_is_reported(prec):
    """A cylinder instance's particles stay within 2h of the cylinder inscribed in the box's
    x-y extent, which lets the brick sweeps leave out the bricks beyond it.  A fluid
    particle placed in a corner of the box (inside the box, beyond the cylinder) is a domain
    error at the first evaluation; one moving there is reported after the step that takes
    it."""
    w = I.make_cylinder(14)
    f = int(np.nonzero(w.kind == I.FLUID)[0][0])
    x = w.x.copy()
    x[0, f], x[1, f] = 0.95, 0.95  # radius 1.34 > 1, in the box [-1, 1]^2
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(w.params, w.n, precision=prec)
    with pytest.raises(L.SphError) as e:
        s.init(x, w.v, w.omega, w.species, w.kind)
        s.sync()
    assert e.value.status == L.E_DOMAIN, e.value
    s.close()
    # moving out: the outermost fluid particle on the diagonal, sent in one step to
    # (0.9, 0.9), inside the box and outside the cylinder
    x, v = w.x.copy(), w.v.copy()
    r = np.hypot(x[0], x[1])
    diag = (w.kind == I.FLUID) & (x[0] > 0) & (np.abs(x[0] - x[1]) < 2 * w.params["dx"])
    f = int(np.argmax(np.where(diag, r, -1.0)))
    dt = 1e-4
    v[0, f], v[1, f], v[2, f] = (0.9 - x[0, f]) / dt, (0.9 - x[1, f]) / dt, 0.0
    s = _sim(I.Workload(w.name, w.params, x, v, w.omega, w.species, w.kind), prec)
    s.step(dt, w.Omega, 1)
    with pytest.raises(L.SphError) as e:
        s.read()
    assert e.value.status == L.E_DOMAIN
    s.close()


def test_invalid_species_is_reported():
    w = I.make_cylinder(10)
    w.species[w.kind != I.FLUID] = 0   # walls must be viscous
    s = _sim(w, MIXED)
    with pytest.raises(L.SphError) as e:
        s.sync()
    assert e.value.status == L.E_INVALID
    s.close()


def test_step_before_init_is_a_state_error():
    from paper_2405_03980_amd import sim as S
    w = I.make_cylinder(10)
    s = S.Simulation(w.params, w.n, precision=MIXED)
    with pytest.raises(L.SphError) as e:
        s.step(1e-4, 1.0, 1)
    assert e.value.status == L.E_STATE
    s.close()


@pytest.mark.parametrize("case", ["cylinder", "box4096", "jitter"])
def test_brick_sweep_matches_thread_sweep(case):
    """The LDS-staged brick sweeps and the per-particle sweeps compute the same FP32-mixed
    fields up to single-precision rounding."""
    sweep = 3
    w = CELL_CASES[case]()
    print(f"[brick] {case} sweep={sweep} n={w.n}", flush=True)
    a = _sim(w, MIXED, sweep=sweep)
    b = _sim(w, MIXED, sweep=1)
    assert a.get_tuning()["sweep"] == sweep and b.get_tuning()["sweep"] == 1
    a.step(1e-4, w.Omega, 5)
    b.step(1e-4, w.Omega, 5)
    oa, ob = a.read(), b.read()
    f = w.kind == I.FLUID
    for k in ("v", "omega", "rho", "acc", "alpha"):
        ref = ob[k][..., f]
        err = np.abs(oa[k][..., f] - ref).max() / np.abs(ref).max()
        assert err < 1e-5, (k, err)
    a.close()
    b.close()


@pytest.mark.parametrize("h_factor", [1.6, 2.2])
def test_brick_fallback_when_cells_are_full(h_factor):
    """Neighbourhoods too large to stage fall back to the per-particle code path."""
    sweep = 3
    w = I.make_box(20, kernel=I.KERNEL_WENDLAND_C2, h_factor=h_factor)
    print(f"[fallback] h/dx={h_factor} sweep={sweep} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, MIXED, sweep=sweep)
    e = field_errors(s.read(), ref, w)
    print("fallback", h_factor, e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < 1e-5, (k, e[k])
    s.close()


@pytest.mark.parametrize("visc_frac", [0.0, 0.5, 1.0])
def test_brick_of_512_targets(visc_frac):
    """One brick alone in an open domain, its eight cells holding 64 particles each (an 8^3
    cluster with h = 2 dx): every cell is taken from the stage, the force sweep's waves get
    shares of up to 69 targets (two rounds of lanes) with either species, all inviscid
    waves or all viscous ones, and every field matches the oracle initially and after a
    step."""
    w = I.make_cluster(8, h_factor=2.0, visc_frac=visc_frac)
    h, x = w.params["h"], w.x
    cells = np.floor(x / (2.0 * h)).astype(int)
    assert np.all((cells >= 2) & (cells <= 3)), "the cluster must fill exactly one brick"
    counts = np.bincount((cells[0] - 2) + 2 * (cells[1] - 2) + 4 * (cells[2] - 2), minlength=8)
    assert np.all(counts == 64), counts
    print(f"[brick512] visc_frac={visc_frac} n={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, MIXED, sweep=3)
    e = field_errors(s.read(), ref, w)
    print("initial", e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < 1e-5, (k, e[k])
    ref.step(1e-4, w.Omega, 1)
    s.step(1e-4, w.Omega, 1)
    e = field_errors(s.read(), ref, w)
    print("one step", e, flush=True)
    assert positions_ok(e, 1e-5, 1), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])
    s.close()


@pytest.mark.parametrize("prec,sweep", [(FP64, None), (MIXED, 1), (MIXED, 3)])
def test_overfull_cell_is_a_capacity_error(prec, sweep):
    """1,100 particles gathered in one cell (more than the 1,024 the search walks): the
    sweeps skip that cell, every kernel stays bounded, and the next synchronising call
    reports SPH_E_CAPACITY."""
    w = I.make_box(12, kernel=I.KERNEL_WENDLAND_C2)
    rng = np.random.default_rng(5)
    lo, edge = 0.25, 0.25  # cell (1, 1, 1) of the 4x4x4 grid
    w.x = w.x.copy()
    w.x[:, :1100] = lo + edge * rng.uniform(0.05, 0.95, size=(3, 1100))
    w.v = np.zeros_like(w.v)
    print(f"[capacity] prec={prec} sweep={sweep} n={w.n}", flush=True)
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(w.params, w.n, precision=prec)
    if sweep:
        s.set_tuning(sweep=sweep)
    with pytest.raises(L.SphError) as e:
        s.init(w.x, w.v, w.omega, w.species, w.kind)
        s.sync()
    assert e.value.status == L.E_CAPACITY, e.value
    s.close()


@pytest.mark.parametrize("value", [2, 4, -1])
def test_tuning_rejects_unknown_sweep(value):
    """Only 0 (keep), 1 and 3 name a sweep; anything else is an argument error that leaves
    the current setting alone."""
    s = _sim(I.make_box(8), MIXED)
    with pytest.raises(L.SphError) as e:
        s.set_tuning(sweep=value)
    assert e.value.status == L.E_INVALID
    assert s.get_tuning()["sweep"] == 3
    s.close()


@pytest.mark.parametrize("n", [19, 23])
def test_candidate_sweep_falls_back_for_long_stencils(n):
    """Boxes whose 27-cell stencils reach 729 candidates (more than the 640 a wave holds):
    those waves take the per-particle path, the rest of the brick the candidate-major one
    (n = 23 also has bricks that fit the density sweep's LDS but not the force sweep's);
    all match the oracle, initially and after a step."""
    w = _jitter_box(n, seed=n, amp=0.05, h_factor=1.3)
    print(f"[cand fallback] box n={n} particles={w.n}", flush=True)
    ref = O.State.from_workload(w)
    s = _sim(w, MIXED, sweep=3)
    e = field_errors(s.read(), ref, w)
    print("initial", e, flush=True)
    for k in ("rho", "P", "acc", "alpha"):
        assert e[k] < 1e-5, (k, e[k])
    ref.step(1e-4, w.Omega, 1)
    s.step(1e-4, w.Omega, 1)
    e = field_errors(s.read(), ref, w)
    print("one step", e, flush=True)
    assert positions_ok(e, 1e-5, 1), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < 1e-5, (k, e[k])
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_single_particle_is_ballistic(prec):
    x = np.array([[0.4], [0.5], [0.6]])
    v = np.array([[0.3], [-0.2], [0.1]])
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, 0.05, [0, 0, 0], [1, 1, 1], 1.0)
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(p, 1, precision=prec)
    s.init(x, v, np.zeros((3, 1)), np.zeros(1, np.uint8), np.zeros(1, np.uint8))
    s.step(1e-3, 0.0, 100)
    out = s.read()
    assert np.allclose(out["x"], x + 0.1 * v, rtol=0, atol=1e-14)
    assert np.array_equal(out["v"], v) and np.all(out["acc"] == 0)
    rho_self = O.default_mass(p)[0] * O.W(p["kernel"], p["h"], 0.0)
    assert abs(out["rho"][0] - rho_self) < (1e-12 if prec == FP64 else 1e-6) * rho_self
    s.close()


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (MIXED, 1e-5)])
def test_two_particles(prec, tol):
    x = np.array([[0.5, 0.5 + 0.031], [0.5, 0.5 + 0.012], [0.5, 0.5 - 0.007]])
    v = np.array([[0.1, -0.2], [0.0, 0.3], [0.05, 0.0]])
    om = np.array([[0.0, 1.0], [2.0, 0.0], [0.5, -0.5]])
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, 0.03, [0, 0, 0], [1, 1, 1], 1.0)
    p["sigma_T"], p["C_l"], p["eta"] = 0.2, 0.3, 0.05
    sp = np.array([0, 1], np.uint8)
    kd = np.zeros(2, np.uint8)
    from paper_2405_03980_amd import sim as S
    s = S.Simulation(p, 2, precision=prec)
    s.init(x, v, om, sp, kd)
    s.step(1e-4, 0.0, 3)
    out = s.read()
    ref = O.State(p, x, v, om, sp, kd)
    ref.step(1e-4, 0.0, 3)
    for k in ("v", "omega", "rho", "acc", "alpha"):
        r = getattr(ref, k)
        assert np.abs(out[k] - r).max() <= tol * np.abs(r).max(), k
    s.close()


@pytest.mark.parametrize("visc_frac", [0.0, 1.0])
@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (MIXED, mixed_tol(5))])
def test_single_species_mixture(visc_frac, prec, tol):
    """No unlike pairs (S = 0 everywhere) or only viscous pairs, 5 steps.  With an
    inviscid fluid the spins come only from the torques of the wall pairs, so the largest
    spin is small and the normwise spin error of the FP32-mixed path, about 1e-5 after 5
    steps, is the largest of any field here: the bar is the path's 1e-5 per step."""
    w = I.make_cylinder(12, visc_frac=visc_frac)
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 5)
    s = _sim(w, prec)
    s.step(1e-4, w.Omega, 5)
    e = field_errors(s.read(), ref, w)
    print("single species", visc_frac, prec, e, flush=True)
    assert positions_ok(e, tol, 5), e
    for k in ("v", "omega", "rho", "P"):
        assert e[k] < tol, (k, e[k])
    s.close()
