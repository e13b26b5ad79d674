"""Pins of the oracle's pressure filter and collision step (Algorithm 1).

The paper names both steps and cites their models without formulas; the oracle follows
this project's reading (a volume-weighted Shepard average of the pressure; a pairwise
restitution impulse between particles closer than coll_alpha dx that approach each
other).  Each test checks what that reading fixes independently of the oracle's code:
preserved constants and linear fields, two-body mechanics (restitution, momentum), a
brute-force enumeration, and the conservation laws of the whole step.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from paper_2405_03980_amd import inputs as I


def _jittered_box(n_side=10, jitter=0.3, vscale=0.5, seed=11, kernel=I.KERNEL_WENDLAND_C2):
    w = I.make_box(n_side, kernel=kernel, rigid=False, seed=(3980, seed))
    rng = np.random.default_rng([3980, 100 + seed])
    dx = w.params["dx"]
    x = w.x + rng.uniform(-jitter, jitter, size=w.x.shape) * dx
    x = np.mod(x, 1.0)
    v = rng.normal(0.0, vscale, size=w.x.shape)
    return w, x, v


# -------------------------------------------------------------- pressure filter -----

def test_filter_keeps_a_constant():
    """A normalised average returns a constant field unchanged, whatever the volumes."""
    w, x, _ = _jittered_box()
    rng = np.random.default_rng([3980, 201])
    rho = rng.uniform(0.8, 1.25, w.n)
    P = np.full(w.n, 3.7)
    Pf = O.pressure_filter(w.params, x, w.species, w.kind, rho, P)
    assert np.abs(Pf - 3.7).max() < 1e-14 * 3.7


def test_filter_keeps_a_linear_field_on_a_lattice():
    """Away from walls every lattice neighbourhood is point-symmetric, so with equal
    volumes the first moment vanishes and a linear field is reproduced."""
    w = I.make_cylinder(16)
    f = w.kind == I.FLUID
    r = np.hypot(w.x[0], w.x[1])
    inner = f & (r < 1.0 - 3 * w.params["dx"] - 2 * w.params["h"] - 1e-9)
    P = 0.25 + 1.5 * w.x[0] - 0.75 * w.x[1] + 0.5 * w.x[2]
    # z enters only through the periodic seam, which breaks linearity: stay away from it
    lo_z, hi_z = 2 * w.params["h"] + 1e-9, 1.0 - 2 * w.params["h"] - 1e-9
    inner &= (w.x[2] > lo_z) & (w.x[2] < hi_z)
    rho = np.ones(w.n)
    Pf = O.pressure_filter(w.params, w.x, w.species, w.kind, rho, P)
    assert inner.sum() > 1000
    assert np.abs(Pf[inner] - P[inner]).max() < 1e-13


def test_filter_is_the_kernel_smoothing_in_the_limit():
    """At fixed h with dx -> 0 the lattice average tends to the kernel convolution, which
    multiplies cos(kx) by the kernel's Fourier transform 4 pi int W(r) sin(kr)/(kr) r^2 dr
    (by quadrature); the self weight is part of that lattice sum."""
    h, k = 0.125, 2 * math.pi
    what, _ = integrate.quad(lambda r: 4 * math.pi * r * r * O.W(I.KERNEL_WENDLAND_C2, h, r)
                             * math.sin(k * r) / (k * r), 0, 2 * h, epsabs=1e-14, epsrel=1e-13,
                             limit=200)
    errs = []
    for n in (16, 32):
        w = I.make_box(n, kernel=I.KERNEL_WENDLAND_C2, rigid=False, noise=0.0, h_factor=h * n)
        e = 0.1 * np.cos(k * w.x[0])
        Pf = O.pressure_filter(w.params, w.x, w.species, w.kind, np.ones(w.n), 1.0 + e)
        errs.append(abs(float(np.dot(Pf - 1.0, e) / np.dot(e, e)) - what))
    assert errs[1] < errs[0] and errs[1] < 5e-6, errs


def _W_wendland(h, r):
    q = r / h
    return 21.0 / (16.0 * math.pi * h ** 3) * (1 - q / 2) ** 4 * (2 * q + 1) if q < 2 else 0.0


def test_filter_two_particles_closed_form():
    """Two particles alone: each average holds the particle's own value at weight V W(0)
    and its partner's at weight V W(r)."""
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, 0.1, [0, 0, 0], [1, 1, 1], 1.0)
    h = p["h"]
    m = O.default_mass(p)
    x = np.array([[0.5, 0.5 + 0.17], [0.5, 0.5], [0.5, 0.5]])
    rho = np.array([1.05, 0.9])
    P = np.array([2.0, -1.0])
    sp = np.array([0, 1], np.uint8)
    Pf = O.pressure_filter(p, x, sp, np.zeros(2, np.uint8), rho, P)
    V = m[sp] / rho
    W0, Wr = _W_wendland(h, 0.0), _W_wendland(h, 0.17)
    e0 = (V[0] * P[0] * W0 + V[1] * P[1] * Wr) / (V[0] * W0 + V[1] * Wr)
    e1 = (V[1] * P[1] * W0 + V[0] * P[0] * Wr) / (V[1] * W0 + V[0] * Wr)
    assert abs(Pf[0] - e0) < 1e-14 and abs(Pf[1] - e1) < 1e-14


def test_filter_ignores_outer_walls():
    """Outer-wall pressures are boundary values: a uniform fluid and inner-wall pressure
    stays uniform next to them, and they keep theirs."""
    w = I.make_cylinder(16)
    P = np.where(w.kind == I.WALL_OUTER, 0.0, 1.3)
    rho = np.ones(w.n)
    Pf = O.pressure_filter(w.params, w.x, w.species, w.kind, rho, P)
    src = w.kind != I.WALL_OUTER
    assert np.abs(Pf[src] - 1.3).max() < 1e-14
    assert np.all(Pf[~src] == 0.0)


def test_filter_cells_equal_brute_force():
    w, x, _ = _jittered_box(8, seed=12)
    rng = np.random.default_rng([3980, 202])
    rho = rng.uniform(0.9, 1.1, w.n)
    P = rng.normal(0.0, 1.0, w.n)
    a = O.pressure_filter(w.params, x, w.species, w.kind, rho, P)
    b = O.pressure_filter(w.params, x, w.species, w.kind, rho, P, brute=True)
    assert np.abs(a - b).max() < 1e-14


def test_filter_is_on_the_pressure_the_forces_use():
    """With the filter on, the evaluation's pressure is the filtered EOS pressure."""
    w, x, v = _jittered_box(8, seed=13)
    p1 = dict(w.params, pressure_filter=1)
    rho, P, S = O.density(w.params, x, w.species, w.kind)
    Pf = O.pressure_filter(w.params, x, w.species, w.kind, rho, P)
    s = O.State(p1, x, v, w.omega, w.species, w.kind)
    assert np.abs(s.P - Pf).max() < 1e-13 * np.abs(Pf).max()
    acc, _ = O.forces(w.params, x, v, w.omega, w.species, w.kind, rho, Pf, S)
    assert np.abs(s.acc - acc).max() <= 1e-13 * np.abs(acc).max()


# -------------------------------------------------------------- collision step ------

def _pair(r, vi, vj, mi=1.0, mj=1.0, e=0.4, alpha=0.8, kinds=(0, 0)):
    dx = 0.1
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_OPEN, dx, [0, 0, 0], [1, 1, 1], 1.0)
    p["mass"] = [mi, mj]
    p["coll_alpha"], p["coll_e"] = alpha, e
    xi = np.array([0.5, 0.5, 0.5])
    x = np.stack([xi, xi - np.asarray(r)], axis=1)
    v = np.stack([np.asarray(vi, float), np.asarray(vj, float)], axis=1)
    sp = np.array([0, 1], np.uint8)
    kind = np.array(kinds, np.uint8)
    return p, x, v, sp, kind


@pytest.mark.parametrize("mi,mj,e", [(1.0, 1.0, 0.4), (1.0, 2.5, 0.0), (0.7, 1.3, 1.0)])
def test_collision_two_body_restitution(mi, mj, e):
    """An approaching pair closer than the collision distance leaves with the normal
    relative speed reversed and scaled by e, the tangential one and the momentum kept."""
    r = np.array([0.05, -0.02, 0.03])   # |r| = 0.0616 < 0.8 dx
    vi, vj = np.array([-1.0, 0.3, 0.2]), np.array([0.5, -0.1, -0.4])
    p, x, v, sp, kind = _pair(r, vi, vj, mi, mj, e)
    out = O.collide(p, x, v, sp, kind)
    n = r / np.linalg.norm(r)
    rel0, rel1 = v[:, 0] - v[:, 1], out[:, 0] - out[:, 1]
    assert rel0 @ n < 0
    assert abs(rel1 @ n + e * (rel0 @ n)) < 1e-14
    t0, t1 = rel0 - (rel0 @ n) * n, rel1 - (rel1 @ n) * n
    assert np.abs(t1 - t0).max() < 1e-14
    assert np.abs(mi * out[:, 0] + mj * out[:, 1] - (mi * vi + mj * vj)).max() < 1e-14
    if e == 1.0:
        E0 = 0.5 * (mi * vi @ vi + mj * vj @ vj)
        E1 = 0.5 * (mi * out[:, 0] @ out[:, 0] + mj * out[:, 1] @ out[:, 1])
        assert abs(E1 - E0) < 1e-14


def test_collision_needs_approach_and_proximity():
    r = np.array([0.05, -0.02, 0.03])
    # receding pair: unchanged
    p, x, v, sp, kind = _pair(r, [1.0, 0, 0], [-1.0, 0, 0])
    assert np.array_equal(O.collide(p, x, v, sp, kind), v)
    # approaching but beyond 0.8 dx: unchanged
    for d in (0.0801, 0.1, 0.2):
        p, x, v, sp, kind = _pair([d, 0, 0], [-1.0, 0, 0], [1.0, 0, 0])
        assert np.array_equal(O.collide(p, x, v, sp, kind), v)
    # just inside: changed
    p, x, v, sp, kind = _pair([0.0799, 0, 0], [-1.0, 0, 0], [1.0, 0, 0])
    assert not np.array_equal(O.collide(p, x, v, sp, kind), v)
    # switched off
    p, x, v, sp, kind = _pair(r, [-1.0, 0, 0], [1.0, 0, 0], alpha=0.0)
    assert np.array_equal(O.collide(p, x, v, sp, kind), v)


def test_collision_with_a_wall():
    """A wall moves as imposed: it keeps its velocity and the fluid particle alone takes
    the restitution, as against an infinite mass."""
    r = np.array([0.0, 0.06, 0.0])
    vi, vj = np.array([0.2, -2.0, 0.1]), np.array([0.3, 0.0, 0.0])
    p, x, v, sp, kind = _pair(r, vi, vj, e=0.25, kinds=(0, 1))
    out = O.collide(p, x, v, sp, kind)
    assert np.array_equal(out[:, 1], vj)
    assert abs((out[:, 0] - vj)[1] - (-0.25) * (vi - vj)[1]) < 1e-15
    assert out[0, 0] == vi[0] and out[2, 0] == vi[2]


def test_collision_conserves_momentum_in_a_crowd():
    """All impulses are central and pairwise opposite between fluid particles: sum m v
    and sum m x × v are unchanged however many pairs collide at once."""
    w = I.make_cluster(9, jitter=0.35, noise=0.5)
    p = dict(w.params, coll_alpha=0.8, coll_e=0.3, mass=[1.0, 1.7])
    out = O.collide(p, w.x, w.v, w.species, w.kind)
    m = np.array([1.0, 1.7])[w.species]
    moved = np.any(out != w.v, axis=0)
    assert moved.sum() > 50
    P0, P1 = (m * w.v).sum(axis=1), (m * out).sum(axis=1)
    J0 = (m * np.cross(w.x.T, w.v.T).T).sum(axis=1)
    J1 = (m * np.cross(w.x.T, out.T).T).sum(axis=1)
    scale = (m * np.abs(w.v)).sum()
    assert np.abs(P1 - P0).max() < 1e-14 * scale
    assert np.abs(J1 - J0).max() < 1e-14 * scale


def test_collision_cells_equal_brute_force():
    w = I.make_cluster(8, jitter=0.35, noise=0.5)
    p = dict(w.params, coll_alpha=0.8, coll_e=0.3)
    a = O.collide(p, w.x, w.v, w.species, w.kind)
    b = O.collide(p, w.x, w.v, w.species, w.kind, brute=True)
    assert np.abs(a - b).max() < 1e-15 * np.abs(a).max()


def test_collision_parameters_are_checked():
    w = I.make_cluster(6)
    for bad in (dict(coll_alpha=-0.1), dict(coll_alpha=2.6 + 1e-9, coll_e=0.5),
                dict(coll_alpha=0.8, coll_e=1.5), dict(coll_alpha=0.8, coll_e=-0.1),
                dict(pressure_filter=2)):
        with pytest.raises(O.OracleError):
            O.collide(dict(w.params, **bad), w.x, w.v, w.species, w.kind)


# ---------------------------------------------------------------- whole step --------

def test_step_with_filter_and_collisions_conserves_momentum():
    """The filtered pressure enters every pair symmetrically and collisions are pairwise
    central, so a free cluster still keeps sum m v and sum (m x × v + I omega)."""
    w = I.make_cluster(8, jitter=0.3, noise=0.3)
    p = dict(w.params, pressure_filter=1, coll_alpha=0.85, coll_e=0.2)
    s = O.State(p, w.x, w.v, w.omega, w.species, w.kind)
    P0, J0, _ = s.diagnostics()
    s.step(1e-4, 0.0, 20)
    P1, J1, _ = s.diagnostics()
    m = O.default_mass(p)
    scale = m[0] * w.n * (np.abs(s.v).max() + 1e-2)
    assert np.abs(P1 - P0).max() < 1e-14 * scale
    assert np.abs(J1 - J0).max() < 1e-14 * (scale + m[0] * p["kappa_I"] * p["dx"] ** 2 * w.n)


def test_step_collision_happens_after_the_drift():
    """One step with the collision on equals: kick and drift, collision of the half-step
    velocities at the new positions, then the evaluation and the closing kick."""
    w = I.make_cluster(7, jitter=0.35, noise=0.5)
    p = dict(w.params, coll_alpha=0.8, coll_e=0.3)
    dt = 1e-4
    s = O.State(p, w.x, w.v, w.omega, w.species, w.kind)
    a0, al0 = s.acc.copy(), s.alpha.copy()
    s.step(dt, 0.0, 1)
    vh = w.v + 0.5 * dt * a0
    x1 = w.x + dt * vh
    vc = O.collide(p, x1, vh, w.species, w.kind)
    wh = w.omega + 0.5 * dt * al0
    ref = O.State(p, x1, vc, wh, w.species, w.kind)
    assert np.array_equal(s.x, x1)
    assert np.abs(s.v - (vc + 0.5 * dt * ref.acc)).max() < 1e-15
    assert np.any(vc != vh)
