"""Pins of the oracle's vortex diagnostic (oracle/vortex.py, oracle.rot_intensity).

The intensity is pinned to the force oracle (it must be the spin part of the viscous pair
force per unit volume), to an invariant (a uniform spin field has no curl) and to the
continuum limit of the fifth term of Eq. 2; the image steps to hand-built layouts and the
component labels to an independent union-find.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import vortex as V
from paper_2405_03980_amd import inputs as I


def _lattice(n, hf=2.0):
    w = I.make_box(n, kernel=I.KERNEL_WENDLAND_C2, visc_frac=1.0, rigid=False, noise=0.0,
                   h_factor=hf)
    p = dict(w.params)
    p["sigma_T"] = p["C_l"] = 0.0
    return w, p


def test_intensity_is_spin_part_of_viscous_force():
    """For a viscous fluid particle with v = 0 the spin enters the force only through the
    viscous term's 2 eta V_i V_j F (w_i + w_j) x r, so I_i = rho_i |a(w) - a(0)|."""
    w = I.make_cylinder(14)
    rng = np.random.default_rng(3)
    om = rng.normal(size=w.omega.shape)
    rho, _, S = O.density(w.params, w.x, w.species, w.kind)
    zero = np.zeros(w.n)
    a1, _ = O.forces(w.params, w.x, 0 * w.v, om, w.species, w.kind, rho, zero, S)
    a0, _ = O.forces(w.params, w.x, 0 * w.v, 0 * om, w.species, w.kind, rho, zero, S)
    inten = O.rot_intensity(w.params, w.x, om, w.species, w.kind, rho)
    visc = (w.kind == I.FLUID) & (w.species == 1)
    expect = rho[visc] * np.linalg.norm(a1[:, visc] - a0[:, visc], axis=0)
    assert np.abs(inten[visc] - expect).max() < 1e-9 * expect.max()
    assert np.all(inten[w.kind != I.FLUID] == 0.0)
    assert np.all(inten[(w.kind == I.FLUID) & (w.species == 0)] > 0.0)  # inviscid too


def test_uniform_spin_has_no_intensity():
    """curl of a uniform spin field vanishes; on a perfect lattice the pair terms cancel."""
    w, p = _lattice(12)
    p["eta"] = 0.3
    om = np.zeros((3, w.n))
    om[:] = np.array([[0.3], [-1.1], [2.0]])
    rho = np.ones(w.n)
    inten = O.rot_intensity(p, w.x, om, w.species, w.kind, rho)
    scale = 2 * p["eta"] * 2.5 / p["h"]
    assert inten.max() < 1e-12 * scale


def test_intensity_curl_limit():
    """Eq. 2 fifth term: omega_z = A sin(kx) gives 2 eta |curl omega| = 2 eta A k |cos kx|."""
    A, K, eta = 0.1, 2 * math.pi, 0.01

    def mult(n):
        w, p = _lattice(n)
        p["eta"] = eta
        om = np.zeros((3, w.n))
        om[2] = A * np.sin(K * w.x[0])
        rho = np.ones(w.n)
        inten = O.rot_intensity(p, w.x, om, w.species, w.kind, rho)
        exp = 2 * eta * A * K * np.abs(np.cos(K * w.x[0]))
        return float(np.dot(inten, exp) / np.dot(exp, exp))

    c16, c32 = mult(16), mult(32)
    assert abs(c32 - 1) < abs(c16 - 1)
    assert abs((4 * c32 - c16) / 3 - 1.0) < 5e-3


def _union_find_labels(on):
    ny, nx = on.shape
    parent = list(range(nx * ny))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for iy in range(ny):
        for ix in range(nx):
            if not on[iy, ix]:
                continue
            for dy, dx in ((0, 1), (1, -1), (1, 0), (1, 1)):
                yy, xx = iy + dy, ix + dx
                if 0 <= yy < ny and 0 <= xx < nx and on[yy, xx]:
                    ra, rb = find(iy * nx + ix), find(yy * nx + xx)
                    if ra != rb:
                        parent[max(ra, rb)] = min(ra, rb)
    lab = np.full((ny, nx), -1, dtype=np.int64)
    for iy in range(ny):
        for ix in range(nx):
            if on[iy, ix]:
                lab[iy, ix] = find(iy * nx + ix)
    # canonical: smallest index of each component
    out = lab.copy()
    for r in np.unique(lab[lab >= 0]):
        m = lab == r
        out[m] = np.flatnonzero(m.ravel()).min()
    return out


@pytest.mark.parametrize("density", [0.2, 0.45, 0.6])
def test_components_equal_union_find(density):
    rng = np.random.default_rng(int(density * 100))
    on = rng.random((37, 53)) < density
    assert np.array_equal(V.components(on), _union_find_labels(on))


def test_component_shapes():
    on = np.zeros((12, 12), dtype=bool)
    on[1:6, 1] = on[1:6, 5] = on[1, 1:6] = on[5, 1:6] = True      # a ring: one component
    on[8, 8] = on[9, 9] = True                                      # diagonal touch: one
    on[8, 2] = True                                                 # a single pixel
    lab = V.components(on)
    assert len(np.unique(lab[lab >= 0])) == 3
    assert lab[3, 3] == -1                                          # the hole is off
    assert lab[9, 9] == 8 * 12 + 8
    assert V.count(lab, 1) == 3 and V.count(lab, 2) == 2 and V.count(lab, 3) == 1


def test_plane_image_layout():
    """Particles at chosen pixel centres and heights: the section keeps -dx <= dz < dx
    (z periodic), a pixel holds the largest intensity of its particles, walls never count."""
    p = dict(lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], dx=0.25)
    assert V.image_dims(p) == (4, 4)
    x = np.array([[0.1, 0.1, 0.6, 0.6, 0.9, 0.35],
                  [0.1, 0.2, 0.6, 0.6, 0.9, 0.35],
                  [0.3, 0.9, 0.5, 0.1, 0.0, 0.01]])
    kind = np.array([0, 0, 0, 0, 0, 1], dtype=np.uint8)
    inten = np.array([4.0, 3.0, 5.0, 2.0, 7.0, 9.0])
    img = V.plane_image(p, x, kind, inten, z0=0.0)
    want = np.zeros((4, 4))
    want[0, 0] = 3.0     # dz = 0.3 is out (>= dx), dz = -0.1 (0.9 wrapped) is in
    want[2, 2] = 2.0     # dz = 0.5 out, dz = 0.1 in
    want[3, 3] = 7.0     # dz = 0 in
    assert np.array_equal(img, want)
    on = V.threshold(img, 0.5)
    assert on.sum() == 1 and on[3, 3]
