"""Cross-check of the C oracle against an independent NumPy all-pairs evaluation.

Not a pin (it restates the same definitions), but a second implementation with nothing in
common with the oracle's code: dense pair matrices instead of cell lists and sorted
neighbour sets, vectorised sums instead of per-particle loops.  It catches slips in the
oracle's indexing, neighbour search, sum order or term selection.  The definitions follow
the readings of the paper: density and Tait EOS (Eq. 4), pressure filter (Algorithm 1),
pressure, interfacial, spin-corrected viscous and mutual-friction pair forces with their
torques (Eqs. 1-2), and the collision step (Algorithm 1).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_03980_amd import inputs as I


def _wendland(h, r):
    q = r / h
    c = 21.0 / (16.0 * math.pi * h ** 3)
    t = np.clip(1.0 - q / 2.0, 0.0, None)
    W = c * t ** 4 * (2.0 * q + 1.0)
    F = c * 5.0 * t ** 3 / h ** 2  # -W'(r)/r
    return W, F


def _eval(p, x, v, w, sp, kind, filt):
    """rho, P, acc, alpha of every particle, all pairs at once (open domain)."""
    n = x.shape[1]
    m = np.asarray(p["mass"])[sp]
    r = x[:, :, None] - x[:, None, :]                      # r_ij = x_i - x_j
    r2 = (r[0] ** 2 + r[1] ** 2) + r[2] ** 2
    nb = (r2 < (2.0 * p["h"]) ** 2) & ~np.eye(n, dtype=bool)
    W, F = _wendland(p["h"], np.sqrt(r2))
    W, F = np.where(nb, W, 0.0), np.where(nb, F, 0.0)
    W0 = _wendland(p["h"], 0.0)[0]
    outer = kind == I.WALL_OUTER
    rho = np.where(outer, p["rho0"], m * (W0 + W.sum(1)))
    unlike = sp[:, None] != sp[None, :]
    S = (W * unlike).sum(1)
    B = p["rho0"] * p["c0"] ** 2 / 7.0
    P = np.where(outer, 0.0, B * ((rho / p["rho0"]) ** 7 - 1.0))
    V = m / rho
    if filt:
        src = ~outer
        num = V * P * W0 + (W * (src * V * P)[None, :]).sum(1)
        den = V * W0 + (W * (src * V)[None, :]).sum(1)
        P = np.where(outer, P, num / den)
    mm = m[:, None] * m[None, :]
    gp = mm * (P / rho ** 2)[:, None] + mm * (P / rho ** 2)[None, :]
    f = gp * F * r                                          # pressure, all pairs
    gT = -p["sigma_T"] * mm * ((1 / rho ** 2)[:, None] + (1 / rho ** 2)[None, :]) * F * unlike
    f[0] += gT * r[0]
    f[1] += gT * r[1]
    vij = v[:, :, None] - v[:, None, :]
    hs = 0.5 * (w[:, :, None] + w[:, None, :])
    u = vij - np.cross(hs, r, axis=0)
    both_n = (sp[:, None] == 1) & (sp[None, :] == 1)
    gv = -4.0 * p["eta"] * V[:, None] * V[None, :] * F * both_n
    VS = np.where(S > 0, V / np.where(S > 0, S, 1.0), 0.0)
    gm = -p["C_l"] * W * (VS[:, None] + VS[None, :]) * unlike
    fnc = gv * u + gm * vij
    f = f + fnc
    tau = -0.5 * np.cross(r, fnc, axis=0)
    tau[0] += -0.5 * gT * (-r[2] * r[1])
    tau[1] += -0.5 * gT * (r[2] * r[0])
    fluid = kind == I.FLUID
    I_ = p["kappa_I"] * m * p["dx"] ** 2
    acc = np.where(fluid, f.sum(2) / m, 0.0)
    alpha = np.where(fluid, tau.sum(2) / I_, 0.0)
    return rho, P, acc, alpha


def _collide(p, x, v, sp, kind):
    n = x.shape[1]
    m = np.asarray(p["mass"])[sp]
    r = x[:, :, None] - x[:, None, :]
    r2 = (r[0] ** 2 + r[1] ** 2) + r[2] ** 2
    rc = p["coll_alpha"] * p["dx"]
    near = (r2 < rc * rc) & ~np.eye(n, dtype=bool)
    vn = ((v[:, :, None] - v[:, None, :]) * r).sum(0)
    act = near & (vn < 0)
    fluid = kind == I.FLUID
    mu = np.where(fluid[None, :], m[None, :] / (m[:, None] + m[None, :]), 1.0)
    g = np.where(act, -(1 + p["coll_e"]) * mu * vn / np.where(r2 > 0, r2, 1.0), 0.0)
    dv = (g * r).sum(2)
    return np.where(fluid, v + dv, v)


def _case(kind_mix):
    w = I.make_cluster(7, jitter=0.35, noise=0.3, spin=1.0)
    p = dict(w.params, mass=[1.3e-4, 1.7e-4], eta=0.3, sigma_T=0.7, C_l=2.0, c0=3.0,
             pressure_filter=1, coll_alpha=0.85, coll_e=0.4)
    kind = w.kind.copy()
    sp = w.species.copy()
    if kind_mix:
        # some inner and outer wall particles (walls are the viscous species)
        rng = np.random.default_rng([3980, 501])
        pick = rng.choice(w.n, 60, replace=False)
        kind[pick[:30]] = I.WALL_INNER
        kind[pick[30:]] = I.WALL_OUTER
        sp[pick] = I.VISCOUS
    return w, p, sp, kind


@pytest.mark.parametrize("filt", [0, 1])
@pytest.mark.parametrize("kind_mix", [False, True])
def test_oracle_evaluation_equals_all_pairs(filt, kind_mix):
    w, p, sp, kind = _case(kind_mix)
    p = dict(p, pressure_filter=filt)
    s = O.State(p, w.x, w.v, w.omega, sp, kind)
    rho, P, acc, alpha = _eval(p, w.x, w.v, w.omega, sp, kind, filt)
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(s.rho, rho) < 1e-13
    assert rel(s.P, P) < 1e-12
    assert rel(s.acc, acc) < 1e-12
    assert rel(s.alpha, alpha) < 1e-12


@pytest.mark.parametrize("kind_mix", [False, True])
def test_oracle_collision_equals_all_pairs(kind_mix):
    w, p, sp, kind = _case(kind_mix)
    out = O.collide(p, w.x, w.v, sp, kind)
    ref = _collide(p, w.x, w.v, sp, kind)
    assert np.any(ref != w.v)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()
