"""Vortex diagnostic on the GPU (sph_vortex_image) against the oracle (oracle/vortex.py).

Images: FP64 path within 1e-12 of the oracle's largest pixel, FP32-mixed path (densities
rounded to FP32) within 1e-5.  On/off pixels: equal wherever the oracle's value is not
within that tolerance of the threshold.  Labels and count: a function of the on pixels
alone, so bit-exact against the oracle's labelling of the GPU's own on pixels, and equal to
the oracle's when no pixel is that close to the threshold.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import vortex as V
from paper_2405_03980_amd import _lib as L
from paper_2405_03980_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, MIXED = L.FP64, L.FP32_MIXED
TOL = {FP64: 1e-12, MIXED: 1e-5}


def _cylinder(nz, seed):
    w = I.make_cylinder(nz, seed=(3980, seed))
    rng = np.random.default_rng(seed)
    w.omega = w.omega + rng.normal(0.0, 1.0, size=w.omega.shape) * (w.kind == I.FLUID)
    return w


def _sim(w, prec):
    from paper_2405_03980_amd import sim as S
    return S.simulation_from(w, precision=prec)


def _compare(got, ref_img, ref_lab, ref_count, theta, min_pixels, tol):
    cnt, img, lab = got
    vmax = ref_img.max()
    assert vmax > 0
    assert np.abs(img - ref_img).max() <= tol * vmax, np.abs(img - ref_img).max() / vmax
    on = lab >= 0
    clear = np.abs(ref_img - theta * vmax) > 2 * tol * vmax
    assert np.array_equal(on[clear], V.threshold(ref_img, theta)[clear])
    assert np.array_equal(lab, V.components(on))
    assert cnt == V.count(lab, min_pixels)
    if clear.all():
        assert cnt == ref_count and np.array_equal(lab, ref_lab)
    return cnt


@pytest.mark.parametrize("prec", [FP64, MIXED])
@pytest.mark.parametrize("z0,theta,min_pixels", [(0.0, 0.5, 2), (0.37, 0.3, 4), (-2.63, 0.4, 2)])
def test_vortex_image_matches_oracle(prec, z0, theta, min_pixels):
    w = _cylinder(24, 5)
    print(f"[vortex] prec={prec} z0={z0} theta={theta} n={w.n}", flush=True)
    s = _sim(w, prec)
    got = s.vortex_image(z0, theta, min_pixels)
    s.close()
    rho, _, _ = O.density(w.params, w.x, w.species, w.kind)
    oc, oimg, olab = V.vortex_image(w.params, w.x, w.omega, w.species, w.kind, rho, z0, theta,
                                    min_pixels)
    cnt = _compare(got, oimg, olab, oc, theta, min_pixels, TOL[prec])
    print("components", cnt, "oracle", oc, flush=True)
    assert cnt > 0


def test_vortex_image_after_steps():
    """After steps with rotating walls: the FP64 path's state follows the oracle's."""
    w = _cylinder(20, 6)
    s = _sim(w, FP64)
    s.step(1e-4, w.Omega, 6)
    got = s.vortex_image(0.0, 0.4, 3)
    s.close()
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 6)
    oc, oimg, olab = V.vortex_image(w.params, ref.x, ref.omega, w.species, w.kind, ref.rho, 0.0,
                                    0.4, 3)
    _compare(got, oimg, olab, oc, 0.4, 3, 1e-11)


@pytest.mark.parametrize("sweep", [3, 1])
def test_mixed_vortex_image_after_steps(sweep):
    """FP32-mixed after steps with rotating walls: the brick intensity (sweep 3, replaying
    the density sweep's masks of the stepped positions) and the per-particle one (sweep 1)
    against the oracle's state, within 1e-5."""
    from paper_2405_03980_amd import sim as S
    w = _cylinder(20, 9)
    s = S.Simulation(w.params, w.n, precision=MIXED)
    s.set_tuning(sweep=sweep)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    s.step(1e-4, w.Omega, 4)
    got = s.vortex_image(0.2, 0.4, 2)
    s.close()
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 4)
    oc, oimg, olab = V.vortex_image(w.params, ref.x, ref.omega, w.species, w.kind, ref.rho, 0.2,
                                    0.4, 2)
    _compare(got, oimg, olab, oc, 0.4, 2, 1e-5)


def test_vortex_image_after_a_sweep_change():
    """Stepping with the brick sweeps, then switching to the per-particle ones and stepping
    again: the image follows the oracle (the stored masks, now of older positions, are not
    replayed)."""
    from paper_2405_03980_amd import sim as S
    w = _cylinder(18, 10)
    s = S.Simulation(w.params, w.n, precision=MIXED)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    s.step(1e-4, w.Omega, 2)
    s.set_tuning(sweep=1)
    s.step(1e-4, w.Omega, 1)
    got = s.vortex_image(0.0, 0.5, 1)
    s.close()
    ref = O.State.from_workload(w)
    ref.step(1e-4, w.Omega, 3)
    oc, oimg, olab = V.vortex_image(w.params, ref.x, ref.omega, w.species, w.kind, ref.rho, 0.0,
                                    0.5, 1)
    _compare(got, oimg, olab, oc, 0.5, 1, 1e-5)


def test_vortex_image_is_reproducible():
    w = _cylinder(20, 7)
    s = _sim(w, MIXED)
    a = s.vortex_image(0.1, 0.5, 1)
    b = s.vortex_image(0.1, 0.5, 1)
    s.close()
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_vortex_image_argument_errors():
    from paper_2405_03980_amd import sim as S
    w = _cylinder(10, 8)
    s = S.Simulation(w.params, w.n, precision=MIXED)
    with pytest.raises(L.SphError) as e:
        s.vortex_image()
    assert e.value.status == L.E_STATE
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    for kw in (dict(theta=-0.1), dict(min_pixels=0), dict(theta=float("nan")),
               dict(z0=float("inf"))):
        with pytest.raises(L.SphError) as e:
            s.vortex_image(**kw)
        assert e.value.status == L.E_INVALID, kw
    s.close()
