"""sph_vortex_image_noalloc (no device allocation; scratch in the library's static device
array) against sph_vortex_image (caller scratch), through the C ABI: identical image,
labels and count on two calls in a row, the second on a smaller image; images beyond the
array's 2^20 pixels are refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2405_03980_amd import _lib as L
from paper_2405_03980_amd import inputs as I

pytestmark = pytest.mark.gpu


def _spun(nz, seed):
    """A cylinder with random spins so that the image has structure."""
    from paper_2405_03980_amd import sim as S
    w = I.make_cylinder(nz, seed=(3980, seed))
    rng = np.random.default_rng(seed)
    f = w.kind == I.FLUID
    w.omega[:, f] = rng.normal(0, 2.0, size=(3, int(f.sum())))
    w.params = dict(w.params, eta=0.05)
    s = S.Simulation(w.params, w.n, precision=L.FP32_MIXED)
    s.init(w.x, w.v, w.omega, w.species, w.kind)
    s.step(1e-4, w.Omega, 2)
    return s


def _both(s, z0=0.0, theta=0.3, min_pixels=2):
    lib = L.lib()
    nx, ny = C.c_int32(), C.c_int32()
    assert lib.sph_vortex_dims(C.byref(s.params), C.byref(nx), C.byref(ny)) == L.OK
    nx, ny = nx.value, ny.value
    with torch.cuda.stream(s.stream):
        img_a = torch.full((ny, nx), -1.0, dtype=torch.float64, device=s.device)
        lab_a = torch.full((ny, nx), -7, dtype=torch.int32, device=s.device)
        scr = torch.empty(nx * ny + 8, dtype=torch.int32, device=s.device)
        img_b = torch.full((ny, nx), -1.0, dtype=torch.float64, device=s.device)
        lab_b = torch.full((ny, nx), -7, dtype=torch.int32, device=s.device)
    ca, cb = C.c_int32(-1), C.c_int32(-1)
    st = lib.sph_vortex_image(s._h, C.c_double(z0), C.c_double(theta), C.c_int32(min_pixels),
                              C.c_void_p(img_a.data_ptr()), C.c_void_p(lab_a.data_ptr()),
                              C.c_void_p(scr.data_ptr()), C.byref(ca))
    assert st == L.OK, lib.sph_last_error(s._h)
    st = lib.sph_vortex_image_noalloc(s._h, C.c_double(z0), C.c_double(theta),
                                      C.c_int32(min_pixels), C.c_void_p(img_b.data_ptr()),
                                      C.c_void_p(lab_b.data_ptr()), C.byref(cb))
    assert st == L.OK, lib.sph_last_error(s._h)
    return (ca.value, img_a.cpu().numpy(), lab_a.cpu().numpy()), (cb.value, img_b.cpu().numpy(),
                                                                  lab_b.cpu().numpy())


def test_noalloc_equals_caller_scratch():
    for nz, seed in ((26, 11), (14, 12)):  # the second image is smaller
        print(f"[noalloc] nz={nz}", flush=True)
        s = _spun(nz, seed)
        (ca, ia, la), (cb, ib, lb) = _both(s)
        assert ca == cb and ca >= 1
        assert np.array_equal(ia, ib)
        assert np.array_equal(la, lb)
        assert (la >= 0).sum() > 0 and ia.max() > 0
        # a second no-alloc call on the same state sees a cleared array again
        (ca2, ia2, la2), (cb2, ib2, lb2) = _both(s, theta=0.6, min_pixels=1)
        assert ca2 == cb2 and np.array_equal(ib2, ia2) and np.array_equal(lb2, la2)
        s.close()


def test_noalloc_refuses_large_images():
    """A thin slab with dx = 1/600 has 1200 x 1200 pixels > 2^20: SPH_E_CAPACITY, nothing
    enqueued (the caller's buffers keep their contents)."""
    from paper_2405_03980_amd import sim as S
    dx = 1.0 / 600
    H = 4 * 2.6 * dx
    p = I.base_params(I.KERNEL_WENDLAND_C2, I.GEOM_CYLINDER_Z, dx, [-1, -1, 0], [1, 1, H], 1.0)
    n = 8
    x = np.stack([np.arange(n) * 1.5 * dx, np.zeros(n), np.full(n, 0.5 * H)])
    s = S.Simulation(p, n, precision=L.FP32_MIXED)
    s.init(x, np.zeros((3, n)), np.zeros((3, n)), np.zeros(n, np.uint8), np.zeros(n, np.uint8))
    s.sync()
    nx, ny = C.c_int32(), C.c_int32()
    assert L.lib().sph_vortex_dims(C.byref(s.params), C.byref(nx), C.byref(ny)) == L.OK
    assert nx.value * ny.value > (1 << 20)
    # full-size buffers, so that the call could not write out of bounds even if it ran
    with torch.cuda.stream(s.stream):
        img = torch.full((ny.value, nx.value), 3.0, dtype=torch.float64, device=s.device)
        lab = torch.full((ny.value, nx.value), 5, dtype=torch.int32, device=s.device)
    cnt = C.c_int32(-3)
    st = L.lib().sph_vortex_image_noalloc(s._h, C.c_double(0.0), C.c_double(0.5), C.c_int32(1),
                                          C.c_void_p(img.data_ptr()), C.c_void_p(lab.data_ptr()),
                                          C.byref(cnt))
    assert st == L.E_CAPACITY
    assert b"2^20" in L.lib().sph_last_error(s._h)
    s.stream.synchronize()
    assert cnt.value == -3
    assert bool((img == 3.0).all()) and bool((lab == 5).all())
    s.close()
