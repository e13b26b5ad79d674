"""Vortex image and count of the z = z0 section (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the tests and the benchmark's check
call it, the product path never does.

The paper counts spinning vortices by image analysis of the rotational-force intensity
(the fifth term of Eq. 2) on the z = 0 section (Sec. 3 and its figure of the image
analysis), with an external image tool whose settings it does not give.  This is the
reading used on both sides, written out step by step:
  1. intensity I_i of every fluid particle (oracle.rot_intensity);
  2. the section: fluid particles with -dx <= dz < dx, dz = z - z0 wrapped into
     [-L_z/2, L_z/2) (z is periodic in both geometries): two lattice layers, whose
     particles sit well inside the section on the initial lattice (at dz = +-dx/2);
  3. the image: square pixels of side dx over the x-y extent of the domain,
     nx = ceil((hi - lo) / dx - 1e-9); a particle falls in pixel floor((x - lo) / dx)
     (clamped to the grid); a pixel holds the largest intensity among its particles,
     0 if it has none;
  4. threshold: a pixel is on when its value is positive and at least theta times the
     largest pixel value;
  5. components: 8-connected sets of on pixels (no wrap at the image edges), each
     labelled by its smallest pixel index iy * nx + ix; off pixels get -1;
  6. count: the components with at least min_pixels pixels.
All arithmetic is IEEE double without fused operations.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

from . import oracle as O

FLUID = 0


def image_dims(params: dict):
    dx = float(params["dx"])
    lo, hi = params["lo"], params["hi"]
    nx = int(math.ceil((hi[0] - lo[0]) / dx - 1e-9))
    ny = int(math.ceil((hi[1] - lo[1]) / dx - 1e-9))
    return nx, ny


def section_mask(params: dict, x: np.ndarray, kind: np.ndarray, z0: float) -> np.ndarray:
    dx = float(params["dx"])
    Lz = float(params["hi"][2] - params["lo"][2])
    dz = x[2] - z0
    dz = dz - Lz * np.floor(dz / Lz + 0.5)   # separately rounded products and sums
    return (np.asarray(kind) == FLUID) & (-dx <= dz) & (dz < dx)


def plane_image(params: dict, x: np.ndarray, kind: np.ndarray, intensity: np.ndarray, z0: float):
    nx, ny = image_dims(params)
    dx = float(params["dx"])
    lo = params["lo"]
    img = np.zeros((ny, nx))
    sel = section_mask(params, x, kind, z0)
    ix = np.clip(np.floor((x[0, sel] - lo[0]) / dx).astype(np.int64), 0, nx - 1)
    iy = np.clip(np.floor((x[1, sel] - lo[1]) / dx).astype(np.int64), 0, ny - 1)
    np.maximum.at(img, (iy, ix), intensity[sel])
    return img


def threshold(img: np.ndarray, theta: float) -> np.ndarray:
    vmax = float(img.max()) if img.size else 0.0
    return (img > 0.0) & (img >= theta * vmax)


def components(on: np.ndarray) -> np.ndarray:
    """8-connected labelling by breadth-first flood fill; label = smallest pixel index."""
    ny, nx = on.shape
    lab = np.full((ny, nx), -1, dtype=np.int64)
    for iy in range(ny):
        for ix in range(nx):
            if not on[iy, ix] or lab[iy, ix] >= 0:
                continue
            # scanning in index order, the first pixel met is the component's smallest
            root = iy * nx + ix
            lab[iy, ix] = root
            q = deque([(iy, ix)])
            while q:
                y, x_ = q.popleft()
                for dy in (-1, 0, 1):
                    for dxp in (-1, 0, 1):
                        yy, xx = y + dy, x_ + dxp
                        if 0 <= yy < ny and 0 <= xx < nx and on[yy, xx] and lab[yy, xx] < 0:
                            lab[yy, xx] = root
                            q.append((yy, xx))
    return lab


def count(labels: np.ndarray, min_pixels: int) -> int:
    roots, sizes = np.unique(labels[labels >= 0], return_counts=True)
    return int(np.sum(sizes >= min_pixels))


def vortex_image(params, x, omega, species, kind, rho, z0=0.0, theta=0.5, min_pixels=4):
    """(count, image [ny, nx], labels [ny, nx]) of the section z = z0."""
    sel = section_mask(params, x, kind, z0)
    inten = O.rot_intensity(params, x, omega, species, kind, rho, mask=sel)
    img = plane_image(params, x, kind, inten, z0)
    lab = components(threshold(img, theta))
    return count(lab, min_pixels), img, lab
