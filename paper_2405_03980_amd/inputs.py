"""Seeded synthetic inputs for the two-fluid SPH step (shared by the HIP path and the oracle).

This module only lays particles out and draws random numbers: it holds none of the
method's arithmetic (no kernel, no density, no force, no mass normalisation).  Both the
HIP library and the FP64 oracle receive exactly the arrays built here.

Workloads follow the paper's rotating-cylinder setup (Sec. 3): fluid particles on a cubic
lattice inside a cylinder, a no-slip wall layer of normal-fluid particles along the inner
circumference, a forced rotation about the z axis, slip (here: periodic) top and bottom,
and inviscid/viscous labels drawn at random in proportion to the density ratio.  Sizes are
non-dimensional (R = H = 1); the paper's physical units need property tables it does not
reproduce, so only the shapes, counts and ratios are kept.

Array conventions (all numpy, C-contiguous):
  x, v, omega : float64 [3, n]   (SoA: row a holds component a of every particle)
  species     : uint8 [n]        0 = inviscid (S), 1 = viscous (N); walls are 1
  kind        : uint8 [n]        0 = fluid, 1 = inner wall layer, 2 = outer wall layers
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KERNEL_CUBIC = 0
KERNEL_WENDLAND_C2 = 1

GEOM_PERIODIC_BOX = 0
GEOM_CYLINDER_Z = 1
GEOM_OPEN = 2

FLUID, WALL_INNER, WALL_OUTER = 0, 1, 2
INVISCID, VISCOUS = 0, 1


@dataclass
class Workload:
    """Particles plus the coefficients of one SPH instance."""
    name: str
    params: dict
    x: np.ndarray
    v: np.ndarray
    omega: np.ndarray
    species: np.ndarray
    kind: np.ndarray
    dt: float = 1e-4
    steps: int = 20
    Omega: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.species.shape[0])

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.kind == FLUID))


def base_params(kernel: int, geometry: int, dx: float, lo, hi, c0: float,
                *, h_factor: float = 1.3, rho0: float = 1.0, nu: float = 1.0 / 88.6,
                sigma_frac: float = 0.05, C_l: float = 0.01, kappa_I: float = 0.4,
                cell_factor: int = 1, pressure_filter: int = 0, coll_alpha: float = 0.0,
                coll_e: float = 0.0) -> dict:
    """Coefficient set of the synthetic workloads.

    nu = 1/88.6 is the non-dimensional kinematic viscosity matching the paper's
    rotation Reynolds number (Sec. 3: eta_n = 0.566 kappa rho_n, Omega = 5 rad/s,
    R = 0.1 cm); the interfacial coefficient is a fixed fraction of the Tait
    stiffness rho0 c0^2 / 7 and the mutual-friction coefficient a small constant.
    pressure_filter, coll_alpha and coll_e switch on Algorithm 1's pressure filter and
    collision step (off by default, as in the benchmarked step).
    """
    gamma = 7.0
    return dict(
        kernel=int(kernel), geometry=int(geometry), dx=float(dx), h=float(h_factor * dx),
        lo=[float(a) for a in lo], hi=[float(a) for a in hi],
        rho0=float(rho0), c0=float(c0), gamma=gamma, mass=[0.0, 0.0],
        eta=float(nu * rho0), sigma_T=float(sigma_frac * rho0 * c0 * c0 / gamma),
        C_l=float(C_l * rho0), kappa_I=float(kappa_I), cell_factor=int(cell_factor),
        pressure_filter=int(pressure_filter), coll_alpha=float(coll_alpha), coll_e=float(coll_e),
    )


def _assign_species(rng: np.random.Generator, n_fluid: int, visc_frac: float) -> np.ndarray:
    sp = np.zeros(n_fluid, dtype=np.uint8)
    n_visc = int(round(visc_frac * n_fluid))
    perm = rng.permutation(n_fluid)
    sp[perm[:n_visc]] = VISCOUS
    return sp


def make_box(n_side: int = 16, *, seed=(3980, 0), kernel: int = KERNEL_CUBIC,
             visc_frac: float = 0.3, Omega: float = 1.0, noise: float = 1e-3,
             rigid: bool = True, geometry: int = GEOM_PERIODIC_BOX,
             h_factor: float = 1.3, cell_factor: int = 1) -> Workload:
    """Unit box with an n_side^3 cubic lattice at (i + 1/2) dx.

    rigid=True: rigid rotation Omega about the vertical line through (1/2, 1/2) plus
    N(0, noise) per component, spin omega = Omega z-hat (the 4,096-particle workload).
    """
    rng = np.random.default_rng(list(seed))
    dx = 1.0 / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).copy()
    n = x.shape[1]
    species = _assign_species(rng, n, visc_frac)
    v = np.zeros((3, n))
    omega = np.zeros((3, n))
    if rigid:
        v[0] = -Omega * (x[1] - 0.5)
        v[1] = Omega * (x[0] - 0.5)
        omega[2] = Omega
    v += rng.normal(0.0, noise, size=(3, n))
    c0 = 10.0 * float(np.max(np.sqrt((v * v).sum(axis=0))))
    if c0 == 0.0:
        c0 = 1.0
    params = base_params(kernel, geometry, dx, [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], c0,
                         h_factor=h_factor, cell_factor=cell_factor)
    kind = np.zeros(n, dtype=np.uint8)
    return Workload(f"box{n_side}", params, x, np.ascontiguousarray(v), omega,
                    species, kind, Omega=Omega)


def cylinder_lattice(nz: int, R: float = 1.0, H: float = 1.0, wall_layers: int = 3):
    """Lattice sites of a cylinder of radius R, height H with dx = H / nz.

    Returns (x [3,n], kind [n], dx).  Sites with r < R are kept; those with
    R - wall_layers*dx <= r are walls, the innermost wall layer being WALL_INNER.
    """
    dx = H / nz
    nxy = int(round(2.0 * R / dx))
    gxy = (np.arange(nxy, dtype=np.float64) + 0.5) * dx - R
    r2 = gxy[:, None] ** 2 + gxy[None, :] ** 2
    inside = r2 < R * R
    ii, jj = np.nonzero(inside)
    rr = np.sqrt(r2[ii, jj])
    kind2 = np.full(ii.shape[0], FLUID, dtype=np.uint8)
    kind2[rr >= R - wall_layers * dx] = WALL_OUTER
    kind2[(rr >= R - wall_layers * dx) & (rr < R - (wall_layers - 1) * dx)] = WALL_INNER
    gz = (np.arange(nz, dtype=np.float64) + 0.5) * dx
    m = ii.shape[0]
    x = np.empty((3, m * nz))
    x[0] = np.repeat(gxy[ii], nz)
    x[1] = np.repeat(gxy[jj], nz)
    x[2] = np.tile(gz, m)
    kind = np.repeat(kind2, nz)
    return x, kind, dx


def make_cylinder(nz: int, *, seed=(3980, 1), kernel: int = KERNEL_WENDLAND_C2,
                  visc_frac: float = 0.3, Omega: float = 1.0, noise: float = 1e-3,
                  R: float = 1.0, H: float = 1.0, h_factor: float = 1.3,
                  cell_factor: int = 1, name: str | None = None) -> Workload:
    """Rotating cylinder: fluid at rest plus N(0, noise), walls turning at Omega.

    z is periodic with period H (the paper's slip top/bottom, read as the inviscid fluid
    continuing).  c0 = 10 max|v| over all particles, walls included.
    """
    rng = np.random.default_rng(list(seed))
    x, kind, dx = cylinder_lattice(nz, R, H)
    n = x.shape[1]
    fluid = kind == FLUID
    nf = int(np.count_nonzero(fluid))
    species = np.ones(n, dtype=np.uint8)
    species[fluid] = _assign_species(rng, nf, visc_frac)
    v = np.zeros((3, n))
    omega = np.zeros((3, n))
    v[:, fluid] = rng.normal(0.0, noise, size=(3, nf))
    wall = ~fluid
    v[0, wall] = -Omega * x[1, wall]
    v[1, wall] = Omega * x[0, wall]
    omega[2, wall] = Omega
    c0 = 10.0 * float(np.max(np.sqrt((v * v).sum(axis=0))))
    params = base_params(kernel, GEOM_CYLINDER_Z, dx, [-R, -R, 0.0], [R, R, H], c0,
                         h_factor=h_factor, cell_factor=cell_factor)
    return Workload(name or f"cylinder_nz{nz}", params, x, v, omega, species, kind,
                    Omega=Omega, meta=dict(nz=nz, R=R, H=H))


def make_cluster(n_side: int = 8, *, seed=(3980, 9), kernel: int = KERNEL_WENDLAND_C2,
                 visc_frac: float = 0.5, noise: float = 1e-2, spin: float = 0.5,
                 jitter: float = 0.1, c0: float = 2.0, h_factor: float = 1.3) -> Workload:
    """A free, wall-free cluster in an open domain, for conservation checks.

    Jittered cubic lattice of n_side^3 particles in the middle of a box three times its
    size; random velocities and spins so that every pair term is active.  With
    h_factor = 2 the cells (edge 2h = 4 dx) hold 4^3 lattice points each, and a cluster of
    8^3 fills exactly the 2x2x2 cells of one brick.
    """
    rng = np.random.default_rng(list(seed))
    dx = 1.0 / (3 * n_side)
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * dx + 1.0 / 3.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).copy()
    n = x.shape[1]
    x += rng.uniform(-jitter, jitter, size=(3, n)) * dx
    species = _assign_species(rng, n, visc_frac)
    v = rng.normal(0.0, noise, size=(3, n))
    omega = rng.normal(0.0, spin, size=(3, n))
    params = base_params(kernel, GEOM_OPEN, dx, [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], c0,
                         h_factor=h_factor)
    kind = np.zeros(n, dtype=np.uint8)
    return Workload(f"cluster{n_side}", params, x, v, omega, species, kind)


def batch_sizes(n_inst: int = 64, seed=(3980, 4), lo: float = 20_000, hi: float = 300_000):
    """Per-instance cylinder resolutions of the batched ensemble.

    N_i is drawn log-uniform in [lo, hi]; the lattice is nz_i = max(19, round(cbrt(N_i/pi))),
    so realised counts are quantised.  Viscous fraction ~ U(0.05, 0.5), Omega ~ U(0.5, 2).
    """
    rng = np.random.default_rng(list(seed))
    N = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_inst))
    nz = np.maximum(19, np.round(np.cbrt(N / math.pi))).astype(int)
    vf = rng.uniform(0.05, 0.5, size=n_inst)
    Om = rng.uniform(0.5, 2.0, size=n_inst)
    return nz, vf, Om


def make_batch(n_inst: int = 64, *, scale: float = 1.0) -> list[Workload]:
    """The ensemble of independent cylinders (instance i seeded with (3980, 4, i)).

    scale < 1 shrinks every instance's particle count (for tests), keeping the recipe.
    """
    nz, vf, Om = batch_sizes(n_inst)
    out = []
    for i in range(n_inst):
        nzi = int(nz[i])
        if scale != 1.0:
            nzi = max(8, int(round(nzi * scale ** (1.0 / 3.0))))
        w = make_cylinder(nzi, seed=(3980, 4, i), visc_frac=float(vf[i]), Omega=float(Om[i]),
                          name=f"inst{i}_nz{nzi}")
        out.append(w)
    return out


# The five named workloads ----------------------------------------------------------------

def config(idx: int) -> Workload:
    """Workload idx of the measurement plan (0: 4,096-particle periodic box, cubic kernel;
    1/2: 2.45M cylinder nz=92, Wendland C2; 3: 19.57M cylinder nz=184)."""
    if idx == 0:
        w = make_box(16, seed=(3980, 0))
        w.steps, w.dt, w.name = 20, 1e-4, "box4096_cubic"
        return w
    if idx in (1, 2):
        w = make_cylinder(92, seed=(3980, 1))
        w.steps, w.dt, w.name = 100, 1e-4, "cylinder_2.45M"
        return w
    if idx == 3:
        w = make_cylinder(184, seed=(3980, 3))
        w.steps, w.dt, w.name = 100, 1e-4, "cylinder_19.57M"
        return w
    raise ValueError(idx)
