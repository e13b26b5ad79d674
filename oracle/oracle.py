"""ctypes wrapper of the FP64 CPU oracle (oracle/sph_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  The oracle defines its own parameter
struct; it shares no header or helper with the HIP library.

Arrays follow the input-generator conventions: x, v, omega float64 [3, n] (SoA),
species / kind uint8 [n], everything indexed by particle id.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, E_INVALID, E_DOMAIN, E_NONFINITE = 0, 1, 5, 6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32), ("geometry", C.c_int32), ("cell_factor", C.c_int32),
        ("pad", C.c_int32),
        ("dx", C.c_double), ("h", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double),
        ("mass", C.c_double * 2),
        ("eta", C.c_double), ("sigma_T", C.c_double), ("C_l", C.c_double),
        ("kappa_I", C.c_double),
        ("pressure_filter", C.c_int32), ("pad2", C.c_int32),
        ("coll_alpha", C.c_double), ("coll_e", C.c_double),
    ]


def params_from(d: dict) -> Params:
    p = Params()
    p.kernel, p.geometry, p.cell_factor = int(d["kernel"]), int(d["geometry"]), int(d.get("cell_factor", 1))
    p.dx, p.h = d["dx"], d["h"]
    for a in range(3):
        p.lo[a], p.hi[a] = d["lo"][a], d["hi"][a]
    p.rho0, p.c0, p.gamma = d["rho0"], d["c0"], d["gamma"]
    p.mass[0], p.mass[1] = d["mass"][0], d["mass"][1]
    p.eta, p.sigma_T, p.C_l, p.kappa_I = d["eta"], d["sigma_T"], d["C_l"], d["kappa_I"]
    p.pressure_filter = int(d.get("pressure_filter", 0))
    p.coll_alpha, p.coll_e = float(d.get("coll_alpha", 0.0)), float(d.get("coll_e", 0.0))
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(Params)
        L.or_W.restype = C.c_double
        L.or_W.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_dWdr.restype = C.c_double
        L.or_dWdr.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_lambda.restype = C.c_double
        L.or_lambda.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_neighbors.restype = C.c_int64
        L.or_num_threads.restype = C.c_int
        for name in ("or_cells", "or_density", "or_forces", "or_evaluate", "or_step",
                     "or_diagnostics", "or_default_mass", "or_grid_dims", "or_eval_subset",
                     "or_rot_intensity", "or_pressure_filter", "or_collide"):
            getattr(L, name).restype = C.c_int
        _ = (dp, pp)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def W(kernel: int, h: float, r: float) -> float:
    return lib().or_W(kernel, h, r)


def dWdr(kernel: int, h: float, r: float) -> float:
    return lib().or_dWdr(kernel, h, r)


def lattice_lambda(kernel: int, h: float, dx: float) -> float:
    return lib().or_lambda(kernel, h, dx)


def default_mass(params: dict) -> np.ndarray:
    out = np.zeros(2)
    p = params_from(params)
    _check(lib().or_default_mass(C.byref(p), _p(out)))
    return out


def grid_dims(params: dict):
    n = np.zeros(3, np.int32)
    e = np.zeros(3)
    p = params_from(params)
    _check(lib().or_grid_dims(C.byref(p), _p(n), _p(e)))
    return n, e


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def _check(st):
    if st != OK:
        raise OracleError(st)


def cells(params: dict, x: np.ndarray):
    """(key_by_id u32[n], perm u32[n], cell_start u32[ncell+1]) in Morton cell order."""
    x = _c(x, np.float64)
    n = x.shape[1]
    dims, _ = grid_dims(params)
    ncell = int(np.prod(dims.astype(np.int64)))
    key = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    cs = np.zeros(ncell + 1, np.uint32)
    nc = C.c_int64(0)
    p = params_from(params)
    _check(lib().or_cells(C.byref(p), C.c_int64(n), _p(x), _p(key), _p(perm), _p(cs), C.byref(nc)))
    return key, perm, cs


def neighbors(params: dict, x: np.ndarray, brute: bool = False, cap: int | None = None):
    """Neighbour CSR by id: (row_ptr int64[n+1], cols int32[nnz]) with ascending cols."""
    x = _c(x, np.float64)
    n = x.shape[1]
    cap = cap if cap is not None else max(1, 200 * n)
    row = np.zeros(n + 1, np.int64)
    cols = np.zeros(cap, np.int32)
    p = params_from(params)
    tot = lib().or_neighbors(C.byref(p), C.c_int64(n), _p(x), C.c_int(int(brute)), _p(row), _p(cols), C.c_int64(cap))
    if tot == -1:
        return neighbors(params, x, brute, cap=int(row[-1]) + 1)
    if tot < 0:
        raise OracleError(int(-tot - 100))
    return row, cols[:tot].copy()


class State:
    """Particle state held by id, advanced by the oracle."""

    def __init__(self, params: dict, x, v, omega, species, kind, brute: bool = False):
        self.params = dict(params)
        self.p = params_from(params)
        self.x = _c(x, np.float64).copy()
        self.v = _c(v, np.float64).copy()
        self.omega = _c(omega, np.float64).copy()
        self.species = _c(species, np.uint8).copy()
        self.kind = _c(kind, np.uint8).copy()
        self.n = self.x.shape[1]
        n = self.n
        for name, a in (("x", self.x), ("v", self.v), ("omega", self.omega)):
            if a.shape != (3, n):
                raise ValueError(f"{name} must be [3, {n}], got {a.shape}")
        if self.species.shape != (n,) or self.kind.shape != (n,):
            raise ValueError("species and kind must have n entries")
        self.rho = np.zeros(n)
        self.P = np.zeros(n)
        self.S = np.zeros(n)
        self.acc = np.zeros((3, n))
        self.alpha = np.zeros((3, n))
        self.brute = int(brute)
        self.evaluate()

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.params, w.x, w.v, w.omega, w.species, w.kind, **kw)

    def evaluate(self):
        _check(lib().or_evaluate(C.byref(self.p), C.c_int64(self.n), _p(self.x), _p(self.v),
                                 _p(self.omega), _p(self.species), _p(self.kind),
                                 C.c_int(self.brute), _p(self.rho), _p(self.P), _p(self.S),
                                 _p(self.acc), _p(self.alpha)))

    def step(self, dt: float, Omega: float = 0.0, nsteps: int = 1):
        _check(lib().or_step(C.byref(self.p), C.c_int64(self.n), _p(self.x), _p(self.v),
                             _p(self.omega), _p(self.species), _p(self.kind), _p(self.rho),
                             _p(self.P), _p(self.S), _p(self.acc), _p(self.alpha),
                             C.c_double(dt), C.c_double(Omega), C.c_int32(nsteps),
                             C.c_int(self.brute)))

    def diagnostics(self):
        out = np.zeros(7)
        _check(lib().or_diagnostics(C.byref(self.p), C.c_int64(self.n), _p(self.x), _p(self.v),
                                    _p(self.omega), _p(self.species), _p(self.kind), _p(out)))
        return out[:3].copy(), out[3:6].copy(), float(out[6])


def density(params, x, species, kind, brute=False):
    x = _c(x, np.float64)
    n = x.shape[1]
    rho, P, S = np.zeros(n), np.zeros(n), np.zeros(n)
    p = params_from(params)
    _check(lib().or_density(C.byref(p), C.c_int64(n), _p(x), _p(_c(species, np.uint8)),
                            _p(_c(kind, np.uint8)), C.c_int(int(brute)), _p(rho), _p(P), _p(S)))
    return rho, P, S


def forces(params, x, v, omega, species, kind, rho, P, S, brute=False):
    """Accelerations from given (possibly injected) rho, P, S fields."""
    x = _c(x, np.float64)
    n = x.shape[1]
    acc, alpha = np.zeros((3, n)), np.zeros((3, n))
    p = params_from(params)
    _check(lib().or_forces(C.byref(p), C.c_int64(n), _p(x), _p(_c(v, np.float64)),
                           _p(_c(omega, np.float64)), _p(_c(species, np.uint8)),
                           _p(_c(kind, np.uint8)), _p(_c(rho, np.float64)), _p(_c(P, np.float64)),
                           _p(_c(S, np.float64)), C.c_int(int(brute)), _p(acc), _p(alpha)))
    return acc, alpha


def pressure_filter(params, x, species, kind, rho, P, brute=False):
    """Filtered pressure from given rho and P fields (Shepard average over the particle
    and its fluid and inner-wall neighbours; outer walls keep theirs)."""
    x = _c(x, np.float64)
    n = x.shape[1]
    out = np.zeros(n)
    p = params_from(params)
    _check(lib().or_pressure_filter(C.byref(p), C.c_int64(n), _p(x), _p(_c(species, np.uint8)),
                                    _p(_c(kind, np.uint8)), _p(_c(rho, np.float64)),
                                    _p(_c(P, np.float64)), C.c_int(int(brute)), _p(out)))
    return out


def collide(params, x, v, species, kind, brute=False):
    """Velocities after the collision step (pairs closer than coll_alpha dx that approach
    each other leave with restitution coll_e; walls are unchanged)."""
    x = _c(x, np.float64)
    n = x.shape[1]
    out = np.zeros((3, n))
    p = params_from(params)
    _check(lib().or_collide(C.byref(p), C.c_int64(n), _p(x), _p(_c(v, np.float64)),
                            _p(_c(species, np.uint8)), _p(_c(kind, np.uint8)),
                            C.c_int(int(brute)), _p(out)))
    return out


def eval_subset(params, x, v, omega, species, kind, idx):
    """rho, P, S, acc [3,k], alpha [3,k] of particles idx, evaluated from the full state."""
    x = _c(x, np.float64)
    n = x.shape[1]
    idx = _c(idx, np.int64)
    k = idx.shape[0]
    rho, P, S = np.zeros(k), np.zeros(k), np.zeros(k)
    acc, alpha = np.zeros((3, k)), np.zeros((3, k))
    p = params_from(params)
    _check(lib().or_eval_subset(C.byref(p), C.c_int64(n), _p(x), _p(_c(v, np.float64)),
                                _p(_c(omega, np.float64)), _p(_c(species, np.uint8)),
                                _p(_c(kind, np.uint8)), C.c_int64(k), _p(idx), _p(rho), _p(P),
                                _p(S), _p(acc), _p(alpha)))
    return rho, P, S, acc, alpha


def rot_intensity(params, x, omega, species, kind, rho, mask=None):
    """Rotational-force intensity |2 eta sum_j V_j F_ij (w_i + w_j) x r_ij| over the viscous
    neighbours of every fluid particle (Eq. 2, fifth term; 0 for other particles).  With a
    boolean mask only those particles are evaluated (rho is read for their neighbours)."""
    x = _c(x, np.float64)
    n = x.shape[1]
    out = np.zeros(n)
    p = params_from(params)
    m = _c(mask, np.uint8) if mask is not None else None
    _check(lib().or_rot_intensity(C.byref(p), C.c_int64(n), _p(x), _p(_c(omega, np.float64)),
                                  _p(_c(species, np.uint8)), _p(_c(kind, np.uint8)),
                                  _p(_c(rho, np.float64)), _p(m) if m is not None else None,
                                  _p(out)))
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())
