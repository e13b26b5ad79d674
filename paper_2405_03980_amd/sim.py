"""Python handles over the C ABI: torch supplies device memory and the stream, the HIP
library does every step of the computation.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

FIELDS = ("x", "v", "omega", "rho", "P", "acc", "alpha")


def _dev(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _aligned_workspace(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


def _check(st: int, where: str, err_fn=None):
    if st != L.OK:
        detail = ""
        if err_fn is not None:
            raw = err_fn()
            detail = raw.decode() if raw else ""
        raise L.SphError(st, where, detail)


class Simulation:
    """One SPH instance.

    params: dict of coefficients (see inputs.base_params); precision: L.FP64 or
    L.FP32_MIXED.  A dedicated non-default stream is used so that steps can be replayed
    from a captured hipGraph.
    """

    def __init__(self, params: dict, n: int, precision: int = L.FP32_MIXED, device="cuda:0",
                 stream: torch.cuda.Stream | None = None):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.n = int(n)
        self.params = L.make_params(params, precision)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nb = C.c_size_t(0)
        _check(self.lib.sph_workspace_bytes(C.byref(self.params), C.c_int64(self.n), C.byref(nb)),
               "sph_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        with torch.cuda.stream(self.stream):
            self._ws, ptr = _aligned_workspace(self.workspace_bytes, self.device)
        self._h = C.c_void_p()
        _check(self.lib.sph_create(C.byref(self.params), C.c_int64(self.n), C.c_void_p(ptr),
                                   C.c_size_t(self.workspace_bytes),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
               "sph_create")
        self._inputs = None

    # -- helpers
    def _err(self):
        return self.lib.sph_last_error(self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            self.lib.sph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API
    def init(self, x, v, omega, species, kind):
        with torch.cuda.stream(self.stream):
            xs = _dev(x, torch.float64, self.device)
            vs = _dev(v, torch.float64, self.device)
            ws = _dev(omega, torch.float64, self.device)
            sp = _dev(species, torch.uint8, self.device)
            kd = _dev(kind, torch.uint8, self.device)
        for t in (xs, vs, ws):
            if tuple(t.shape) != (3, self.n):
                raise ValueError(f"expected [3, {self.n}] arrays, got {tuple(t.shape)}")
        if sp.numel() != self.n or kd.numel() != self.n:
            raise ValueError("species/kind must have n entries")
        self._inputs = (xs, vs, ws, sp, kd)  # alive until the enqueued load has run
        _check(self.lib.sph_init_particles(self._h, xs.data_ptr(), vs.data_ptr(), ws.data_ptr(),
                                           sp.data_ptr(), kd.data_ptr()), "sph_init_particles", self._err)
        return self

    def step(self, dt: float, Omega: float = 0.0, nsteps: int = 1):
        _check(self.lib.sph_step(self._h, C.c_double(dt), C.c_double(Omega), C.c_int32(nsteps)),
               "sph_step", self._err)

    def sync(self):
        _check(self.lib.sph_sync(self._h), "sph_sync", self._err)
        self._inputs = None

    def read(self, fields=FIELDS, to_numpy: bool = True) -> dict:
        out = {}
        with torch.cuda.stream(self.stream):
            for f in fields:
                shape = (self.n,) if f in ("rho", "P") else (3, self.n)
                out[f] = torch.empty(shape, dtype=torch.float64, device=self.device)
        ptrs = [out[f].data_ptr() if f in out else None for f in FIELDS]
        _check(self.lib.sph_read_fields(self._h, *ptrs), "sph_read_fields", self._err)
        self._inputs = None
        if to_numpy:
            return {k: t.cpu().numpy() for k, t in out.items()}
        return out

    def diagnostics(self):
        out = (C.c_double * 7)()
        _check(self.lib.sph_diagnostics(self._h, out), "sph_diagnostics", self._err)
        a = np.array(out[:])
        return a[:3], a[3:6], float(a[6])

    def debug_cells(self):
        dims = (C.c_int32 * 3)()
        _check(self.lib.sph_grid_dims(C.byref(self.params), dims), "sph_grid_dims")
        ncell = int(dims[0]) * int(dims[1]) * int(dims[2])
        with torch.cuda.stream(self.stream):
            key = torch.empty(self.n, dtype=torch.int32, device=self.device)
            perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
            cs = torch.empty(ncell + 1, dtype=torch.int32, device=self.device)
        _check(self.lib.sph_debug_cells(self._h, key.data_ptr(), perm.data_ptr(), cs.data_ptr()),
               "sph_debug_cells", self._err)
        self.sync()
        f = lambda t: t.cpu().numpy().view(np.uint32)
        return f(key), f(perm), f(cs)

    def debug_neighbors(self, cap: int | None = None):
        cap = cap if cap is not None else 200 * self.n
        with torch.cuda.stream(self.stream):
            row = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
            cols = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        nnz = C.c_int64(0)
        st = self.lib.sph_debug_neighbors(self._h, row.data_ptr(), cols.data_ptr(), C.c_int64(cap),
                                          C.byref(nnz))
        if st == L.E_CAPACITY and cap < nnz.value:
            return self.debug_neighbors(int(nnz.value))
        _check(st, "sph_debug_neighbors", self._err)
        return row.cpu().numpy(), cols[: nnz.value].cpu().numpy()

    def debug_masks(self, cap: int | None = None):
        """Neighbour CSR by id of the hit masks the FP32-mixed brick sweeps used."""
        cap = cap if cap is not None else 200 * self.n
        with torch.cuda.stream(self.stream):
            row = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
            cols = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        nnz = C.c_int64(0)
        st = self.lib.sph_debug_masks(self._h, row.data_ptr(), cols.data_ptr(), C.c_int64(cap),
                                      C.byref(nnz))
        if st == L.E_CAPACITY and cap < nnz.value:
            return self.debug_masks(int(nnz.value))
        _check(st, "sph_debug_masks", self._err)
        return row.cpu().numpy(), cols[: nnz.value].cpu().numpy()

    def debug_near(self):
        """(count uint8 [n], ids int32 [n, 6]) of the near lists of the collision step."""
        with torch.cuda.stream(self.stream):
            cnt = torch.empty(self.n, dtype=torch.uint8, device=self.device)
            ids = torch.empty((self.n, 6), dtype=torch.int32, device=self.device)
        _check(self.lib.sph_debug_near(self._h, cnt.data_ptr(), ids.data_ptr()), "sph_debug_near",
               self._err)
        return cnt.cpu().numpy(), ids.cpu().numpy()

    def vortex_image(self, z0: float = 0.0, theta: float = 0.5, min_pixels: int = 4,
                     to_numpy: bool = True):
        """(count, image [ny, nx], labels [ny, nx]) of the rotational-force intensity on the
        section z = z0 (sph_vortex_image)."""
        nx, ny = C.c_int32(), C.c_int32()
        _check(self.lib.sph_vortex_dims(C.byref(self.params), C.byref(nx), C.byref(ny)),
               "sph_vortex_dims")
        nx, ny = int(nx.value), int(ny.value)
        with torch.cuda.stream(self.stream):
            img = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
            lab = torch.empty((ny, nx), dtype=torch.int32, device=self.device)
            scratch = torch.empty(nx * ny + 8, dtype=torch.int32, device=self.device)
        cnt = C.c_int32()
        _check(self.lib.sph_vortex_image(self._h, C.c_double(z0), C.c_double(theta),
                                         C.c_int32(min_pixels), C.c_void_p(img.data_ptr()),
                                         C.c_void_p(lab.data_ptr()),
                                         C.c_void_p(scratch.data_ptr()), C.byref(cnt)),
               "sph_vortex_image", self._err)
        if to_numpy:
            return int(cnt.value), img.cpu().numpy(), lab.cpu().numpy()
        return int(cnt.value), img, lab

    def set_tuning(self, block_density=0, block_force=0, block_stream=0, use_graph=-1, sweep=0,
                   xcd_run=0, list_targets=0):
        t = L.SphTuning(block_density, block_force, block_stream, use_graph, sweep, xcd_run,
                        list_targets)
        _check(self.lib.sph_set_tuning(self._h, C.byref(t)), "sph_set_tuning", self._err)

    def profile_begin(self):
        _check(self.lib.sph_profile_begin(self._h), "profile_begin", self._err)

    def profile_end(self) -> tuple[dict, int]:
        """Summed milliseconds per kernel group over the profiled steps, and the step count."""
        ms = (C.c_double * len(L.KERNEL_GROUPS))()
        n = C.c_int32(0)
        _check(self.lib.sph_profile_end(self._h, ms, C.byref(n)), "profile_end", self._err)
        return dict(zip(L.KERNEL_GROUPS, ms[:])), int(n.value)

    def get_tuning(self) -> dict:
        t = L.SphTuning()
        _check(self.lib.sph_get_tuning(self._h, C.byref(t)), "sph_get_tuning", self._err)
        return dict(block_density=t.block_density, block_force=t.block_force,
                    block_stream=t.block_stream, use_graph=t.use_graph, sweep=t.sweep,
                    xcd_run=t.xcd_run, list_targets=t.list_targets)


class Batch:
    """An ensemble of independent instances advanced by shared kernel launches."""

    def __init__(self, params_list: list[dict], counts, precision: int = L.FP32_MIXED,
                 device="cuda:0", stream: torch.cuda.Stream | None = None):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.n_inst = len(params_list)
        self.counts = np.asarray(counts, dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)])
        self.N = int(self.offsets[-1])
        arr = (L.SphParams * self.n_inst)()
        for i, d in enumerate(params_list):
            arr[i] = L.make_params(d, precision)
        self.params = arr
        self._counts_c = (C.c_int64 * self.n_inst)(*[int(c) for c in self.counts])
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nb = C.c_size_t(0)
        _check(self.lib.sph_batch_workspace_bytes(self.n_inst, arr, self._counts_c, C.byref(nb)),
               "sph_batch_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        with torch.cuda.stream(self.stream):
            self._ws, ptr = _aligned_workspace(self.workspace_bytes, self.device)
        self._h = C.c_void_p()
        _check(self.lib.sph_batch_create(self.n_inst, arr, self._counts_c, C.c_void_p(ptr),
                                         C.c_size_t(self.workspace_bytes),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
               "sph_batch_create")
        self._inputs = None

    def _err(self):
        return self.lib.sph_batch_last_error(self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            self.lib.sph_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, x, v, omega, species, kind):
        with torch.cuda.stream(self.stream):
            t = [_dev(x, torch.float64, self.device), _dev(v, torch.float64, self.device),
                 _dev(omega, torch.float64, self.device), _dev(species, torch.uint8, self.device),
                 _dev(kind, torch.uint8, self.device)]
        for a in t[:3]:
            if tuple(a.shape) != (3, self.N):
                raise ValueError(f"expected [3, {self.N}] arrays")
        self._inputs = t
        _check(self.lib.sph_batch_init(self._h, *[a.data_ptr() for a in t]), "sph_batch_init", self._err)
        return self

    def step(self, dt: float, Omega, nsteps: int = 1):
        om = (C.c_double * self.n_inst)(*[float(o) for o in np.broadcast_to(Omega, (self.n_inst,))])
        _check(self.lib.sph_batch_step(self._h, C.c_double(dt), om, C.c_int32(nsteps)),
               "sph_batch_step", self._err)

    def sync(self):
        _check(self.lib.sph_batch_sync(self._h), "sph_batch_sync", self._err)
        self._inputs = None

    def read(self, fields=FIELDS, to_numpy: bool = True) -> dict:
        out = {}
        with torch.cuda.stream(self.stream):
            for f in fields:
                shape = (self.N,) if f in ("rho", "P") else (3, self.N)
                out[f] = torch.empty(shape, dtype=torch.float64, device=self.device)
        ptrs = [out[f].data_ptr() if f in out else None for f in FIELDS]
        _check(self.lib.sph_batch_read_fields(self._h, *ptrs), "sph_batch_read_fields", self._err)
        self._inputs = None
        if to_numpy:
            return {k: t.cpu().numpy() for k, t in out.items()}
        return out

    def diagnostics(self) -> np.ndarray:
        out = (C.c_double * (7 * self.n_inst))()
        _check(self.lib.sph_batch_diagnostics(self._h, out), "sph_batch_diagnostics", self._err)
        return np.array(out[:]).reshape(self.n_inst, 7)

    def set_tuning(self, block_density=0, block_force=0, block_stream=0, use_graph=-1, sweep=0,
                   xcd_run=0, list_targets=0):
        t = L.SphTuning(block_density, block_force, block_stream, use_graph, sweep, xcd_run,
                        list_targets)
        _check(self.lib.sph_batch_set_tuning(self._h, C.byref(t)), "sph_batch_set_tuning", self._err)

    def profile_begin(self):
        _check(self.lib.sph_batch_profile_begin(self._h), "profile_begin", self._err)

    def profile_end(self) -> tuple[dict, int]:
        """Summed milliseconds per kernel group over the profiled steps, and the step count."""
        ms = (C.c_double * len(L.KERNEL_GROUPS))()
        n = C.c_int32(0)
        _check(self.lib.sph_batch_profile_end(self._h, ms, C.byref(n)), "profile_end", self._err)
        return dict(zip(L.KERNEL_GROUPS, ms[:])), int(n.value)


def simulation_from(workload, precision: int = L.FP32_MIXED, device="cuda:0") -> Simulation:
    """Create and initialise a Simulation from an inputs.Workload."""
    s = Simulation(workload.params, workload.n, precision=precision, device=device)
    s.init(workload.x, workload.v, workload.omega, workload.species, workload.kind)
    return s


def batch_from(workloads, precision: int = L.FP32_MIXED, device="cuda:0") -> Batch:
    """Create and initialise a Batch from a list of inputs.Workload (concatenated)."""
    counts = [w.n for w in workloads]
    b = Batch([w.params for w in workloads], counts, precision=precision, device=device)
    x = np.concatenate([w.x for w in workloads], axis=1)
    v = np.concatenate([w.v for w in workloads], axis=1)
    om = np.concatenate([w.omega for w in workloads], axis=1)
    sp = np.concatenate([w.species for w in workloads])
    kd = np.concatenate([w.kind for w in workloads])
    b.init(x, v, om, sp, kd)
    return b
