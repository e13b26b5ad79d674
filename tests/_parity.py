"""Per-field error measures used by the GPU parity tests.

Normwise relative error over fluid particles: max_i |f_i - f_ref_i| / max_i |f_ref_i|
(vectors by Euclidean norm); positions as displacement from the initial state (periodic
axes by minimum image); pressure normalised by the Tait stiffness B.
"""
import numpy as np


def _norm(a):
    return np.sqrt((a * a).sum(axis=0)) if a.ndim == 2 else np.abs(a)


def min_image(d, params):
    d = d.copy()
    L = np.array(params["hi"]) - np.array(params["lo"])
    geom = params["geometry"]
    per = [geom == 0] * 3 if geom != 1 else [False, False, True]
    for a in range(3):
        if per[a]:
            d[a] = d[a] - L[a] * np.round(d[a] / L[a])
    return d


def positions_ok(e: dict, tol: float, steps: int) -> bool:
    """Displacement within tol, or positions within 2 ulps per step (rounding-limited:
    the drift x + dt v is rounded once per step, fused on the GPU, twice in the oracle)."""
    return e["x"] < tol or e["x_ulp"] <= 2 * max(steps, 1)


def field_errors(out: dict, ref, w, x0=None) -> dict:
    """out: fields read from the library; ref: oracle State (same particles, by id)."""
    f = w.kind == 0
    p = w.params
    B = p["rho0"] * p["c0"] ** 2 / 7.0
    e = {}
    if x0 is None:
        x0 = w.x
    disp_ref = min_image(ref.x - x0, p)[:, f]
    dx = min_image(out["x"] - ref.x, p)[:, f]
    e["x"] = float(_norm(dx).max() / max(_norm(disp_ref).max(), 1e-300))
    # the same difference in units of the coordinates' own spacing (ulp): positions cannot
    # agree better than their rounding, whatever the displacement
    e["x_ulp"] = float((np.abs(dx) / np.spacing(np.abs(ref.x[:, f]))).max())
    for k, r in (("v", ref.v), ("omega", ref.omega), ("acc", ref.acc), ("alpha", ref.alpha),
                 ("rho", ref.rho)):
        if k in out:
            rr = r[..., f]
            e[k] = float(_norm(out[k][..., f] - rr).max() / max(_norm(rr).max(), 1e-300))
    if "P" in out:
        e["P"] = float(np.abs(out["P"][f] - ref.P[f]).max() / B)
    return e


def mixed_tol(steps: int) -> float:
    """Bar of the FP32-mixed path after `steps` steps: 1e-5 per step, 1e-3 after 100 steps."""
    return min(1e-3, 1e-5 * max(1, int(steps)))
