"""Shared helpers of the test-suite: error metrics and GPU availability."""

from __future__ import annotations

import numpy as np


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def field_errors(gpu, ref):
    """Per-field relative errors of (rho, ux, uy, T) tuples.

    rho and T: max|a-b| / max|b| and rms(a-b) / rms(b).  u is a vector and is
    computed by cancellation (rho u = sum c_l f_l with summands of the size of
    the thermal speed sqrt(T)), so its error is scaled by
    max(max |u|, sqrt(min T)): the larger of the flow speed and the thermal
    speed.  The error relative to max |u| alone is reported as info_u_max.
    """
    g = [np.asarray(a, dtype=np.float64) for a in gpu]
    r = [np.asarray(a, dtype=np.float64) for a in ref]
    out = {}
    for name, i in (("rho", 0), ("T", 3)):
        d = g[i] - r[i]
        out[name + "_max"] = float(np.abs(d).max() / np.abs(r[i]).max())
        out[name + "_rms"] = float(np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(r[i] * r[i])))
    du = np.hypot(g[1] - r[1], g[2] - r[2])
    un = np.hypot(r[1], r[2])
    scale = max(float(un.max()), float(np.sqrt(r[3].min())))
    out["u_max"] = float(du.max() / scale)
    out["u_rms"] = float(np.sqrt(np.mean(du * du)) / scale)
    out["info_u_max"] = float(du.max() / max(un.max(), 1e-300))
    return out


def worst(errs) -> float:
    return max(v for k, v in errs.items() if not k.startswith("info_"))
