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

    rho and T: max|a-b| / max|b| and rms(a-b) / rms(b).  u is a vector whose
    pointwise relative error is undefined where u = 0, so its error is the
    vector error over the largest speed: max|du| / max|u| and
    rms|du| / rms|u|.  The same error scaled by the thermal speed
    sqrt(min T) instead (never larger than the flow speeds of these
    workloads allow) is reported as info_u_thermal and is not asserted.
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
    out["u_max"] = float(du.max() / max(float(un.max()), 1e-300))
    out["u_rms"] = float(np.sqrt(np.mean(du * du)) / max(float(np.sqrt(np.mean(un * un))), 1e-300))
    out["info_u_thermal"] = float(du.max() / float(np.sqrt(r[3].min())))
    out["info_max_u"] = float(un.max())
    return out


def worst(errs) -> float:
    return max(v for k, v in errs.items() if not k.startswith("info_"))
