"""Flow-field quality measures against synthetic ground truth.

The paper scores raw correspondence fields on non-occluded pixels by the
share of flows with endpoint error below 3 px, the endpoint error clipped at
10 px per flow (EPE10) and the plain endpoint error (Sec. 4.2, the measures
listed before Table "tesin").  Density and EPE of the pixels kept by the
consistency check describe the filtered field.
"""
from __future__ import annotations

import numpy as np


def epe_stats(flow: np.ndarray, flow_gt: np.ndarray, occ: np.ndarray, keep: np.ndarray | None = None,
              valid: np.ndarray | None = None) -> dict:
    f = flow.astype(np.float64)
    g = flow_gt.astype(np.float64)
    err = np.hypot(f[..., 0] - g[..., 0], f[..., 1] - g[..., 1])
    m = ~occ
    if valid is not None:
        m &= valid
    e = err[m]
    out = {
        "epe": float(e.mean()) if e.size else float("nan"),
        "le3px": float((e <= 3.0).mean()) if e.size else float("nan"),
        "epe10": float(np.minimum(e, 10.0).mean()) if e.size else float("nan"),
        "n_nonocc": int(m.sum()),
    }
    if keep is not None:
        k = keep.astype(bool) & m
        ek = err[k]
        out["kept_density"] = float(k.sum() / max(1, m.sum()))
        out["kept_epe"] = float(ek.mean()) if ek.size else float("nan")
        out["kept_le3px"] = float((ek <= 3.0).mean()) if ek.size else float("nan")
    return out
