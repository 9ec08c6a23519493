"""Float patch cost and its gradient, float64 (oracle of the learned-feature path).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a learned data term (Sec. 3.5, the CNN features of the cited follow-up
work) the matching error of the subsampled patch P^n_r (Eq. 3) is read as
the sum of squared differences of the feature vectors:

    C(p, f) = sum_{u,v=-r..r} sum_c ( f1(clamp(p + n(u,v)))[c] - f2(clamp(p + f + n(u,v)))[c] )^2

with the replicate border of Sec. 3.6 (clamp to the nearest pixel).  Its
gradient with respect to the two feature maps, for an upstream gradient g
per evaluated (p, f):

    dL/df1[q] += 2 g (f1(q) - f2(t)),   dL/df2[t] -= 2 g (f1(q) - f2(t))

for every patch position, q = clamp(p + n(u,v)), t = clamp(p + f + n(u,v)).
Entries are rows (x, y, fx, fy): the pixel p and the candidate flow f.
"""
from __future__ import annotations

import numpy as np


def _positions(entries, W, H, n, r):
    e = np.asarray(entries, dtype=np.int64).reshape(-1, 4)
    off = np.arange(-r, r + 1) * n
    ov, ou = np.meshgrid(off, off, indexing="ij")  # v outer, u inner
    ou, ov = ou.reshape(-1), ov.reshape(-1)
    qx = np.clip(e[:, 0:1] + ou[None, :], 0, W - 1)
    qy = np.clip(e[:, 1:2] + ov[None, :], 0, H - 1)
    tx = np.clip(e[:, 0:1] + e[:, 2:3] + ou[None, :], 0, W - 1)
    ty = np.clip(e[:, 1:2] + e[:, 3:4] + ov[None, :], 0, H - 1)
    return qx, qy, tx, ty


def cost_f64(f1, f2, entries, n: int = 1, r: int = 3) -> np.ndarray:
    """C(p, f) for every entry, float64."""
    f1 = np.asarray(f1, np.float64)
    f2 = np.asarray(f2, np.float64)
    H, W = f1.shape[:2]
    qx, qy, tx, ty = _positions(entries, W, H, n, r)
    d = f1[qy, qx] - f2[ty, tx]          # [entries][positions][C]
    return (d * d).sum(axis=(1, 2))


def grad_f64(f1, f2, entries, g, n: int = 1, r: int = 3):
    """(dL/df1, dL/df2) for upstream gradient g per entry, float64.

    Also returns the per-element sum of |contributions|, the scale of the
    rounding error of any finite-precision accumulation of the same terms.
    """
    f1 = np.asarray(f1, np.float64)
    f2 = np.asarray(f2, np.float64)
    H, W, C = f1.shape
    qx, qy, tx, ty = _positions(entries, W, H, n, r)
    g = np.asarray(g, np.float64).reshape(-1, 1, 1)
    d = 2.0 * g * (f1[qy, qx] - f2[ty, tx])  # [entries][positions][C]
    g1 = np.zeros_like(f1)
    g2 = np.zeros_like(f2)
    a1 = np.zeros_like(f1)
    a2 = np.zeros_like(f2)
    np.add.at(g1, (qy.reshape(-1), qx.reshape(-1)), d.reshape(-1, C))
    np.add.at(g2, (ty.reshape(-1), tx.reshape(-1)), -d.reshape(-1, C))
    np.add.at(a1, (qy.reshape(-1), qx.reshape(-1)), np.abs(d).reshape(-1, C))
    np.add.at(a2, (ty.reshape(-1), tx.reshape(-1)), np.abs(d).reshape(-1, C))
    return g1, g2, a1, a2
