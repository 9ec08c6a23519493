"""Pins of the oracle's learned-feature schedule (float cost, quantised NN).

The float cost is tied to the float64 formula of oracle.float_cost within the
single-precision accumulation bound; the quantiser to its closed-form
properties; the whole schedule to the zero field on identical maps and to
exact recovery of an integer translation of a feature canvas.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from oracle.float_cost import cost_f64


def feature_canvas(seed, H, W, C=16):
    """Smooth random 16-channel float features (random 5x5 filters of noise)."""
    rng = np.random.default_rng(seed)
    base = rng.random((H, W))
    out = np.empty((H, W, C), np.float32)
    for c in range(C):
        k = rng.normal(size=(5, 5))
        out[..., c] = ndi.correlate(base, k, mode="nearest")
    return out


def feature_pyramid(F, levels):
    """Per-scale maps: scale 2^l uses the map smoothed by a box of half-width
    max(1, 2^l / 2) (a low-pass stand-in; any per-scale maps are valid input)."""
    maps = [F]
    for l in range(1, levels):
        h = max(1, (1 << l) // 2)
        maps.append(ndi.uniform_filter(F, size=(2 * h + 1, 2 * h + 1, 1), mode="nearest").astype(np.float32))
    return maps


@pytest.mark.parametrize("n", [1, 2, 4])
def test_cost_f32_within_single_precision_of_f64(n):
    Fa = feature_canvas(1, 30, 40)
    Fb = feature_canvas(2, 30, 40)
    rng = np.random.default_rng(n)
    for _ in range(40):
        x, y = int(rng.integers(0, 40)), int(rng.integers(0, 30))
        fx, fy = int(rng.integers(-x, 40 - x)), int(rng.integers(-y, 30 - y))
        got = oracle.cost_f32(Fa, Fb, n, 3, x, y, fx, fy)
        ref = cost_f64(Fa, Fb, np.array([[x, y, fx, fy]]), n, 3)[0]
        assert abs(got - ref) <= 784 * 2.0 ** -24 * ref + 1e-6
    assert oracle.cost_f32(Fa, Fa, n, 3, 5, 5, 0, 0) == 0.0


def test_quantize_closed_form_properties():
    f = feature_canvas(3, 20, 30).reshape(-1)
    q = oracle.quantize_u8(f)
    lo, hi = f.min(), f.max()
    assert q[np.argmin(f)] == 0 and q[np.argmax(f)] == 255
    exact = (f.astype(np.float64) - lo) * 255.0 / (float(hi) - float(lo))
    assert np.all(np.abs(q - exact) <= 0.5 + 1e-3)
    order = np.argsort(f, kind="stable")
    assert np.all(np.diff(q[order].astype(int)) >= 0)  # monotone
    assert np.all(oracle.quantize_u8(np.full(50, 3.25, np.float32)) == 0)  # degenerate range


def test_identical_features_give_zero_field():
    F = feature_canvas(4, 40, 56)
    maps = feature_pyramid(F, 3)
    o = oracle.flow_fields_f32(maps, maps, 3, 4, nthreads=2)
    assert np.all(o["flow_fwd"] == 0) and np.all(o["flow_bwd"] == 0)
    assert np.all(o["cost_fwd"] == 0) and np.all(o["keep_fwd"] == 1)


@pytest.mark.parametrize("t", [(4, -3), (-7, 5)])
def test_translated_features_exact_recovery(t):
    H, W, pad = 48, 64, 12
    canvas = feature_canvas(5, H + 2 * pad, W + 2 * pad)
    F1 = canvas[pad:pad + H, pad:pad + W].copy()
    F2 = canvas[pad - t[1]:pad - t[1] + H, pad - t[0]:pad - t[0] + W].copy()
    L = 2
    o = oracle.flow_fields_f32([F1, F1], [F2, F2], L, 4, nthreads=2)
    ys, xs = np.mgrid[0:H, 0:W]
    m = 3 * (1 << (L - 1))  # patch reach at the coarsest scale
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    assert inner.sum() > 400
    f = o["flow_fwd"]
    assert np.all(f[inner][:, 0] == t[0]) and np.all(f[inner][:, 1] == t[1])
    assert np.all(o["cost_fwd"][inner].view(np.float32) == 0.0)


def test_quantize_pair_shares_one_range():
    """Both maps are quantised with the range of their union: the closed form
    per element, equal values give equal bytes in both maps."""
    f1 = feature_canvas(6, 20, 30)
    f2 = feature_canvas(7, 20, 30) * 3.0 + 1.0
    q1, q2 = oracle.quantize_pair_u8(f1, f2)
    lo = float(min(f1.min(), f2.min()))
    hi = float(max(f1.max(), f2.max()))
    for f, q in ((f1, q1), (f2, q2)):
        exact = (f.astype(np.float64) - lo) * 255.0 / (hi - lo)
        assert np.all(np.abs(q - exact) <= 0.5 + 1e-3)
    assert q1.min() > 0 or q2.min() == 0
    both = np.concatenate([f1.ravel(), f2.ravel()])
    qb = np.concatenate([q1.ravel(), q2.ravel()])
    assert qb[np.argmin(both)] == 0 and qb[np.argmax(both)] == 255


def test_quantized_nn_recovers_a_shift_under_a_different_value_range():
    """Image 2's features are image 1's shifted by t, except for a strip of
    content entering at the border with values far outside image 1's range.
    One shared range maps equal features to equal bytes, so the byte-space
    nearest neighbour of every grid cell whose match lies inside image 2 is
    its shifted pixel (Sec. 3.1 seed: the nearest neighbour in feature
    space).  Separate ranges per image break that (the check that this pin
    can fail)."""
    H, W, pad, t = 40, 56, 8, (5, -3)
    canvas = feature_canvas(21, H + 2 * pad, W + 2 * pad)
    F1 = canvas[pad:pad + H, pad:pad + W].copy()
    F2 = canvas[pad - t[1]:pad - t[1] + H, pad - t[0]:pad - t[0] + W].copy()
    F2[:, W - 4:] = F2[:, W - 4:] * 4.0 + 6.0  # entering content with another value range
    nc = 4
    q1, q2 = oracle.quantize_pair_u8(F1, F2)
    idx, dist = oracle.nn(q1, q2, nc)
    sep1, sep2 = oracle.quantize_u8(F1), oracle.quantize_u8(F2)
    idx_sep, _ = oracle.nn(sep1, sep2, nc)
    Hc, Wc = idx.shape
    checked = wrong_sep = 0
    for j in range(Hc):
        for i in range(Wc):
            x, y = i * nc + t[0], j * nc + t[1]
            if not (0 <= x < W - 4 and 0 <= y < H):
                continue
            checked += 1
            assert idx[j, i] == y * W + x and dist[j, i] == 0, (i, j)
            wrong_sep += idx_sep[j, i] != y * W + x
    assert checked > 80
    assert wrong_sep > checked // 2
