"""Pins of the oracle's subpixel form (Sec. 3.1: random-search offsets with
subpixel accuracy, the target patch's colours by bilinear interpolation):
flows in units of 1/2^s pixel, image b's descriptors bilinearly
interpolated at the target, costs scaled by 4^s so they stay exact
integers.  Tied to the integer cost (integer flows), to SciPy's bilinear
interpolation (a library routine), to the exact zero of a linear ramp under
a subpixel shift, to hand-worked consistency cases and to the invariants of
the schedule."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from ffgen import random_images, translated_crops

UNSET = oracle.UNSET


def _descs(img, n):
    return oracle.descriptor(oracle.blur(img, n), n)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_integer_flows_give_scaled_integer_cost(s):
    ia, ib = random_images(41 + s, 26, 31)
    Da, Db = _descs(ia, 2), _descs(ib, 2)
    rng = np.random.default_rng(s)
    S = 1 << s
    for _ in range(40):
        x, y = int(rng.integers(0, 31)), int(rng.integers(0, 26))
        fx, fy = int(rng.integers(-x, 31 - x)), int(rng.integers(-y, 26 - y))
        assert oracle.cost_sub(Da, Db, 2, 3, x, y, fx * S, fy * S, s) == S * S * oracle.cost(Da, Db, 2, 3, x, y, fx,
                                                                                               fy)


def _cost_scipy(Da, Db, n, r, x, y, fx, fy, s):
    """Eq. 3 on image b's descriptors interpolated bilinearly at the target
    (scipy.ndimage.map_coordinates, order 1, border replicated), times 4^s."""
    S = 1 << s
    H, W = Da.shape[:2]
    tot = 0.0
    for v in range(-r, r + 1):
        for u in range(-r, r + 1):
            a = Da[min(max(y + n * v, 0), H - 1), min(max(x + n * u, 0), W - 1)].astype(np.float64)
            ty, tx = y + fy / S + n * v, x + fx / S + n * u
            b = np.array([ndi.map_coordinates(Db[..., c].astype(np.float64), [[ty], [tx]], order=1,
                                              mode="nearest")[0] for c in range(16)])
            tot += np.abs(S * S * a - S * S * b).sum()
    return tot


@pytest.mark.parametrize("s,n", [(3, 1), (3, 2), (2, 1), (1, 4)])
def test_subpixel_cost_is_bilinear_interpolation(s, n):
    """Exact equality with SciPy's bilinear interpolation of the
    descriptors at every patch position (in the interior and through the
    border, targets up to the last pixel)."""
    ia, ib = random_images(60 + s + n, 20, 23)
    Da, Db = _descs(ia, n), _descs(ib, n)
    H, W = ia.shape
    S = 1 << s
    rng = np.random.default_rng(7 * s + n)
    cases = [(0, 0, 0, 0), (W - 1, H - 1, 0, 0), (W - 2, H - 2, S - 1, S - 1), (3, 4, 5, -7)]
    for _ in range(25):
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        tx8, ty8 = int(rng.integers(0, (W - 1) * S + 1)), int(rng.integers(0, (H - 1) * S + 1))
        cases.append((x, y, tx8 - x * S, ty8 - y * S))
    for x, y, fx, fy in cases:
        assert 0 <= x * S + fx <= (W - 1) * S and 0 <= y * S + fy <= (H - 1) * S
        got = oracle.cost_sub(Da, Db, n, 3, x, y, fx, fy, s)
        assert got == _cost_scipy(Da, Db, n, 3, x, y, fx, fy, s), (x, y, fx, fy)


def test_linear_ramp_under_a_subpixel_shift_costs_zero():
    """A linear ramp stays linear under the box blur (symmetric mean) and
    under bilinear interpolation, so image b = image a shifted by 3/8 px
    to the left has zero cost exactly at the flow 3/8 (interior pixels),
    and no other flow on the 1/8 grid along x costs zero."""
    H, W = 28, 30
    ys, xs = np.mgrid[0:H, 0:W]
    a = (8 * xs + 0 * ys).astype(np.uint8)           # 0 .. 232
    b = np.clip(8 * xs + 3, 0, 255).astype(np.uint8)  # a(x + 3/8): b(x) = a(x) + 3
    Da, Db = _descs(a, 1), _descs(b, 1)
    for x, y in ((12, 14), (9, 8), (20, 20)):
        # the target x - 3/8 has value 8 (x - 3/8) + 3 = 8x
        assert oracle.cost_sub(Da, Db, 1, 3, x, y, -3, 0, 3) == 0
        others = [oracle.cost_sub(Da, Db, 1, 3, x, y, fx, 0, 3) for fx in range(-16, 9) if fx != -3]
        assert min(others) > 0


def test_consistency_sub_hand_worked():
    """Nearest pixel of the target (halves up) and the threshold in 1/8 px."""
    H, W, s = 3, 6, 3
    fa = np.zeros((H, W, 2), np.int16)
    fb = np.zeros((H, W, 2), np.int16)
    ca = np.zeros((H, W), np.uint32)
    cb = np.zeros((H, W), np.uint32)
    fa[1, 1] = (3, 0)    # target 1 + 3/8 -> pixel 1
    fb[1, 1] = (-3, 0)   # exact inverse: kept
    fa[1, 2] = (4, 0)    # target 2 + 1/2 -> pixel 3 (half up)
    fb[1, 3] = (-11, 0)  # |4 - 11| = 7 < 8: kept
    fa[1, 3] = (-12, 4)  # target (1.5, 1.5) -> pixel (2, 2)
    fb[2, 2] = (12, 4)   # |(0, 8)| = 8, not < 8: removed
    fa[0, 4] = (8, 0)    # target pixel 5, UNSET in b: removed
    cb[0, 5] = UNSET
    keep = oracle.consistency_sub(fa, ca, fb, cb, s, 1.0)
    assert keep[1, 1] == 1 and keep[1, 2] == 1 and keep[1, 3] == 0 and keep[0, 4] == 0
    assert keep[0, 0] == 1  # zero flow against zero flow
    # the integer form is the special case s = 0
    fi = (fa // 8).astype(np.int16)
    gi = (fb // 8).astype(np.int16)
    assert np.array_equal(oracle.consistency_sub(fi, ca, gi, cb, 0, 1.0), oracle.consistency(fi, ca, gi, cb, 1.0))


def test_subpixel_steps_keep_costs_consistent_and_monotone():
    """Propagation and random search of the subpixel form: costs never rise,
    every stored cost recomputes from its flow, every target stays in the
    image, and random search reaches flows off the integer grid."""
    ia, ib = random_images(91, 22, 30)
    s, S, n = 3, 8, 1
    Da, Db = _descs(ia, n), _descs(ib, n)
    idx, _ = oracle.nn(Da, Db, 1)
    H, W = ia.shape
    ys, xs = np.mgrid[0:H, 0:W]
    flow = np.stack([(idx % W - xs) * S, (idx // W - ys) * S], -1).astype(np.int16)
    cost = np.array([[oracle.cost_sub(Da, Db, n, 3, x, y, int(flow[y, x, 0]), int(flow[y, x, 1]), s)
                      for x in range(W)] for y in range(H)], np.uint32)
    for t in range(3):
        f2, c2, _ = oracle.propagate_sub(Da, Db, n, s, t, flow, cost)
        assert np.all(c2 <= cost)
        f3, c3, ne = oracle.random_search_sub(Da, Db, n, s, 1, 12345, 0, 0, t, f2, c2)
        assert ne > 0 and np.all(c3 <= c2)
        flow, cost = f3, c3
    tx, ty = xs * S + flow[..., 0], ys * S + flow[..., 1]
    assert np.all((tx >= 0) & (tx <= (W - 1) * S) & (ty >= 0) & (ty <= (H - 1) * S))
    for y in range(0, H, 3):
        for x in range(0, W, 4):
            assert cost[y, x] == oracle.cost_sub(Da, Db, n, 3, x, y, int(flow[y, x, 0]), int(flow[y, x, 1]), s)
    assert np.any(flow % S != 0)


@pytest.mark.parametrize("t", [(5, -3), (-9, 4)])
def test_subpixel_field_recovers_an_integer_translation(t):
    """Two crops of one canvas offset by an integer t: the subpixel field
    is exactly 8t with zero cost at every pixel whose coarsest-scale patch
    lies inside both frames (zero is the least cost, so no subpixel offset
    can replace it)."""
    H, W, L = 48, 64, 3
    ia, ib = translated_crops(33, H, W, t[0], t[1])
    o = oracle.flow_fields(ia, ib, L, 4, nthreads=2, subpixel=3)
    ys, xs = np.mgrid[0:H, 0:W]
    m = 3 * (1 << (L - 1)) + 1
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    assert inner.sum() > 300
    f = o["flow_fwd"]
    assert np.all(f[inner][:, 0] == 8 * t[0]) and np.all(f[inner][:, 1] == 8 * t[1])
    assert np.all(o["cost_fwd"][inner] == 0)


def test_subpixel_zero_bits_is_the_integer_field():
    ia, ib = random_images(5, 40, 52)
    a = oracle.flow_fields(ia, ib, 3, 4, nthreads=2)
    b = oracle.flow_fields(ia, ib, 3, 4, nthreads=2, subpixel=0)
    for k in ("flow_fwd", "flow_bwd", "cost_fwd", "keep_fwd"):
        assert np.array_equal(a[k], b[k])
