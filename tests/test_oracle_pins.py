"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties one oracle function to something other than itself: a value
worked by hand, a library routine, a closed form, an invariant of the method
or brute force on tiny inputs.  Sections cited are those of Bailer, Taetz,
Stricker, "Flow Fields" (the journal version).
"""
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from ffgen import make_pair, random_images, translated_crops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNSET = oracle.UNSET


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ---------------------------------------------------------------- blur (Sec. 3.2, Sec. 3.6)

def test_blur_hand_worked_example():
    rows = [list(map(int, r.split())) for r in _read_golden("blur_desc_5x4.txt")]
    img = np.array(rows[:4], np.uint8)
    expect = np.array(rows[4:], np.uint8)
    assert np.array_equal(oracle.blur(img, 1), expect)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_blur_equals_library_box_sum(n):
    img, _ = random_images(11 + n, 37, 53, kind="uniform")
    h = max(1, n // 2)
    k = np.ones((2 * h + 1, 2 * h + 1), np.int64)
    s = ndi.correlate(img.astype(np.int64), k, mode="nearest")
    A = (2 * h + 1) ** 2
    assert np.array_equal(oracle.blur(img, n), ((s + A // 2) // A).astype(np.uint8))


def test_blur_constant_image_is_constant():
    img = np.full((9, 13), 77, np.uint8)
    for n in (1, 4, 16):
        assert np.all(oracle.blur(img, n) == 77)


# ---------------------------------------------------------------- descriptor (Sec. 3.6, F2)

@pytest.mark.parametrize("n", [1, 2, 4])
def test_descriptor_channels_are_edge_padded_shifts(n):
    b, _ = random_images(5, 23, 31, kind="uniform")
    d = oracle.descriptor(b, n)
    m = 3 * n
    p = np.pad(b, m, mode="edge")
    H, W = b.shape
    for gy in range(4):
        for gx in range(4):
            oy, ox = n * (2 * gy - 3), n * (2 * gx - 3)
            assert np.array_equal(d[..., 4 * gy + gx], p[m + oy:m + oy + H, m + ox:m + ox + W])


def test_descriptor_constant_image():
    d = oracle.descriptor(np.full((7, 6), 200, np.uint8), 2)
    assert np.all(d == 200)


# ---------------------------------------------------------------- cost E_n (Eq. 3)

W13 = np.array([1, 1, 2, 2, 3, 3, 4, 3, 3, 2, 2, 1, 1], np.int64)


def _weighted_13x13(Ba, Bb, n, p, q):
    """E_n in the interior written on the blurred images: every descriptor
    channel is one blurred sample, patch offset u plus descriptor offset
    2g-3 covers a = -6..6 with multiplicity W13[a+6] per axis."""
    s = 0
    for b in range(-6, 7):
        for a in range(-6, 7):
            va = int(Ba[p[1] + n * b, p[0] + n * a])
            vb = int(Bb[q[1] + n * b, q[0] + n * a])
            s += W13[a + 6] * W13[b + 6] * abs(va - vb)
    return s


@pytest.mark.parametrize("n", [1, 2, 4])
def test_cost_interior_weighted_identity(n):
    H, W = 40 + 12 * n, 44 + 12 * n
    ia, ib = random_images(3 * n, H, W)
    Ba, Bb = oracle.blur(ia, n), oracle.blur(ib, n)
    Da, Db = oracle.descriptor(Ba, n), oracle.descriptor(Bb, n)
    rng = np.random.default_rng(n)
    lo = 6 * n
    for _ in range(25):
        p = (int(rng.integers(lo, W - lo)), int(rng.integers(lo, H - lo)))
        q = (int(rng.integers(lo, W - lo)), int(rng.integers(lo, H - lo)))
        e = oracle.cost(Da, Db, n, 3, p[0], p[1], q[0] - p[0], q[1] - p[1])
        assert e == _weighted_13x13(Ba, Bb, n, p, q)


def _weighted_13x13_clamped(Ba, Bb, n, p, q):
    """The 13 x 13 weighted sum with the blurred samples read through the
    image border (replicate): the descriptors' own clamp."""
    H, W = Ba.shape
    s = 0
    for b in range(-6, 7):
        ya, yb = min(max(p[1] + n * b, 0), H - 1), min(max(q[1] + n * b, 0), H - 1)
        for a in range(-6, 7):
            xa, xb = min(max(p[0] + n * a, 0), W - 1), min(max(q[0] + n * a, 0), W - 1)
            s += W13[a + 6] * W13[b + 6] * abs(int(Ba[ya, xa]) - int(Bb[yb, xb]))
    return s


@pytest.mark.parametrize("n", [1, 2, 4])
def test_cost_weighted_identity_holds_3n_inside(n):
    """The weighted identity with clamped blurred samples holds exactly when
    the pixel and the target are at least 3n inside the image (every patch
    position is then in the image, so the patch clamp does nothing and only
    the descriptors' own clamp remains), and fails just outside."""
    H, W = 30 + 8 * n, 34 + 8 * n
    ia, ib = random_images(5 * n, H, W)
    Ba, Bb = oracle.blur(ia, n), oracle.blur(ib, n)
    Da, Db = oracle.descriptor(Ba, n), oracle.descriptor(Bb, n)
    rng = np.random.default_rng(n)
    lo = 3 * n

    def pick(L):  # biased to the edge of the interior
        return int((lo, L - 1 - lo, rng.integers(lo, L - lo), lo + 1)[rng.integers(0, 4)])

    for _ in range(120):
        p, q = (pick(W), pick(H)), (pick(W), pick(H))
        e = oracle.cost(Da, Db, n, 3, p[0], p[1], q[0] - p[0], q[1] - p[1])
        assert e == _weighted_13x13_clamped(Ba, Bb, n, p, q), (p, q)
    outside = 0
    for _ in range(40):
        p = (lo - 1, int(rng.integers(lo, H - lo)))
        q = (int(rng.integers(lo, W - lo)), int(rng.integers(lo, H - lo)))
        outside += oracle.cost(Da, Db, n, 3, p[0], p[1], q[0] - p[0], q[1] - p[1]) != \
            _weighted_13x13_clamped(Ba, Bb, n, p, q)
    assert outside > 30


def test_cost_border_is_edge_replication():
    n, r = 2, 3
    ia, ib = random_images(9, 20, 26)
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    M = 3 * n * 2 + 30
    Pa = np.ascontiguousarray(np.pad(Da, ((M, M), (M, M), (0, 0)), mode="edge"))
    Pb = np.ascontiguousarray(np.pad(Db, ((M, M), (M, M), (0, 0)), mode="edge"))
    H, W = ia.shape
    rng = np.random.default_rng(0)
    for _ in range(40):
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        tx, ty = int(rng.integers(0, W)), int(rng.integers(0, H))
        e = oracle.cost(Da, Db, n, r, x, y, tx - x, ty - y)
        e_pad = oracle.cost(Pa, Pb, n, r, x + M, y + M, tx - x, ty - y)
        assert e == e_pad


def test_cost_zero_symmetry_and_bound():
    ia, ib = random_images(4, 18, 22)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    assert oracle.cost(Da, Da, 1, 3, 5, 7, 0, 0) == 0
    rng = np.random.default_rng(1)
    for _ in range(30):
        x, y = int(rng.integers(0, 22)), int(rng.integers(0, 18))
        tx, ty = int(rng.integers(0, 22)), int(rng.integers(0, 18))
        e = oracle.cost(Da, Db, 1, 3, x, y, tx - x, ty - y)
        # roles of the images swapped, seen from the target pixel
        assert e == oracle.cost(Db, Da, 1, 3, tx, ty, x - tx, y - ty)
        assert e <= 49 * 16 * 255
    white = np.full_like(Da, 255)
    black = np.zeros_like(Da)
    assert oracle.cost(white, black, 1, 3, 3, 3, 1, 1) == 49 * 16 * 255


# ---------------------------------------------------------------- NN seed (Sec. 3.1 / 3.2 init)

@pytest.mark.parametrize("nc", [1, 2, 4])
def test_nn_equals_numpy_brute_force(nc):
    ia, ib = random_images(21 + nc, 17, 23, kind="uniform")
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    idx, dist = oracle.nn(Da, Db, nc, nthreads=2)
    H, W = ia.shape
    q = Da[::nc, ::nc].reshape(-1, 16).astype(np.int64)
    refs = Db.reshape(-1, 16).astype(np.int64)
    d = ((q[:, None, :] - refs[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(idx.reshape(-1), np.argmin(d, axis=1))  # first minimum = smallest index
    assert np.array_equal(dist.reshape(-1), d.min(axis=1))


def test_nn_ties_go_to_smallest_index():
    ia, _ = random_images(2, 12, 14)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = np.full_like(Da, 100)
    idx, _ = oracle.nn(Da, Db, 2)
    assert np.all(idx == 0)
    Db = Db.copy()
    Db[5, 7] = Da[4, 6]
    Db[9, 2] = Da[4, 6]
    idx, dist = oracle.nn(Da, Db, 2)
    assert idx[2, 3] == 5 * 14 + 7 and dist[2, 3] == 0


def test_init_coarse_flow_is_target_minus_pixel():
    ia, ib = random_images(8, 21, 27)
    nc = 4
    Da1 = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db1 = oracle.descriptor(oracle.blur(ib, 1), 1)
    Dac = oracle.descriptor(oracle.blur(ia, nc), nc)
    Dbc = oracle.descriptor(oracle.blur(ib, nc), nc)
    idx, _ = oracle.nn(Da1, Db1, nc)
    flow, cost, ne = oracle.init_coarse(idx, Dac, Dbc, nc)
    Hc, Wc = idx.shape
    assert ne == Hc * Wc
    for j in range(Hc):
        for i in range(Wc):
            qx, qy = idx[j, i] % 27, idx[j, i] // 27
            assert tuple(flow[j, i]) == (qx - i * nc, qy - j * nc)
            assert 0 <= i * nc + flow[j, i, 0] < 27 and 0 <= j * nc + flow[j, i, 1] < 21


@pytest.mark.parametrize("nc", [4, 8])
def test_init_coarse_cost_is_the_scale_nc_cost(nc):
    """The seed cost is E_nc (Eq. 4 ranks the candidates with the cost of
    the coarsest scale): on cells whose pixel and target are 6 nc inside
    the image it equals the 13 x 13 weighted sum over the scale-nc blurred
    images, which is not the sum over the level-1 blurred images."""
    H, W, pad, t = 14 * nc + 16, 16 * nc + 20, 12, (3, -2)
    big, _ = random_images(70 + nc, H + 2 * pad, W + 2 * pad)
    ia = big[pad:pad + H, pad:pad + W].copy()
    ib = big[pad - t[1]:pad - t[1] + H, pad - t[0]:pad - t[0] + W].copy()
    ib = np.clip(ib.astype(int) + np.random.default_rng(nc).integers(-6, 7, ib.shape), 0, 255).astype(np.uint8)
    B1a, B1b = oracle.blur(ia, 1), oracle.blur(ib, 1)
    Bca, Bcb = oracle.blur(ia, nc), oracle.blur(ib, nc)
    Da1, Db1 = oracle.descriptor(B1a, 1), oracle.descriptor(B1b, 1)
    Dac, Dbc = oracle.descriptor(Bca, nc), oracle.descriptor(Bcb, nc)
    idx, _ = oracle.nn(Da1, Db1, nc, nthreads=2)
    flow, cost, _ = oracle.init_coarse(idx, Dac, Dbc, nc)
    Hc, Wc = idx.shape
    lo = 6 * nc
    checked = differs = 0
    for j in range(Hc):
        for i in range(Wc):
            p = (i * nc, j * nc)
            q = (p[0] + int(flow[j, i, 0]), p[1] + int(flow[j, i, 1]))
            if not all(lo <= v < hi - lo for v, hi in ((p[0], W), (p[1], H), (q[0], W), (q[1], H))):
                continue
            checked += 1
            assert cost[j, i] == _weighted_13x13(Bca, Bcb, nc, p, q), (i, j)
            differs += cost[j, i] != _weighted_13x13(B1a, B1b, 1, p, q)
    assert checked >= 4 and differs == checked


# ---------------------------------------------------------------- level seeding (Sec. 3.2)

def test_seed_level_keeps_shared_pixels_and_unsets_others():
    ia, ib = random_images(12, 19, 25)
    n = 2
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    Wc, Hc = -(-25 // 4), -(-19 // 4)
    rng = np.random.default_rng(3)
    cflow = np.stack([rng.integers(-3, 4, (Hc, Wc)), rng.integers(-3, 4, (Hc, Wc))], -1).astype(np.int16)
    ccost = rng.integers(0, 1000, (Hc, Wc)).astype(np.uint32)
    ccost[1, 2] = UNSET
    cflow[1, 2] = 0
    flow, cost, ne = oracle.seed_level(cflow, ccost, Da, Db, n)
    Hn, Wn = cost.shape
    assert (Wn, Hn) == (13, 10)
    n_set = 0
    for j in range(Hn):
        for i in range(Wn):
            if i % 2 == 0 and j % 2 == 0 and ccost[j // 2, i // 2] != UNSET:
                assert tuple(flow[j, i]) == tuple(cflow[j // 2, i // 2])
                fx, fy = map(int, flow[j, i])
                assert cost[j, i] == oracle.cost(Da, Db, n, 3, i * n, j * n, fx, fy)
                n_set += 1
            else:
                assert cost[j, i] == UNSET and tuple(flow[j, i]) == (0, 0)
    assert ne == n_set


# ---------------------------------------------------------------- propagation (Eq. 2, Fig. 4)

QUADRANT = {0: (+1, +1), 1: (-1, -1), 2: (-1, +1), 3: (+1, -1)}


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_propagation_spreads_into_its_quadrant(d):
    """A lone seed spreads within one 90-degree quadrant per step (Fig. 4a/c);
    the first direction is right and down (Sec. 3.1).  With two
    half-sweeps, odd cells first, one step reaches Manhattan distance 2."""
    ia, ib = random_images(30 + d, 24, 24)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    flow = np.zeros((24, 24, 2), np.int16)
    cost = np.full((24, 24), UNSET, np.uint32)
    i0, j0 = 12, 10
    cost[j0, i0] = 5
    flow2, cost2, ne = oracle.propagate(Da, Db, 1, d, flow, cost)
    sx, sy = QUADRANT[d]
    expect = {(i0 + sx * a, j0 + sy * b) for a in range(3) for b in range(3) if a + b <= 2}
    got = {(i, j) for j in range(24) for i in range(24) if cost2[j, i] != UNSET}
    assert got == expect
    # one evaluation per new cell: the diagonal cell's second source holds the
    # flow it has just taken and is skipped
    assert ne == 5
    assert np.all(flow2 == 0)


def _tie_case(b_values):
    """A 24 x 24 level-1 case in which image b's descriptors are constant per
    vertical band (b_values: band of x < 12, band of x >= 12), so E_1 of a
    target depends only on the band its patch falls in."""
    ia, _ = random_images(77, 24, 24)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = np.empty_like(Da)
    Db[:, :12] = b_values[0]
    Db[:, 12:] = b_values[1]
    return Da, Db


def _step_from(Da, Db, cell_state):
    """Propagation step 0 (sources: left and top) from a grid in which only
    the given cells are set; returns the flow of cell (11, 10) (odd, first
    half-sweep) and the step's evaluation count."""
    flow = np.zeros((24, 24, 2), np.int16)
    cost = np.full((24, 24), UNSET, np.uint32)
    for (i, j), f in cell_state.items():
        flow[j, i] = f
        cost[j, i] = oracle.cost(Da, Db, 1, 3, i, j, f[0], f[1])
    f2, c2, ne = oracle.propagate(Da, Db, 1, 0, flow, cost)
    return tuple(int(v) for v in f2[10, 11]), int(c2[10, 11]), ne


def test_propagation_ties_prefer_horizontal_then_keep_own():
    """Sec. 4.4 remarks that propagation prefers the horizontal source when
    matching errors are identical; a candidate replaces the held flow only
    if strictly better (Eq. 2).  Cell (11, 10) reads its left source
    (10, 10) and its top source (11, 9); both targets lie in the same
    band of image b (equal errors) or in different bands (strict order)."""
    fh, fv = (-8, 2), (-9, -4)  # both targets of cell (11, 10) in the band x < 12
    Da, Db = _tie_case((100, 100))
    # an UNSET cell with two equal candidates takes the horizontal one
    got, c, _ = _step_from(Da, Db, {(10, 10): fh, (11, 9): fv})
    assert got == fh and c == oracle.cost(Da, Db, 1, 3, 11, 10, *fh)
    # a held flow of equal error stays (neither candidate is strictly lower)
    got, _, _ = _step_from(Da, Db, {(10, 10): fh, (11, 9): fv, (11, 10): (-5, 1)})
    assert got == (-5, 1)
    # strict differences decide, whichever source holds the better flow:
    # image b's band x >= 12 (the target of fr) matches worse, then better
    fr = (4, 3)
    for bands in ((100, 250), (250, 100)):
        Da, Db = _tie_case(bands)
        e_r = oracle.cost(Da, Db, 1, 3, 11, 10, *fr)
        e_h = oracle.cost(Da, Db, 1, 3, 11, 10, *fh)
        assert e_r != e_h
        best = fr if e_r < e_h else fh
        for h, v in ((fr, fh), (fh, fr)):  # the better flow on the horizontal, then the vertical source
            got, c, _ = _step_from(Da, Db, {(10, 10): h, (11, 9): v})
            assert got == best and c == min(e_r, e_h), (bands, h, v)


def test_propagation_is_monotone_and_consistent():
    ia, ib = random_images(40, 20, 28)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    idx, _ = oracle.nn(Da, Db, 1)
    flow, cost, _ = oracle.init_coarse(idx, Da, Db, 1)
    for t in range(4):
        f2, c2, _ = oracle.propagate(Da, Db, 1, t, flow, cost)
        assert np.all(c2 <= cost)
        for j in range(20):
            for i in range(28):
                fx, fy = map(int, f2[j, i])
                assert c2[j, i] == oracle.cost(Da, Db, 1, 3, i, j, fx, fy)
        # every new flow came from a cell of the old or half-updated field
        old = {tuple(v) for v in flow.reshape(-1, 2)}
        assert {tuple(v) for v in f2.reshape(-1, 2)} <= old
        flow, cost = f2, c2


def test_propagation_half_sweep_optimality():
    """After a step, an even cell (second half-sweep) is at least as good as
    both of its source flows, which it read in their final state."""
    ia, ib = random_images(41, 18, 26)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    idx, _ = oracle.nn(Da, Db, 1)
    flow, cost, _ = oracle.init_coarse(idx, Da, Db, 1)
    for d in range(4):
        f2, c2, _ = oracle.propagate(Da, Db, 1, d, flow, cost)
        hx, vy = {0: (-1, -1), 1: (1, 1), 2: (1, -1), 3: (-1, 1)}[d]
        for j in range(18):
            for i in range(26):
                if (i + j) % 2:
                    continue
                for (si, sj) in ((i + hx, j), (i, j + vy)):
                    if 0 <= si < 26 and 0 <= sj < 18:
                        fx, fy = map(int, f2[sj, si])
                        if 0 <= i + fx < 26 and 0 <= j + fy < 18:
                            assert c2[j, i] <= oracle.cost(Da, Db, 1, 3, i, j, fx, fy)


# ---------------------------------------------------------------- random search (Sec. 3.1)

def test_splitmix64_known_answer():
    expect = [int(s, 16) for s in _read_golden("splitmix64_seed0.txt")]
    M = (1 << 64) - 1
    x, got = 0, []
    for _ in range(3):
        x = (x + 0x9E3779B97F4A7C15) & M
        got.append(oracle.mix64(x))
    assert got == expect


def test_rs_offsets_uniform_on_square():
    for Rn in (1, 2, 6):
        side = 2 * Rn + 1
        counts = np.zeros((side, side), np.int64)
        for j in range(60):
            for i in range(100):
                ox, oy = oracle.rs_offset(12345, 0, 2, 1, j, i, Rn)
                assert -Rn <= ox <= Rn and -Rn <= oy <= Rn
                counts[oy + Rn, ox + Rn] += 1
        exp = counts.sum() / side ** 2
        chi2 = ((counts - exp) ** 2 / exp).sum()
        dof = side ** 2 - 1
        assert chi2 < dof + 6 * np.sqrt(2 * dof)
    a = [oracle.rs_offset(7, 0, 0, 0, 0, i, 6) for i in range(64)]
    for other in ([oracle.rs_offset(7, 1, 0, 0, 0, i, 6) for i in range(64)],
                  [oracle.rs_offset(7, 0, 1, 0, 0, i, 6) for i in range(64)],
                  [oracle.rs_offset(7, 0, 0, 1, 0, i, 6) for i in range(64)],
                  [oracle.rs_offset(8, 0, 0, 0, 0, i, 6) for i in range(64)]):
        assert sum(x == y for x, y in zip(a, other)) < 16


def test_rs_radius_floor():
    assert [oracle.rs_radius(n, 1, 1) for n in (1, 2, 4, 8)] == [1, 2, 4, 8]
    assert [oracle.rs_radius(n, 3, 2) for n in (1, 2, 4, 8, 16)] == [1, 3, 6, 12, 24]


def test_random_search_never_worsens_and_moves_locally():
    ia, ib = random_images(50, 22, 30)
    n = 2
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    idx, _ = oracle.nn(oracle.descriptor(oracle.blur(ia, 1), 1), oracle.descriptor(oracle.blur(ib, 1), 1), n)
    flow, cost, _ = oracle.init_coarse(idx, Da, Db, n)
    cost[0, 0] = UNSET
    flow[0, 0] = 0
    f2, c2, ne = oracle.random_search(Da, Db, n, 2, 99, 0, 1, 0, flow, cost)
    assert np.all(c2 <= cost)
    assert c2[0, 0] == UNSET
    moved = np.any(f2 != flow, axis=-1)
    assert moved.any()
    assert np.abs(f2.astype(int) - flow.astype(int)).max() <= 2
    assert ne <= cost.size - 1


# ---------------------------------------------------------------- consistency (Sec. 3.7)

def test_consistency_closed_form():
    H, W = 10, 12
    fa = np.zeros((H, W, 2), np.int16)
    fa[..., 0] = 3
    fa[..., 1] = -1
    fb = -fa.copy()
    ca = np.zeros((H, W), np.uint32)
    cb = np.zeros((H, W), np.uint32)
    # every target must be in the image: the method never holds an outside target
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    out = (xs + 3 >= W) | (ys - 1 < 0)
    ca[out] = UNSET
    fa[out] = 0
    keep = oracle.consistency(fa, ca, fb, cb, 1.0)
    assert np.array_equal(keep.astype(bool), ~out)
    fb2 = fb.copy()
    fb2[4, 7] = (-3, 2)  # off by one px from the inverse of (3, -1) at pixel (4, 5)
    keep2 = oracle.consistency(fa, ca, fb2, cb, 1.0)
    assert keep2[5, 4] == 0 and keep2.sum() == keep.sum() - 1
    assert oracle.consistency(fa, ca, fb2, cb, 1.5)[5, 4] == 1   # |d| = 1 < 1.5
    cb2 = cb.copy()
    cb2[4, 7] = UNSET
    assert oracle.consistency(fa, ca, fb, cb2, 5.0)[5, 4] == 0


def test_consistency_kept_sets_are_in_bijection():
    p = make_pair(1)
    o = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4)
    kf, kb = o["keep_fwd"].astype(bool), o["keep_bwd"].astype(bool)
    ff, fb = o["flow_fwd"].astype(int), o["flow_bwd"].astype(int)
    ys, xs = np.nonzero(kf)
    qx, qy = xs + ff[ys, xs, 0], ys + ff[ys, xs, 1]
    assert np.all(kb[qy, qx])
    assert np.array_equal(fb[qy, qx], -ff[ys, xs])
    assert kf.sum() == kb.sum()


# ---------------------------------------------------------------- whole field (Sec. 3.2)

def test_identical_images_give_zero_field():
    img, _ = random_images(60, 48, 64)
    o = oracle.flow_fields(img, img, 3, 4, nthreads=2)
    for k in ("flow_fwd", "flow_bwd"):
        assert np.all(o[k] == 0)
    assert np.all(o["cost_fwd"] == 0) and np.all(o["cost_bwd"] == 0)
    assert np.all(o["keep_fwd"] == 1)


@pytest.mark.parametrize("t", [(5, -3), (-9, 4), (0, 7)])
def test_integer_translation_exact_recovery(t):
    img1, img2 = translated_crops(70, 56, 72, t[0], t[1])
    o = oracle.flow_fields(img1, img2, 3, 4, nthreads=2)
    H, W = img1.shape
    m = 7  # blur 1 + descriptor 3 + patch 3 pixels of support at n = 1
    ys, xs = np.mgrid[0:H, 0:W]
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    assert inner.sum() > 500
    f = o["flow_fwd"]
    assert np.all(f[inner][:, 0] == t[0]) and np.all(f[inner][:, 1] == t[1])
    assert np.all(o["cost_fwd"][inner] == 0)


def test_final_cost_recomputes_and_bounds_exhaustive_min():
    ia, ib = random_images(80, 24, 32)
    o = oracle.flow_fields(ia, ib, 2, 4, nthreads=2)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    H, W = ia.shape
    for (y, x) in [(0, 0), (5, 9), (23, 31), (12, 16), (3, 28)]:
        fx, fy = map(int, o["flow_fwd"][y, x])
        c = int(o["cost_fwd"][y, x])
        assert c == oracle.cost(Da, Db, 1, 3, x, y, fx, fy)
        best = min(oracle.cost(Da, Db, 1, 3, x, y, qx - x, qy - y) for qy in range(H) for qx in range(W))
        assert c >= best


def test_thread_count_does_not_change_results():
    p = make_pair(1)
    a = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=1)
    b = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=5)
    for k in ("flow_fwd", "flow_bwd", "cost_fwd", "cost_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(a[k], b[k])
    assert a["n_evals"] == b["n_evals"]


def test_evaluation_count_bound():
    """At most 2 evaluations per cell and propagation step and 1 per random
    search step, plus one per seed: 4*2 + 3 = 11 per cell and scale at four
    steps (the count quoted in Sec. 4.2 for the upsampling strategy)."""
    p = make_pair(1)
    L, T = 3, 4
    o = oracle.flow_fields(p.img1, p.img2, L, T, nthreads=4)
    H, W = p.img1.shape
    bound = 0
    for l in range(L):
        n = 1 << l
        cells = (-(-W // n)) * (-(-H // n))
        bound += cells * (2 * T + T - 1) + cells  # + one seed evaluation per cell at most
    assert max(o["n_evals"]) <= bound
    assert min(o["n_evals"]) > 0


# ---------------------------------------------------------------- Flow Fields+ schedules (Sec. 3.3, 3.4)

def _scale_steps_by_hand(level, T, P, Tfine):
    """(steps at R^+, steps at R) of one scale, restated from Sec. 3.3 and
    3.4: P steps at R^+ then T at R; the Fast finest scale only Tfine at R."""
    if level == 0 and Tfine > 0:
        return 0, Tfine
    return P, T


@pytest.mark.parametrize("P,Rp,Tfine", [(4, 2, 0), (4, 2, 4), (2, 3, 0), (3, 2, 1)])
def test_flow_fields_plus_is_the_step_sequence_of_the_paper(P, Rp, Tfine):
    """The oracle's Flow Fields+ driver equals the composition of its
    separately pinned steps in the order Sec. 3.3 gives: P propagation steps
    with random searches at R_n^+ = R^+ n between them, then T steps with
    random searches at R_n between them (none between the two groups), the
    step index running on across both (directions t mod 4); Fast (Sec. 3.4):
    only Tfine steps at R on the finest scale."""
    p = make_pair(1)
    L, T, seed = 3, 4, 777
    o = oracle.flow_fields(p.img1, p.img2, L, T, seed=seed, nthreads=4, plus_iters=P, Rp_num=Rp,
                           fine_iters=Tfine)
    Da, Db = oracle.descriptors_all(p.img1, L), oracle.descriptors_all(p.img2, L)
    nc = 1 << (L - 1)
    idx, _ = oracle.nn(Da[0], Db[0], nc, nthreads=4)
    flow, cost, ne = oracle.init_coarse(idx, Da[L - 1], Db[L - 1], nc)
    for level in range(L - 1, -1, -1):
        n = 1 << level
        if level < L - 1:
            flow, cost, k = oracle.seed_level(flow, cost, Da[level], Db[level], n)
            ne += k
        Pl, Tl = _scale_steps_by_hand(level, T, P, Tfine)
        for t in range(Pl + Tl):
            flow, cost, k = oracle.propagate(Da[level], Db[level], n, t, flow, cost, nthreads=4)
            ne += k
            if t != Pl - 1 and t != Pl + Tl - 1:
                Rn = n * Rp if t < Pl else n  # R = 1, R^+ = Rp
                flow, cost, k = oracle.random_search(Da[level], Db[level], n, Rn, seed, 0, level, t, flow, cost,
                                                     nthreads=4)
                ne += k
    assert np.array_equal(o["flow_fwd"], flow)
    assert np.array_equal(o["cost_fwd"], cost)
    assert o["n_evals"][0] == ne


def test_fast_with_all_steps_at_the_finest_scale_is_the_original_schedule():
    """Without an R^+ group, Fast with Tfine = T is the original schedule."""
    p = make_pair(1)
    a = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4)
    b = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4, fine_iters=4)
    for k in ("flow_fwd", "flow_bwd", "cost_fwd", "cost_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(a[k], b[k])
    assert a["n_evals"] == b["n_evals"]


@pytest.mark.parametrize("t", [(6, -4), (-11, 3)])
def test_flow_fields_plus_recovers_an_integer_translation(t):
    img1, img2 = translated_crops(71, 56, 72, t[0], t[1])
    o = oracle.flow_fields(img1, img2, 3, 8, nthreads=2, plus_iters=4, Rp_num=2)
    H, W = img1.shape
    m = 7
    ys, xs = np.mgrid[0:H, 0:W]
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    f = o["flow_fwd"]
    assert np.all(f[inner][:, 0] == t[0]) and np.all(f[inner][:, 1] == t[1])
    assert np.all(o["cost_fwd"][inner] == 0)


def test_flow_fields_plus_evaluation_count_bound():
    """At most 2 evaluations per cell and step, 1 per random search (P - 1
    + T - 1 of them) and 1 seed evaluation per cell and scale."""
    p = make_pair(1)
    L, T, P = 3, 8, 4
    o = oracle.flow_fields(p.img1, p.img2, L, T, nthreads=4, plus_iters=P, Rp_num=2)
    H, W = p.img1.shape
    bound = 0
    for lv in range(L):
        n = 1 << lv
        cells = (-(-W // n)) * (-(-H // n))
        bound += cells * (2 * (P + T) + (P - 1) + (T - 1)) + cells
    assert 0 < min(o["n_evals"]) and max(o["n_evals"]) <= bound


def test_flow_fields_plus_rejects_bad_schedules():
    img, _ = random_images(3, 20, 20)
    for kw in ({"plus_iters": -1}, {"fine_iters": -2}, {"plus_iters": 60, "Rp_num": 2}, {"Rp_num": -1}):
        with pytest.raises(ValueError):
            oracle.flow_fields(img, img, 2, 8, **kw)


# ---------------------------------------------------------------- two backward fields (Sec. 3.7)

def test_consistency2_closed_form():
    """Constructed fields: a pixel consistent with only one backward field is
    deleted; UNSET targets in either field delete; both consistent keeps."""
    H, W = 3, 4
    fa = np.zeros((H, W, 2), np.int16)
    ca = np.zeros((H, W), np.uint32)
    fa[0, 0] = (1, 0)   # -> (1, 0): b1 returns (-1, 0), b2 returns (-1, 1): |(0, 1)| = 1, not < 1
    fa[1, 1] = (2, 1)   # -> (3, 2): both return (-2, -1)
    fa[2, 0] = (0, -2)  # -> (0, 0): b2 UNSET there
    ca[0, 1] = oracle.UNSET
    fb1 = np.zeros((H, W, 2), np.int16)
    fb2 = np.zeros((H, W, 2), np.int16)
    cb1 = np.zeros((H, W), np.uint32)
    cb2 = np.zeros((H, W), np.uint32)
    fb1[0, 1] = (-1, 0)
    fb2[0, 1] = (-1, 1)
    fb1[2, 3] = fb2[2, 3] = (-2, -1)
    fb1[0, 0] = (0, 2)
    cb2[0, 0] = oracle.UNSET
    keep = oracle.consistency2(fa, ca, fb1, cb1, fb2, cb2, 1.0)
    assert keep[1, 1] == 1  # consistent with both
    assert keep[0, 0] == 0  # consistent with b1 only (residual (0, 1) against b2)
    assert keep[2, 0] == 0  # its target (0, 0) is UNSET in b2
    assert keep[0, 1] == 0  # UNSET in a
    assert keep[1, 0] == 1 and keep[2, 2] == 1  # zero flows meeting zero flows
    assert keep[2, 3] == 0  # zero flow meeting (-2, -1) in both
    keep15 = oracle.consistency2(fa, ca, fb1, cb1, fb2, cb2, 1.5)
    assert keep15[0, 0] == 1  # |(0, 1)| < 1.5


@pytest.mark.parametrize("eps", [0.5, 1.0, 2.5])
def test_consistency2_is_both_single_checks(eps):
    """Deleted iff inconsistent with one of the two backward fields: the
    mask equals the AND of the two single checks (each pinned above)."""
    p = make_pair(1)
    o1 = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4)
    o2 = oracle.flow_fields(p.img2, p.img1, 3, 4, radius=2, seed=999, nthreads=4)
    k = oracle.consistency2(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], o2["flow_fwd"],
                            o2["cost_fwd"], eps)
    k1 = oracle.consistency(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], eps)
    k2 = oracle.consistency(o1["flow_fwd"], o1["cost_fwd"], o2["flow_fwd"], o2["cost_fwd"], eps)
    assert np.array_equal(k, k1 & k2)
    assert k.sum() < k1.sum()  # the second field deletes some pixels the first check kept


# ---------------------------------------------------------------- q x q sparsification (Sec. 3.8)

def _sparsify_numpy(fa, keep, fb1, fb2, q, e):
    """Brute force restated with NumPy: per region, the kept in-image
    candidates ordered by (summed error, pixel index)."""
    H, W = keep.shape
    ys, xs = np.mgrid[0:H, 0:W]
    tx, ty = xs + fa[..., 0], ys + fa[..., 1]
    inside = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H)
    txc, tyc = np.clip(tx, 0, W - 1), np.clip(ty, 0, H - 1)
    err = np.zeros((H, W))
    for fb in [fb1] + ([fb2] if fb2 is not None else []):
        d = fa.astype(np.float64) + fb[tyc, txc].astype(np.float64)
        err = err + np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    out = np.full((-(-H // q), -(-W // q)), -1, np.int32)
    for ry in range(out.shape[0]):
        for rx in range(out.shape[1]):
            sl = (slice(ry * q, ry * q + q), slice(rx * q, rx * q + q))
            k, cand = keep[sl].astype(bool), keep[sl].astype(bool) & inside[sl]
            if k.sum() < e or not cand.any():
                continue
            idx = (ys[sl] * W + xs[sl])[cand]
            order = np.lexsort((idx, err[sl][cand]))
            out[ry, rx] = idx[order[0]]
    return out


@pytest.mark.parametrize("q,e,two", [(3, 1, True), (3, 4, True), (4, 2, False), (2, 1, True), (5, 7, False)])
def test_sparsify_equals_numpy_brute_force(q, e, two):
    rng = np.random.default_rng(q * 10 + e)
    H, W = 23, 31
    fa = rng.integers(-3, 4, size=(H, W, 2)).astype(np.int16)
    fb1 = rng.integers(-3, 4, size=(H, W, 2)).astype(np.int16)
    fb2 = rng.integers(-3, 4, size=(H, W, 2)).astype(np.int16) if two else None
    keep = (rng.random((H, W)) < 0.6).astype(np.uint8)
    got = oracle.sparsify(fa, keep, fb1, fb2, q, e)
    assert np.array_equal(got, _sparsify_numpy(fa, keep, fb1, fb2, q, e))


def test_sparsify_hand_worked_region():
    """One 3x3 region: three kept samples with errors 1, sqrt(2), 1 against a
    single backward field: the earlier of the two at error 1 wins; with
    e = 4 the region is dropped; nothing kept gives -1."""
    fa = np.zeros((3, 3, 2), np.int16)
    fb = np.zeros((3, 3, 2), np.int16)
    keep = np.zeros((3, 3), np.uint8)
    keep[0, 2] = keep[1, 1] = keep[2, 0] = 1
    fb[0, 2] = (1, 0)   # error 1 at index 2
    fb[1, 1] = (1, 1)   # error sqrt(2) at index 4
    fb[2, 0] = (0, -1)  # error 1 at index 6
    assert oracle.sparsify(fa, keep, fb, None, 3, 1)[0, 0] == 2
    assert oracle.sparsify(fa, keep, fb, None, 3, 3)[0, 0] == 2
    assert oracle.sparsify(fa, keep, fb, None, 3, 4)[0, 0] == -1
    assert oracle.sparsify(fa, np.zeros_like(keep), fb, None, 3, 0)[0, 0] == -1
    fb2 = np.zeros_like(fb)
    fb2[0, 2] = (2, 0)  # index 2 now sums 3, index 6 sums 1 + 0
    assert oracle.sparsify(fa, keep, fb, fb2, 3, 1)[0, 0] == 6


def test_sparsify_on_a_field_selects_kept_samples_of_least_error():
    p = make_pair(1)
    o = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4)
    H, W = p.img1.shape
    sel = oracle.sparsify(o["flow_fwd"], o["keep_fwd"], o["flow_bwd"], None, 3, 2)
    assert (sel >= 0).sum() > 0.5 * sel.size
    for ry, rx in zip(*np.nonzero(sel >= 0)):
        k = int(sel[ry, rx])
        y, x = divmod(k, W)
        assert y // 3 == ry and x // 3 == rx and o["keep_fwd"][y, x] == 1
        # kept samples passed the check: |F + F_b|^2 < 1, so the error is 0 (integer flows)
        f = o["flow_fwd"][y, x].astype(int)
        assert np.all(f + o["flow_bwd"][y + f[1], x + f[0]] == 0)


# ---------------------------------------------------------------- region filter (Sec. 3.7)

def _region_filter_union_find(flow, cost, keep, s):
    """Independent restatement: union-find over the kept pixels' linked
    4-neighbour pairs, then the size and removed-outlier tests per region."""
    H, W = keep.shape
    parent = list(range(H * W))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    f = flow.astype(np.int64)

    def linked(a, b):
        d = f[a // W, a % W] - f[b // W, b % W]
        return int(d[0] ** 2 + d[1] ** 2) < 9

    for y in range(H):
        for x in range(W):
            a = y * W + x
            for b in ([a + 1] if x + 1 < W else []) + ([a + W] if y + 1 < H else []):
                if keep[y, x] and keep.flat[b] and linked(a, b):
                    parent[find(a)] = find(b)
    size, touch = {}, {}
    for y in range(H):
        for x in range(W):
            if not keep[y, x]:
                continue
            a = y * W + x
            r = find(a)
            size[r] = size.get(r, 0) + 1
            for nx, ny in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                if 0 <= nx < W and 0 <= ny < H and not keep[ny, nx] and cost[ny, nx] != UNSET and \
                        linked(a, ny * W + nx):
                    touch[r] = True
    out = keep.copy()
    for y in range(H):
        for x in range(W):
            if keep[y, x]:
                r = find(y * W + x)
                if size[r] < s and touch.get(r, False):
                    out[y, x] = 0
    return out


@pytest.mark.parametrize("seed,s", [(1, 5), (2, 12), (3, 40), (4, 1)])
def test_region_filter_equals_union_find(seed, s):
    rng = np.random.default_rng(seed)
    H, W = 19, 27
    flow = rng.integers(-4, 5, size=(H, W, 2)).astype(np.int16)
    flow[: H // 2] = rng.integers(-1, 2, size=(H // 2, W, 2))  # smooth part: large regions
    cost = rng.integers(0, 100, size=(H, W)).astype(np.uint32)
    cost[rng.random((H, W)) < 0.05] = UNSET
    keep = ((rng.random((H, W)) < 0.7) & (cost != UNSET)).astype(np.uint8)
    got = oracle.region_filter(flow, cost, keep, s)
    assert np.array_equal(got, _region_filter_union_find(flow, cost, keep, s))


def test_region_filter_constant_flow_is_connected_components():
    """With one flow everywhere every 4-neighbour pair links: the regions are
    the 4-connected components of the mask (scipy.ndimage.label), and a
    component is deleted iff it is smaller than s and borders a removed
    (set, not kept) pixel."""
    rng = np.random.default_rng(7)
    H, W = 30, 40
    keep = (rng.random((H, W)) < 0.55).astype(np.uint8)
    flow = np.zeros((H, W, 2), np.int16)
    cost = np.zeros((H, W), np.uint32)
    cost[::3, ::4] = UNSET
    s = 6
    lab, n = ndi.label(keep)
    removed = (keep == 0) & (cost != UNSET)
    grown = ndi.binary_dilation(removed, structure=ndi.generate_binary_structure(2, 1))
    expect = keep.copy()
    for c in range(1, n + 1):
        m = lab == c
        if m.sum() < s and (m & grown).any():
            expect[m] = 0
    assert np.array_equal(oracle.region_filter(flow, cost, keep, s), expect)


def test_region_filter_hand_worked():
    """A 2-pixel region next to a removed outlier of similar flow is deleted;
    next to one of dissimilar flow (difference 3 px) it stays; s = 2 keeps it."""
    flow = np.zeros((1, 4, 2), np.int16)
    cost = np.zeros((1, 4), np.uint32)
    keep = np.array([[1, 1, 0, 1]], np.uint8)
    flow[0, 2] = (2, 2)  # removed outlier, |diff| = sqrt(8) < 3 from (0, 0)
    flow[0, 3] = (7, 0)  # lone kept pixel, dissimilar to the outlier ((2, 2): 29, (3, 0): 16)
    out = oracle.region_filter(flow, cost, keep, 3)
    assert out.tolist() == [[0, 0, 0, 1]]
    flow[0, 2] = (3, 0)  # now |diff| = 3: not below 3 px
    assert oracle.region_filter(flow, cost, keep, 3).tolist() == [[1, 1, 0, 1]]
    flow[0, 2] = (2, 2)
    assert oracle.region_filter(flow, cost, keep, 2).tolist() == [[1, 1, 0, 1]]
    cost[0, 2] = UNSET  # an UNSET pixel is no removed outlier
    assert oracle.region_filter(flow, cost, keep, 3).tolist() == [[1, 1, 0, 1]]


def test_outlier_chain_masks_only_shrink():
    """Consistency against one, then two backward fields, then the region
    filter: each step keeps a subset of the previous mask; the sparse
    samples are kept pixels, one per region at most."""
    p = make_pair(1)
    o1 = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=4)
    o2 = oracle.flow_fields(p.img2, p.img1, 3, 4, radius=2, seed=4321, nthreads=4)
    k1 = o1["keep_fwd"]
    k2 = oracle.consistency2(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], o2["flow_fwd"],
                             o2["cost_fwd"])
    k3 = oracle.region_filter(o1["flow_fwd"], o1["cost_fwd"], k2, 30)
    assert np.all(k2 <= k1) and np.all(k3 <= k2) and k3.sum() > 0
    sel = oracle.sparsify(o1["flow_fwd"], k3, o1["flow_bwd"], o2["flow_fwd"], 3, 1)
    picked = sel[sel >= 0]
    assert len(np.unique(picked)) == len(picked)
    assert np.all(k3.ravel()[picked] == 1)
