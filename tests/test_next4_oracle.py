"""Pins of the oracle's seed rerank (Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 4: the best
of the l candidates of a kd-tree leaf by matching error; leaf size l = 8 in
Sec. 4.1) and of its serial-order propagation step (Sec. 3.1, Eq. 2: a cell
is processed after its left and upper neighbours, so a flow can spread
anywhere within the 90-degree quadrant in one step, Fig. 3a).

The candidate set is read as the l nearest pixels by (squared descriptor
distance, linear index).  The pins: NumPy's lexicographic sort of the whole
distance matrix, NumPy's first-occurrence argmin over the pinned E_n, the
nesting of candidate sets in l, the quadrant reach of Fig. 3a on an exact
translation, and the per-cell fixed-point equations of the serial scan.
"""
import numpy as np
import pytest

import oracle
from ffgen import random_images, translated_crops

UNSET = oracle.UNSET


def _desc1(img):
    return oracle.descriptor(oracle.blur(img, 1), 1)


def _brute_topl(Da1, Db1, nc, l):
    H, W = Da1.shape[:2]
    Wc, Hc = oracle.core.cells(W, H, nc)
    B = Db1.reshape(-1, 16).astype(np.int64)
    idx = np.full((Hc, Wc, l), -1, np.int32)
    dist = np.full((Hc, Wc, l), np.iinfo(np.int64).max, np.int64)
    for j in range(Hc):
        for i in range(Wc):
            a = Da1[j * nc, i * nc].astype(np.int64)
            d = ((B - a) ** 2).sum(1)
            order = np.lexsort((np.arange(d.size), d))[:l]  # by distance, then index
            idx[j, i, :order.size] = order
            dist[j, i, :order.size] = d[order]
    return idx, dist


# ---------------------------------------------------------------- top-l candidates (Sec. 3.1, R28)

@pytest.mark.parametrize("kind,nc,l", [("uniform", 4, 8), ("box", 2, 8), ("levels", 4, 8), ("levels", 1, 3),
                                       ("box", 8, 16)])
def test_topl_equals_sorted_distance_matrix(kind, nc, l):
    if kind == "levels":
        # two grey levels: many exactly equal descriptors, so ties by index decide
        rng = np.random.default_rng(7)
        a = (rng.integers(0, 2, size=(19, 23)) * 200).astype(np.uint8)
        b = (rng.integers(0, 2, size=(19, 23)) * 200).astype(np.uint8)
    else:
        a, b = random_images(31 + nc, 19, 23, kind=kind)
    Da1, Db1 = _desc1(a), _desc1(b)
    idx, dist = oracle.nn_topl(Da1, Db1, nc, l)
    eidx, edist = _brute_topl(Da1, Db1, nc, l)
    assert np.array_equal(idx, eidx)
    assert np.array_equal(dist, edist)


def test_topl_fewer_pixels_than_candidates():
    a, b = random_images(3, 2, 3, kind="uniform")
    idx, dist = oracle.nn_topl(_desc1(a), _desc1(b), 1, 8)
    assert np.all(idx[..., 6:] == -1) and np.all(dist[..., 6:] == np.iinfo(np.int64).max)
    assert np.all(np.sort(idx[..., :6], axis=-1) == np.arange(6))


def test_top1_is_the_nearest_neighbour():
    a, b = random_images(5, 29, 37, kind="box")
    Da1, Db1 = _desc1(a), _desc1(b)
    idx1, d1 = oracle.nn(Da1, Db1, 4)
    idx, dist = oracle.nn_topl(Da1, Db1, 4, 8)
    assert np.array_equal(idx[..., 0], idx1) and np.array_equal(dist[..., 0], d1)


# ---------------------------------------------------------------- rerank (Eq. 1, Eq. 4)

@pytest.mark.parametrize("nc", [2, 4])
def test_rerank_is_first_argmin_of_patch_cost(nc):
    a, b = random_images(11 * nc, 26, 34, kind="box")
    Da1, Db1 = _desc1(a), _desc1(b)
    Dac, Dbc = [oracle.descriptor(oracle.blur(im, nc), nc) for im in (a, b)]
    cand, _ = oracle.nn_topl(Da1, Db1, nc, 8)
    flow, cost, ne = oracle.init_coarse_l(cand, Dac, Dbc, nc)
    H, W = a.shape
    assert ne == cand.size
    for j in range(cand.shape[0]):
        for i in range(cand.shape[1]):
            x, y = i * nc, j * nc
            e = [oracle.cost(Dac, Dbc, nc, 3, x, y, q % W - x, q // W - y) for q in cand[j, i]]
            k = int(np.argmin(e))  # first occurrence: the earlier rank wins ties
            q = int(cand[j, i, k])
            assert (flow[j, i, 0], flow[j, i, 1]) == (q % W - x, q // W - y)
            assert cost[j, i] == e[k]


def test_rerank_with_one_candidate_is_the_plain_seed():
    a, b = random_images(4, 21, 30, kind="box")
    Da1, Db1 = _desc1(a), _desc1(b)
    Dac, Dbc = [oracle.descriptor(oracle.blur(im, 4), 4) for im in (a, b)]
    idx, _ = oracle.nn(Da1, Db1, 4)
    f1, c1, n1 = oracle.init_coarse(idx, Dac, Dbc, 4)
    fl, cl, nl = oracle.init_coarse_l(idx[..., None], Dac, Dbc, 4)
    assert np.array_equal(f1, fl) and np.array_equal(c1, cl) and n1 == nl


def test_rerank_cost_never_rises_with_l():
    # candidate sets are nested prefixes of one ranking, so the best cost can only fall
    a, b = random_images(12, 33, 41, kind="box")
    Da1, Db1 = _desc1(a), _desc1(b)
    Dac, Dbc = [oracle.descriptor(oracle.blur(im, 4), 4) for im in (a, b)]
    cand, _ = oracle.nn_topl(Da1, Db1, 4, 8)
    prev = None
    for l in (1, 2, 4, 8):
        _, c, _ = oracle.init_coarse_l(np.ascontiguousarray(cand[..., :l]), Dac, Dbc, 4)
        if prev is not None:
            assert np.all(c <= prev)
        prev = c
    assert np.any(prev < oracle.init_coarse_l(np.ascontiguousarray(cand[..., :1]), Dac, Dbc, 4)[1])


# ---------------------------------------------------------------- serial-order propagation (Eq. 2, R29)

_SOURCES = {0: (-1, -1), 1: (+1, +1), 2: (+1, -1), 3: (-1, +1)}  # (horizontal di, vertical dj)


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_raster_step_fills_the_whole_quadrant(d):
    """Fig. 3a: one correct seed on an exact translation spreads to every
    interior cell of its quadrant in ONE serial step, and to no cell outside
    it."""
    H, W, t = 40, 52, (3, -2)
    a, b = translated_crops(21 + d, H, W, *t)
    Da, Db = oracle.descriptor(oracle.blur(a, 1), 1), oracle.descriptor(oracle.blur(b, 1), 1)
    bad = (-4, 5)
    flow = np.empty((H, W, 2), np.int16)
    flow[..., 0], flow[..., 1] = bad
    cost = np.array([[oracle.cost(Da, Db, 1, 3, x, y, *bad) for x in range(W)] for y in range(H)], np.uint32)
    i0, j0 = 26, 20
    flow[j0, i0] = t
    cost[j0, i0] = oracle.cost(Da, Db, 1, 3, i0, j0, *t)
    assert cost[j0, i0] == 0
    f, c, _ = oracle.propagate_raster(Da, Db, 1, d, flow, cost)
    hdi, vdj = _SOURCES[d]
    m = 8  # blur 1 + descriptor 3 + patch 3, plus one: reads of both ends stay inside both frames
    inside = lambda x, y: m <= x < W - m and m <= y < H - m and m <= x + t[0] < W - m and m <= y + t[1] < H - m
    in_quad = lambda i, j: (i - i0) * hdi <= 0 and (j - j0) * vdj <= 0
    reached = 0
    for j in range(H):
        for i in range(W):
            if in_quad(i, j) and inside(i, j):
                assert tuple(f[j, i]) == t and c[j, i] == 0, (i, j)
                reached += 1
            elif not in_quad(i, j):
                assert tuple(f[j, i]) == bad, (i, j)
    assert reached >= 100


def test_checkerboard_step_does_not_reach_as_far():
    # the same seed with the checkerboard step of R1 stays within a few cells
    H, W, t = 40, 52, (3, -2)
    a, b = translated_crops(21, H, W, *t)
    Da, Db = oracle.descriptor(oracle.blur(a, 1), 1), oracle.descriptor(oracle.blur(b, 1), 1)
    bad = (-4, 5)
    flow = np.empty((H, W, 2), np.int16)
    flow[..., 0], flow[..., 1] = bad
    cost = np.array([[oracle.cost(Da, Db, 1, 3, x, y, *bad) for x in range(W)] for y in range(H)], np.uint32)
    flow[20, 26] = t
    cost[20, 26] = 0
    f, _, _ = oracle.propagate(Da, Db, 1, 0, flow, cost)
    took = np.argwhere(np.all(f == np.array(t, np.int16), axis=-1))
    assert np.abs(took - np.array([20, 26])).sum(1).max() <= 2


def _random_state(seed, Da, Db, n, unset_frac=0.3, R=6):
    H, W = Da.shape[:2]
    Wn, Hn = oracle.core.cells(W, H, n)
    rng = np.random.default_rng(seed)
    flow = np.zeros((Hn, Wn, 2), np.int16)
    cost = np.full((Hn, Wn), UNSET, np.uint32)
    for j in range(Hn):
        for i in range(Wn):
            if rng.random() < unset_frac:
                continue
            x, y = i * n, j * n
            fx = int(np.clip(x + rng.integers(-R, R + 1), 0, W - 1)) - x
            fy = int(np.clip(y + rng.integers(-R, R + 1), 0, H - 1)) - y
            flow[j, i] = (fx, fy)
            cost[j, i] = oracle.cost(Da, Db, n, 3, x, y, fx, fy)
    return flow, cost


@pytest.mark.parametrize("d", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [1, 2])
def test_raster_step_solves_the_serial_fixed_point(d, n):
    """Each cell's result is the strict-< best of its own input value and the
    two source cells' RESULTS (the defining property of processing the
    sources first), checked cell by cell from the outputs alone."""
    a, b = random_images(40 + d + 4 * n, 27, 33, kind="box")
    Da = oracle.descriptor(oracle.blur(a, n), n)
    Db = oracle.descriptor(oracle.blur(b, n), n)
    flow, cost = _random_state(d + 10 * n, Da, Db, n)
    f, c, ne = oracle.propagate_raster(Da, Db, n, d, flow, cost)
    H, W = a.shape
    Hn, Wn = cost.shape
    hdi, vdj = _SOURCES[d]
    count = 0
    for j in range(Hn):
        for i in range(Wn):
            bc, bf = int(cost[j, i]), tuple(int(v) for v in flow[j, i])
            for si, sj in ((i + hdi, j), (i, j + vdj)):
                if not (0 <= si < Wn and 0 <= sj < Hn) or c[sj, si] == UNSET:
                    continue
                fs = tuple(int(v) for v in f[sj, si])
                if bc != UNSET and fs == bf:
                    continue
                x, y = i * n, j * n
                if not (0 <= x + fs[0] < W and 0 <= y + fs[1] < H):
                    continue
                e = oracle.cost(Da, Db, n, 3, x, y, *fs)
                count += 1
                if e < bc:
                    bc, bf = e, fs
            assert c[j, i] == bc and tuple(f[j, i]) == bf, (i, j)
    assert ne == count


def test_raster_schedule_state_is_consistent():
    # every set cell's stored cost is E_1 of its flow; targets stay inside
    a, b = random_images(77, 30, 44, kind="box")
    out = oracle.flow_fields(a, b, levels=3, iters=4, raster=True, nn_l=8)
    H, W = a.shape
    Da, Db = _desc1(a), _desc1(b)
    for key, (A, B) in (("fwd", (Da, Db)), ("bwd", (Db, Da))):
        f, c = out["flow_" + key], out["cost_" + key]
        assert np.all(c != UNSET)
        for j in range(0, H, 3):
            for i in range(0, W, 3):
                fx, fy = int(f[j, i, 0]), int(f[j, i, 1])
                assert 0 <= i + fx < W and 0 <= j + fy < H
                assert c[j, i] == oracle.cost(A, B, 1, 3, i, j, fx, fy)


def test_default_options_reproduce_the_plain_schedule():
    a, b = random_images(78, 24, 31, kind="box")
    base = oracle.flow_fields(a, b, levels=3, iters=4)
    ext = oracle.lib()
    H, W = a.shape
    outs = {k: np.empty_like(v) for k, v in base.items() if k != "n_evals"}
    ne = np.zeros(2, np.uint64)
    p = oracle.core._p
    rc = ext.or_flow_fields_x(p(np.ascontiguousarray(a)), p(np.ascontiguousarray(b)), W, H, 3, 4, 3, 1, 1, 0, 0, 0,
                              0, 1, 0, 0, 0, 1.0, 12345, 1, p(outs["flow_fwd"]), p(outs["flow_bwd"]), p(outs["cost_fwd"]),
                              p(outs["cost_bwd"]), p(outs["keep_fwd"]), p(outs["keep_bwd"]), p(ne))
    assert rc == 0
    for k, v in outs.items():
        assert np.array_equal(v, base[k]), k
    assert tuple(int(v) for v in ne) == base["n_evals"]


def test_topl_and_raster_change_the_field():
    a, b = random_images(79, 30, 40, kind="box")
    base = oracle.flow_fields(a, b, levels=3, iters=4)
    top = oracle.flow_fields(a, b, levels=3, iters=4, nn_l=8)
    ras = oracle.flow_fields(a, b, levels=3, iters=4, raster=True)
    assert not np.array_equal(top["flow_fwd"], base["flow_fwd"])
    assert not np.array_equal(ras["flow_fwd"], base["flow_fwd"])


def test_rerank_ties_go_to_the_earlier_rank():
    """Image b repeats a pattern with period 9 px in x, so pixels 9 px apart
    have equal descriptors and, inside the frame, equal patch costs: such
    candidates sit next to each other in the ranking (equal distance, index
    order) and the rerank must keep the earlier one."""
    rng = np.random.default_rng(5)
    pat = rng.integers(0, 256, size=(30, 9)).astype(np.uint8)
    b = np.tile(pat, (1, 6))
    a = np.roll(b, 2, axis=1)
    a[:, :4] = rng.integers(0, 256, size=(30, 4))
    Da1, Db1 = _desc1(a), _desc1(b)
    nc = 2
    Dac, Dbc = [oracle.descriptor(oracle.blur(im, nc), nc) for im in (a, b)]
    cand, dist = oracle.nn_topl(Da1, Db1, nc, 8)
    flow, cost, _ = oracle.init_coarse_l(cand, Dac, Dbc, nc)
    H, W = a.shape
    ties = 0
    for j in range(cand.shape[0]):
        for i in range(cand.shape[1]):
            x, y = i * nc, j * nc
            e = np.array([oracle.cost(Dac, Dbc, nc, 3, x, y, q % W - x, q // W - y) for q in cand[j, i]])
            k = int(np.flatnonzero(e == e.min())[0])
            if np.count_nonzero(e == e.min()) > 1:
                ties += 1
            q = int(cand[j, i, k])
            assert tuple(int(v) for v in flow[j, i]) == (q % W - x, q // W - y)
    assert ties >= 20
