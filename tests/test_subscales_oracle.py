"""Pins of the oracle's sub-scales (Sec. 3.3): stages whose patch size, blur
and random-search distance follow a sub-scale n* (not a power of two) while
propagation and random-search positions stay on the grid of an ordinary
scale n.  The pins: the paper's table of scales and sub-scales, the box
filter and descriptor spacing at n* = 3, 6, 12 against SciPy and NumPy
shifts, the patch cost on a grid of another scale, the composition of the
separately pinned steps, and recovery of an integer translation.
"""
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from ffgen import make_pair, random_images, translated_crops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNSET = oracle.UNSET


def test_stages_reproduce_the_papers_table():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "subscales_table.txt")) if not ln.startswith("#")]
    n, m = [list(map(int, r)) for r in rows]
    assert oracle.stages(4, subscales=True) == list(zip(n, m))
    # without sub-scales: the ordinary scales, n* = n
    assert oracle.stages(4) == [(8, 8), (4, 4), (2, 2), (1, 1)]


@pytest.mark.parametrize("m", [3, 6, 12])
def test_blur_at_a_subscale_is_the_library_box_filter(m):
    img, _ = random_images(70 + m, 41, 57, kind="uniform")
    h = max(1, m // 2)
    s = ndi.correlate(img.astype(np.int64), np.ones((2 * h + 1, 2 * h + 1), np.int64), mode="nearest")
    A = (2 * h + 1) ** 2
    assert np.array_equal(oracle.blur(img, m), ((s + A // 2) // A).astype(np.uint8))


@pytest.mark.parametrize("m", [3, 6])
def test_descriptor_at_a_subscale_samples_with_spacing_2m(m):
    b, _ = random_images(80 + m, 37, 45, kind="uniform")
    D = oracle.descriptor(b, m)
    H, W = b.shape
    ys, xs = np.mgrid[0:H, 0:W]
    for gy in range(4):
        for gx in range(4):
            yy = np.clip(ys + m * (2 * gy - 3), 0, H - 1)
            xx = np.clip(xs + m * (2 * gx - 3), 0, W - 1)
            assert np.array_equal(D[..., 4 * gy + gx], b[yy, xx])


def test_rescore_evaluates_the_patch_of_the_new_scale_on_the_same_grid():
    a, b = random_images(9, 40, 52)
    n, m = 4, 6
    Da, Db = [oracle.descriptor(oracle.blur(im, m), m) for im in (a, b)]
    H, W = a.shape
    Wn, Hn = -(-W // n), -(-H // n)
    rng = np.random.default_rng(2)
    ys, xs = np.mgrid[0:Hn, 0:Wn] * n
    flow = np.stack([rng.integers(0, W, (Hn, Wn)) - xs, rng.integers(0, H, (Hn, Wn)) - ys], -1).astype(np.int16)
    cost = np.zeros((Hn, Wn), np.uint32)
    cost[rng.random((Hn, Wn)) < 0.2] = UNSET
    c, ne = oracle.rescore(Da, Db, n, m, flow, cost)
    assert ne == int(np.count_nonzero(cost != UNSET))
    for j in range(Hn):
        for i in range(Wn):
            if cost[j, i] == UNSET:
                assert c[j, i] == UNSET
            else:
                assert c[j, i] == oracle.cost(Da, Db, m, 3, i * n, j * n, int(flow[j, i, 0]), int(flow[j, i, 1]))


@pytest.mark.parametrize("P,Rp,Tfine", [(4, 2, 0), (0, 0, 0), (2, 3, 2)])
def test_subscale_schedule_is_the_step_sequence_of_the_paper(P, Rp, Tfine):
    """The driver equals the composition of the pinned steps over the stages
    of the table: seeds at the coarsest scale; on a new grid the hand-over
    with costs at the stage's patch scale, on the same grid the costs moved
    to the new patch scale; Flow Fields+ steps with random-search distances
    R n* and R^+ n* at grid positions; the generator's level field log2 n,
    plus 16 on a sub-scale stage."""
    p = make_pair(1)
    L, T, seed, R = 3, 4, 99, 1
    o = oracle.flow_fields(p.img1, p.img2, L, T, seed=seed, nthreads=4, plus_iters=P, Rp_num=Rp, fine_iters=Tfine,
                           subscales=True)
    st = oracle.stages(L, subscales=True)
    assert st == [(4, 4), (2, 3), (2, 2), (1, 1)]
    D = {mm: [oracle.descriptor(oracle.blur(im, mm), mm) for im in (p.img1, p.img2)] for _, mm in st}
    D1 = [oracle.descriptor(oracle.blur(im, 1), 1) for im in (p.img1, p.img2)]
    nc = st[0][0]
    idx, _ = oracle.nn(D1[0], D1[1], nc, nthreads=4)
    flow, cost, ne = oracle.init_coarse(idx, D[nc][0], D[nc][1], nc)
    for k, (n, m) in enumerate(st):
        Da, Db = D[m]
        if k > 0 and n == st[k - 1][0]:
            cost, e = oracle.rescore(Da, Db, n, m, flow, cost)
            ne += e
        elif k > 0:
            flow, cost, e = oracle.seed_level_m(flow, cost, Da, Db, n, m)
            ne += e
        Pl, Tl = (0, Tfine) if (k == len(st) - 1 and Tfine > 0) else (P, T)
        gen = int(np.log2(n)) + (16 if m != n else 0)
        for t in range(Pl + Tl):
            flow, cost, e = oracle.propagate_m(Da, Db, n, m, t, flow, cost, nthreads=4)
            ne += e
            if t != Pl - 1 and t != Pl + Tl - 1:
                Rn = (Rp if t < Pl else R) * m
                flow, cost, e = oracle.random_search_m(Da, Db, n, m, Rn, seed, 0, gen, t, flow, cost, nthreads=4)
                ne += e
    assert np.array_equal(o["flow_fwd"], flow)
    assert np.array_equal(o["cost_fwd"], cost)
    assert o["n_evals"][0] == ne


@pytest.mark.parametrize("t", [(6, -4), (-11, 3)])
def test_subscales_recover_an_integer_translation(t):
    img1, img2 = translated_crops(71, 56, 72, t[0], t[1])
    o = oracle.flow_fields(img1, img2, 3, 8, nthreads=2, plus_iters=4, Rp_num=2, subscales=True)
    H, W = img1.shape
    m = 7
    ys, xs = np.mgrid[0:H, 0:W]
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    f = o["flow_fwd"]
    assert np.all(f[inner][:, 0] == t[0]) and np.all(f[inner][:, 1] == t[1])
    assert np.all(o["cost_fwd"][inner] == 0)


def test_subscales_change_the_field_and_exclude_fast_x2():
    a, b = random_images(5, 40, 56)
    base = oracle.flow_fields(a, b, 3, 4)
    sub = oracle.flow_fields(a, b, 3, 4, subscales=True)
    assert not np.array_equal(base["flow_fwd"], sub["flow_fwd"])
    assert sub["n_evals"][0] > base["n_evals"][0]  # one more stage per scale below the coarsest but the finest
    with pytest.raises(ValueError):
        oracle.flow_fields(a, b, 3, 4, subscales=True, fast_x2=True)
