"""Pins of the oracle's Flow Fields+ Fast x2 (Sec. 3.4): the finest scale is
not run, the second finest runs only the Fast step count at R, the kd-tree
holds one pixel of every 2x2 region (read as the pixel with even x and y),
and each 2x2 region gets one match (the fields and masks live on the grid of
scale 2).  The pins: NumPy's sort of the distance matrix over the even
pixels, the composition of the separately pinned steps in the paper's
order, the full-resolution check on fields replicated over 2x2 regions,
exact recovery of an even integer translation, and the state invariants.
"""
import numpy as np
import pytest

import oracle
from ffgen import make_pair, random_images, translated_crops

UNSET = oracle.UNSET


def _desc1(img):
    return oracle.descriptor(oracle.blur(img, 1), 1)


@pytest.mark.parametrize("shape,nc,l", [((19, 23), 2, 8), ((26, 35), 4, 1), ((7, 9), 2, 8)])
def test_even_pixel_candidates_equal_the_sorted_distance_matrix(shape, nc, l):
    a, b = random_images(50 + nc, *shape, kind="uniform")
    Da, Db = _desc1(a), _desc1(b)
    H, W = a.shape
    idx, dist = oracle.nn_topl(Da, Db, nc, l, rstep=2)
    ys, xs = np.mgrid[0:H:2, 0:W:2]
    q = (ys * W + xs).ravel()
    B = Db.reshape(-1, 16)[q].astype(np.int64)
    for j in range(idx.shape[0]):
        for i in range(idx.shape[1]):
            d = ((B - Da[j * nc, i * nc].astype(np.int64)) ** 2).sum(1)
            order = np.lexsort((q, d))[:l]
            k = order.size
            assert np.array_equal(idx[j, i, :k], q[order]) and np.array_equal(dist[j, i, :k], d[order])
            assert np.all(idx[j, i, k:] == -1)


def test_grid_check_at_scale_1_is_the_pixel_check():
    a, b = random_images(9, 30, 41)
    o = oracle.flow_fields(a, b, 3, 4, nthreads=2)
    H, W = a.shape
    k = oracle.consistency_grid(o["flow_fwd"], o["cost_fwd"], o["flow_bwd"], o["cost_bwd"], W, H, 1)
    assert np.array_equal(k, o["keep_fwd"])


def test_grid_check_is_the_pixel_check_of_fields_replicated_over_regions():
    """A field on the grid of scale 2 stands for its 2x2 regions: replicate
    both fields over their regions and the full-resolution check at the
    region anchors (even pixels) gives the grid check."""
    rng = np.random.default_rng(3)
    H, W = 31, 44
    Hn, Wn = -(-H // 2), -(-W // 2)
    ys, xs = np.mgrid[0:Hn, 0:Wn] * 2
    fields = []
    for s in range(2):
        tx = rng.integers(0, W, size=(Hn, Wn))
        ty = rng.integers(0, H, size=(Hn, Wn))
        f = np.stack([tx - xs, ty - ys], -1).astype(np.int16)
        c = rng.integers(0, 1000, size=(Hn, Wn)).astype(np.uint32)
        c[rng.random((Hn, Wn)) < 0.1] = UNSET
        fields.append((f, c))
    # make many forward matches consistent: b's region at the target points back
    (fa, ca), (fb, cb) = fields
    for j in range(Hn):
        for i in range(0, Wn, 2):
            tx, ty = xs[j, i] + fa[j, i, 0], ys[j, i] + fa[j, i, 1]
            fb[ty // 2, tx // 2] = -fa[j, i] + rng.integers(-1, 2, size=2)
    grid = oracle.consistency_grid(fa, ca, fb, cb, W, H, 2)
    rep = lambda x: np.repeat(np.repeat(x, 2, 0), 2, 1)[:H, :W]
    full = oracle.consistency(np.ascontiguousarray(rep(fa)), np.ascontiguousarray(rep(ca)),
                              np.ascontiguousarray(rep(fb)), np.ascontiguousarray(rep(cb)))
    assert np.array_equal(grid, full[::2, ::2])
    assert 0 < grid.sum() < grid.size


@pytest.mark.parametrize("P,Rp,Tfine", [(4, 2, 4), (0, 0, 2), (2, 3, 0)])
def test_fast_x2_is_the_step_sequence_of_the_paper(P, Rp, Tfine):
    """The Fast x2 driver equals the composition of the separately pinned
    steps: seeds from the even pixels, scales n = 2^(L-1) .. 2, Flow
    Fields+ groups on every scale but the second finest, which runs only
    Tfine steps at R (all P + T steps when Tfine = 0); no finest scale."""
    p = make_pair(1)
    L, T, seed = 3, 4, 4242
    o = oracle.flow_fields(p.img1, p.img2, L, T, seed=seed, nthreads=4, plus_iters=P, Rp_num=Rp,
                           fine_iters=Tfine, fast_x2=True)
    Da, Db = oracle.descriptors_all(p.img1, L), oracle.descriptors_all(p.img2, L)
    nc = 1 << (L - 1)
    cand, _ = oracle.nn_topl(Da[0], Db[0], nc, 1, nthreads=4, rstep=2)
    flow, cost, ne = oracle.init_coarse(np.ascontiguousarray(cand[..., 0]), Da[L - 1], Db[L - 1], nc)
    for level in range(L - 1, 0, -1):
        n = 1 << level
        if level < L - 1:
            flow, cost, k = oracle.seed_level(flow, cost, Da[level], Db[level], n)
            ne += k
        Pl, Tl = (0, Tfine) if (level == 1 and Tfine > 0) else (P, T)
        for t in range(Pl + Tl):
            flow, cost, k = oracle.propagate(Da[level], Db[level], n, t, flow, cost, nthreads=4)
            ne += k
            if t != Pl - 1 and t != Pl + Tl - 1:
                Rn = n * Rp if t < Pl else n
                flow, cost, k = oracle.random_search(Da[level], Db[level], n, Rn, seed, 0, level, t, flow, cost,
                                                     nthreads=4)
                ne += k
    assert np.array_equal(o["flow_fwd"], flow)
    assert np.array_equal(o["cost_fwd"], cost)
    assert o["n_evals"][0] == ne


@pytest.mark.parametrize("t", [(6, -4), (-10, 8)])
def test_fast_x2_recovers_an_even_translation(t):
    """An even translation maps every region anchor onto a region anchor, so
    the even-pixel seeds contain the exact matches; every interior cell of
    the scale-2 grid ends on the translation with cost 0 and passes the
    check."""
    img1, img2 = translated_crops(91, 60, 80, t[0], t[1])
    o = oracle.flow_fields(img1, img2, 4, 6, nthreads=4, plus_iters=4, Rp_num=2, fine_iters=4, fast_x2=True)
    H, W = img1.shape
    m = 14  # scale-2 patch (3 * 2) + descriptor (3 * 2) + blur, both ends inside both frames
    ys, xs = np.mgrid[0:H:2, 0:W:2]
    inner = (xs >= m) & (xs < W - m) & (ys >= m) & (ys < H - m)
    inner &= (xs + t[0] >= m) & (xs + t[0] < W - m) & (ys + t[1] >= m) & (ys + t[1] < H - m)
    f = o["flow_fwd"]
    assert inner.sum() > 200
    assert np.all(f[inner][:, 0] == t[0]) and np.all(f[inner][:, 1] == t[1])
    assert np.all(o["cost_fwd"][inner] == 0)
    assert np.all(o["keep_fwd"][inner] == 1)


def test_fast_x2_state_is_consistent():
    a, b = random_images(61, 33, 47)
    o = oracle.flow_fields(a, b, 3, 4, nthreads=2, fast_x2=True, fine_iters=2)
    H, W = a.shape
    D = [oracle.descriptor(oracle.blur(im, 2), 2) for im in (a, b)]
    for key, (A, B) in (("fwd", (D[0], D[1])), ("bwd", (D[1], D[0]))):
        f, c = o["flow_" + key], o["cost_" + key]
        assert f.shape == (-(-H // 2), -(-W // 2), 2)
        assert np.all(c != UNSET)
        for j in range(f.shape[0]):
            for i in range(f.shape[1]):
                x, y = 2 * i, 2 * j
                fx, fy = int(f[j, i, 0]), int(f[j, i, 1])
                assert 0 <= x + fx < W and 0 <= y + fy < H
                assert c[j, i] == oracle.cost(A, B, 2, 3, x, y, fx, fy)


def test_fast_x2_needs_two_scales():
    a, b = random_images(1, 20, 20)
    with pytest.raises(ValueError):
        oracle.flow_fields(a, b, 1, 2, fast_x2=True)
