"""Flow Fields+ Fast x2 (Sec. 3.4) on the GPU, bit for bit against the
oracle: whole fields, costs, masks and evaluation counts on the grid of
scale 2 (small, ragged and tiny frames, with the Flow Fields+ step groups,
with the seed rerank and with serial-order propagation, the 160x120 and
1024x436 workloads), and the grid check on its own."""
import os

import numpy as np
import pytest

import oracle
import paper_1703_02563_amd as ff
from ffgen import CONFIG_PARAMS, make_pair, random_images
from test_gpu_parity import as_u32, dev, host

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def _compare(g, o):
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(host(g[k]), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(as_u32(g[k]), o[k]), k
    assert tuple(int(v) for v in host(g["n_evals"])) == o["n_evals"]


def _run(ia, ib, L, T, **kw):
    prm = ff.Params(levels=L, iters=T, fast_x2=True, **kw)
    o = oracle.flow_fields(ia, ib, L, T, nthreads=NT, fast_x2=True, **kw)
    g = ff.flow_fields(dev(ia), dev(ib), prm)
    return g, o


@pytest.mark.parametrize("shape,L,T,kw", [((96, 128), 3, 4, {}),
                                         ((61, 95), 3, 8, dict(plus_iters=4, Rp_num=2, fine_iters=4)),
                                         ((5, 7), 2, 2, {}), ((33, 2), 2, 3, dict(fine_iters=1)),
                                         ((70, 90), 4, 4, dict(nn_l=8)), ((50, 66), 3, 3, dict(raster=True)),
                                         ((44, 60), 2, 4, dict(radius=2))])
def test_fast_x2_fields_bit_exact(shape, L, T, kw):
    H, W = shape
    ia, ib = random_images(2100 + H + W, H, W)
    g, o = _run(ia, ib, L, T, **kw)
    assert host(g["flow_fwd"]).shape == (-(-H // 2), -(-W // 2), 2)
    _compare(g, o)


def test_fast_x2_config1_bit_exact():
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    g, o = _run(p.img1, p.img2, c.levels, 8, plus_iters=4, Rp_num=2, fine_iters=4)
    _compare(g, o)
    assert o["keep_fwd"].mean() > 0.3  # the layers' matches survive the region check


def test_fast_x2_full_size_bit_exact():
    """1024x436, 5 scales with the paper's Flow Fields+ Fast x2 steps (4 at
    R^+ = 2R and 8 at R on the coarser scales, 4 at R on scale 2)."""
    p = make_pair(2)
    g, o = _run(p.img1, p.img2, 5, 8, plus_iters=4, Rp_num=2, fine_iters=4)
    _compare(g, o)


@pytest.mark.parametrize("n", [1, 2, 4])
def test_grid_check_bit_exact(n):
    rng = np.random.default_rng(n)
    H, W = 57, 83
    Hn, Wn = -(-H // n), -(-W // n)
    ys, xs = np.mgrid[0:Hn, 0:Wn] * n
    fl = []
    for _ in range(2):
        tx = rng.integers(0, W, size=(Hn, Wn))
        ty = rng.integers(0, H, size=(Hn, Wn))
        f = np.stack([tx - xs, ty - ys], -1).astype(np.int16)
        c = rng.integers(0, 999, size=(Hn, Wn)).astype(np.uint32)
        c[rng.random((Hn, Wn)) < 0.2] = oracle.UNSET
        fl.append((f, c))
    (fa, ca), (fb, cb) = fl
    for j in range(Hn):  # half of the forward matches point back (within one pixel)
        for i in range(0, Wn, 2):
            t = (xs[j, i] + fa[j, i, 0], ys[j, i] + fa[j, i, 1])
            fb[t[1] // n, t[0] // n] = -fa[j, i] + rng.integers(-1, 2, size=2)
    ea = oracle.consistency_grid(fa, ca, fb, cb, W, H, n)
    eb = oracle.consistency_grid(fb, cb, fa, ca, W, H, n)
    ka, kb = ff.consistency_filter_grid(dev(fa), dev(ca.view(np.int32)), dev(fb), dev(cb.view(np.int32)), W, H, n)
    assert np.array_equal(host(ka), ea) and np.array_equal(host(kb), eb)
    assert 0 < ea.sum() < ea.size


def test_fast_x2_needs_two_scales():
    ia, ib = random_images(5, 20, 24)
    with pytest.raises(ff.FlowFieldsError):
        ff.flow_fields(dev(ia), dev(ib), ff.Params(levels=1, iters=2, fast_x2=True))
    with pytest.raises(ff.FlowFieldsError):
        ff.flow_fields(dev(ia), dev(ib), ff.Params(levels=2, iters=2, fast_x2=True, subpixel=3))
