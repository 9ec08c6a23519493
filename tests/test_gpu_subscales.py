"""Sub-scales (Sec. 3.3) on the GPU, bit for bit against the oracle: the
descriptor maps of the sub-scales n* = 3, 6, 12 (rows in image order), the
patch-scale change on one grid, and whole fields over the stages of the
table of scales and sub-scales (with the Flow Fields+ groups, the rerank,
serial order and the subpixel form; the 160x120 and 1024x436 workloads)."""
import os

import numpy as np
import pytest

import oracle
import paper_1703_02563_amd as ff
from ffgen import CONFIG_PARAMS, make_pair, random_images
from test_gpu_parity import _random_level_state, as_u32, counter, dev, host, to_lib
from tuning_util import with_tuning

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def to_lib_plain(D, m):
    """Row-major descriptors -> the map of a sub-scale m: replicated border
    of 4m pixels, the pixels of a row in image order."""
    P = 4 * m
    H, W = D.shape[:2]
    return np.ascontiguousarray(D[np.clip(np.arange(-P, H + P), 0, H - 1)][:, np.clip(np.arange(-P, W + P), 0, W - 1)])


@pytest.mark.parametrize("shape", [(37, 53), (1, 1), (120, 160), (9, 300)])
@pytest.mark.parametrize("m", [3, 6, 12])
def test_subscale_descriptors_bit_exact(shape, m):
    img, _ = random_images(300 + m, *shape, kind="uniform")
    blurred, desc, plain = ff.descriptors(dev(img), m, rowmajor=True)
    eb = oracle.blur(img, m)
    ed = oracle.descriptor(eb, m)
    assert np.array_equal(host(blurred), eb)
    assert np.array_equal(host(plain), ed)
    assert np.array_equal(host(desc), to_lib_plain(ed, m))


@pytest.mark.parametrize("n,m", [(4, 6), (2, 3), (8, 12), (2, 2)])
def test_rescore_bit_exact(n, m):
    H, W = 61, 83
    ia, ib = random_images(400 + m, H, W)
    Da, Db = [oracle.descriptor(oracle.blur(im, m), m) for im in (ia, ib)]
    flow, cost = _random_level_state(m, H, W, n)
    ec, ene = oracle.rescore(Da, Db, n, m, flow, cost)
    lay = (lambda D: to_lib(D, m)) if (m & (m - 1)) == 0 else (lambda D: to_lib_plain(D, m))
    gc, cnt = dev(cost.view(np.int32)), counter()
    ff.rescore_level(dev(lay(Da)), dev(lay(Db)), W, H, n, m, dev(flow), gc, n_evals=cnt)
    assert np.array_equal(as_u32(gc), ec)
    assert int(host(cnt)[0]) == ene


def _compare(g, o):
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(host(g[k]), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(as_u32(g[k]), o[k]), k
    assert tuple(int(v) for v in host(g["n_evals"])) == o["n_evals"]


def _run(ia, ib, L, T, **kw):
    prm = ff.Params(levels=L, iters=T, subscales=True, **kw)
    o = oracle.flow_fields(ia, ib, L, T, nthreads=NT, subscales=True, **kw)
    return ff.flow_fields(dev(ia), dev(ib), prm), o


@pytest.mark.parametrize("shape,L,T,kw", [((96, 128), 4, 4, {}),
                                         ((61, 95), 3, 8, dict(plus_iters=4, Rp_num=2, fine_iters=4)),
                                         ((5, 7), 3, 2, {}), ((33, 2), 2, 3, {}), ((1, 1), 1, 1, {}),
                                         ((70, 90), 4, 3, dict(nn_l=8)), ((50, 66), 3, 3, dict(raster=True)),
                                         ((44, 60), 3, 3, dict(subpixel=3)), ((40, 52), 3, 4, dict(radius=2))])
def test_subscale_fields_bit_exact(shape, L, T, kw):
    H, W = shape
    ia, ib = random_images(2300 + H + W, H, W)
    g, o = _run(ia, ib, L, T, **kw)
    _compare(g, o)


def test_subscale_stages_every_variant():
    """The (n, 3n/2) stages run on the blocked descriptor-quad kernel of the
    table's window halo: every variant of the table (one-lane, quad and
    weight-class entries, each mapped to its quad kernel) gives the oracle's
    fields, costs and counts."""
    H, W = 61, 95
    ia, ib = random_images(2417, H, W)
    kw = dict(plus_iters=4, Rp_num=2)
    o = oracle.flow_fields(ia, ib, 3, 6, nthreads=NT, subscales=True, **kw)
    for v in range(int(ff.lib().ff_level_variant_count())):
        for passes in (0, 2):
            prm = with_tuning(ff.Params(levels=3, iters=6, subscales=True, **kw), variant=[v] * 7,
                              passes=[passes] * 7)
            g = ff.flow_fields(dev(ia), dev(ib), prm)
            _compare(g, o)


def test_subscales_config1_bit_exact():
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    g, o = _run(p.img1, p.img2, c.levels, 8, plus_iters=4, Rp_num=2)
    _compare(g, o)


def test_subscales_full_size_bit_exact():
    """1024x436: stages (16,16) (8,12) (8,8) (4,6) (4,4) (2,3) (2,2) (1,1)
    with the paper's Flow Fields+ steps (4 at R^+ = 2R, 8 at R)."""
    p = make_pair(2)
    assert oracle.stages(5, subscales=True)[1] == (8, 12)
    g, o = _run(p.img1, p.img2, 5, 8, plus_iters=4, Rp_num=2)
    _compare(g, o)


def test_subscales_rejected_where_unsupported():
    ia, ib = random_images(7, 30, 40)
    with pytest.raises(ff.FlowFieldsError):
        ff.flow_fields(dev(ia), dev(ib), ff.Params(levels=3, iters=2, subscales=True, fast_x2=True))
