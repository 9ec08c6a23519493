"""The temporally blocked level kernels at patch radii 2 and 4 (the second
backward field's r2 = 2 of the conference setting and the radius r = 4 of
Flow Fields+ with r2 = 3, Sec. 3.7 and 4.1), bit for bit against the
oracle: every launch-table index (each maps to a descriptor-quad kernel of
the same window halo), every run length, whole fields on small, ragged and
full-size frames, one scale through ff_run_level, and the check against two
backward fields."""
import os

import numpy as np
import pytest

import oracle
import paper_1703_02563_amd as ff
from ffgen import CONFIG_PARAMS, make_pair, random_images
from test_gpu_parity import as_u32, counter, dev, host, to_lib
from tuning_util import with_tuning

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def _compare(g, o):
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(host(g[k]), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(as_u32(g[k]), o[k]), k
    assert tuple(int(v) for v in host(g["n_evals"])) == o["n_evals"]


@pytest.mark.parametrize("radius", [2, 4])
@pytest.mark.parametrize("shape,L,T", [((96, 128), 3, 4), ((61, 95), 4, 6), ((5, 7), 2, 2), ((1, 1), 1, 1),
                                      ((33, 2), 2, 3)])
def test_radius_fields_bit_exact(shape, L, T, radius):
    H, W = shape
    ia, ib = random_images(2500 + H + W, H, W)
    o = oracle.flow_fields(ia, ib, L, T, radius, nthreads=NT)
    _compare(ff.flow_fields(dev(ia), dev(ib), ff.Params(levels=L, iters=T, radius=radius)), o)


@pytest.mark.parametrize("radius", [2, 4])
def test_radius_every_table_index_bit_exact(radius):
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    prm = ff.Params(levels=c.levels, iters=c.iters, radius=radius)
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, radius, nthreads=NT)
    for v in range(int(ff.lib().ff_level_variant_count())):
        for passes in (0, 1, 2):
            g = ff.flow_fields(dev(p.img1), dev(p.img2), with_tuning(prm, variant=[v] * 7, passes=[passes] * 7))
            for k in ("flow_fwd", "flow_bwd", "keep_fwd"):
                assert np.array_equal(host(g[k]), o[k]), (v, passes, k)
            assert np.array_equal(as_u32(g["cost_fwd"]), o["cost_fwd"]), (v, passes)
            assert tuple(int(x) for x in host(g["n_evals"])) == o["n_evals"], (v, passes)


@pytest.mark.parametrize("radius", [2, 4])
def test_radius_full_size_bit_exact(radius):
    p = make_pair(2)
    c = CONFIG_PARAMS[2]
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, radius, c.R_num, c.R_den, c.eps, c.seed, nthreads=NT)
    _compare(ff.flow_fields(dev(p.img1), dev(p.img2), ff.Params(levels=c.levels, iters=c.iters, radius=radius)), o)


def test_plus_radius4_full_size_bit_exact():
    """Flow Fields+ at the paper's radius r = 4 (4 steps at R^+ = 2R, 8 at R)."""
    p = make_pair(2)
    c = CONFIG_PARAMS[2]
    o = oracle.flow_fields(p.img1, p.img2, c.levels, 8, 4, nthreads=NT, plus_iters=4, Rp_num=2)
    _compare(ff.flow_fields(dev(p.img1), dev(p.img2),
                            ff.Params(levels=c.levels, iters=8, radius=4, plus_iters=4, Rp_num=2)), o)


@pytest.mark.parametrize("radius", [2, 4])
@pytest.mark.parametrize("level", [0, 1])
def test_radius_run_level_bit_exact(level, radius):
    """One scale from the coarser grid's seeds (mode 2) against the oracle's
    step sequence."""
    H, W, T = 61, 83, 4
    n = 1 << level
    ia, ib = random_images(2600 + level + radius, H, W)
    Da, Db = oracle.descriptor(oracle.blur(ia, n), n), oracle.descriptor(oracle.blur(ib, n), n)
    rng = np.random.default_rng(level)
    Wc, Hc = -(-W // (2 * n)), -(-H // (2 * n))
    ys, xs = np.mgrid[0:Hc, 0:Wc] * 2 * n
    cflow = np.stack([rng.integers(0, W, (Hc, Wc)) - xs, rng.integers(0, H, (Hc, Wc)) - ys], -1).astype(np.int16)
    ccost = rng.integers(0, 60000, size=(Hc, Wc)).astype(np.uint32)
    flow, cost, ne = oracle.seed_level(cflow, ccost, Da, Db, n, r=radius)
    for t in range(T):
        flow, cost, k = oracle.propagate(Da, Db, n, t, flow, cost, r=radius, nthreads=NT)
        ne += k
        if t < T - 1:
            flow, cost, k = oracle.random_search(Da, Db, n, n, 12345, 0, level, t, flow, cost, r=radius,
                                                 nthreads=NT)
            ne += k
    prm = ff.Params(levels=level + 1, iters=T, radius=radius)
    Wn, Hn = -(-W // n), -(-H // n)
    import torch
    gf = torch.empty((Hn, Wn, 2), dtype=torch.int16, device="cuda")
    gc = torch.empty((Hn, Wn), dtype=torch.int32, device="cuda")
    cnt = counter()
    ff.run_level(dev(to_lib(Da, n)), dev(to_lib(Db, n)), level, prm, 0, 2, gf, gc, coarse_flow=dev(cflow),
                 coarse_cost=dev(ccost.view(np.int32)), n_evals=cnt)
    assert np.array_equal(host(gf), flow)
    assert np.array_equal(as_u32(gc), cost)
    assert int(host(cnt)[0]) == ne


@pytest.mark.parametrize("r,r2", [(3, 2), (4, 3)])
def test_two_backward_fields_bit_exact(r, r2):
    """The check against two backward fields (the second with another seed
    and radius r2; the paper's pairs (3, 2) and (4, 3)), every field from the
    blocked kernels."""
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    prm = ff.Params(levels=c.levels, iters=c.iters, radius=r)
    g = ff.flow_fields_two_backward(dev(p.img1), dev(p.img2), prm, radius2=r2)
    o1 = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, r, nthreads=NT)
    o2 = oracle.flow_fields(p.img2, p.img1, c.levels, c.iters, r2, seed=prm.seed + 1, nthreads=NT)
    assert np.array_equal(host(g["flow_bwd2"]), o2["flow_fwd"])
    keep = oracle.consistency2(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], o2["flow_fwd"],
                               o2["cost_fwd"])
    assert np.array_equal(host(g["keep_fwd"]), keep)
