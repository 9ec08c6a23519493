"""Flow Fields+ (Sec. 3.3) and Flow Fields+ Fast (Sec. 3.4) schedules on
every GPU path, bit for bit against the oracle, whose schedule is pinned
against the composition of its pinned steps: P steps with random searches at
R^+ first, then T at R, random searches only inside a group, the step index
running on over both groups; Fast: only the given number of steps at R on the
finest scale.  Also the check against two backward fields and the region
filter (Sec. 3.7) and the q x q sparsification (Sec. 3.8)."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1703_02563_amd as ff
from tuning_util import with_tuning
from ffgen import CONFIG_PARAMS, batch_shapes, make_pair, random_images
from paper_1703_02563_amd.batch import BatchFlowFields
from test_gpu_parity import _compare_full, _random_level_state, as_u32, counter, dev, host, to_lib
from test_learned_oracle import feature_canvas, feature_pyramid

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))
KEYS = ("flow_fwd", "flow_bwd", "cost_fwd", "cost_bwd", "keep_fwd", "keep_bwd", "n_evals")

# (plus_iters, Rp_num, iters, fine_iters): the paper's 4 x R+ then 8 x R, its
# Fast form, and short schedules with odd group ends
SCHEDULES = [(4, 2, 8, 0), (4, 2, 8, 4), (1, 3, 2, 0), (3, 2, 1, 2), (2, 4, 3, 1)]


def _params(config, sched, **kw):
    c = CONFIG_PARAMS[config]
    P, Rp, T, Tf = sched
    return ff.Params(levels=c.levels, iters=T, R_num=c.R_num, R_den=c.R_den, eps=c.eps, seed=c.seed,
                     plus_iters=P, Rp_num=Rp * c.R_num, fine_iters=Tf, **kw)


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("config", [1, 2])
def test_plus_schedules_bit_exact(config, sched):
    p = make_pair(config)
    print(f"plus schedule {sched} config {config}", flush=True)
    _compare_full(p.img1, p.img2, _params(config, sched))


@pytest.mark.parametrize("shape,L,R", [((1, 1), 1, (1, 1)), ((23, 1), 3, (1, 1)), ((31, 45), 3, (3, 2)),
                                       ((66, 97), 4, (2, 1))])
@pytest.mark.parametrize("sched", SCHEDULES[:3])
def test_plus_small_shapes(shape, L, R, sched):
    ia, ib = random_images(610 + L, *shape)
    P, Rp, T, Tf = sched
    _compare_full(ia, ib, ff.Params(levels=L, iters=T, R_num=R[0], R_den=R[1], plus_iters=P, Rp_num=Rp * R[0],
                                    fine_iters=Tf))


def test_plus_other_patch_radius():
    """Radius other than 3: the per-step path (one launch per step)."""
    ia, ib = random_images(710, 40, 56)
    for r in (1, 2):
        _compare_full(ia, ib, ff.Params(levels=2, iters=3, radius=r, plus_iters=2, Rp_num=2, fine_iters=2))


def test_plus_every_level_variant():
    """Each blocked variant and the step-wise schedule, with run lengths that
    end inside and at the border of the R^+ group."""
    p = make_pair(1)
    prm = _params(1, SCHEDULES[0])
    o = oracle.flow_fields(p.img1, p.img2, prm.levels, prm.iters, prm.radius, prm.R_num, prm.R_den, prm.eps,
                           prm.seed, nthreads=NT, plus_iters=prm.plus_iters, Rp_num=prm.Rp_num)
    for passes in (0, 3):
        for v in range(int(ff.lib().ff_level_variant_count())):
            pv = with_tuning(prm, variant=[v] * 7, passes=[passes] * 7)
            g = ff.flow_fields(dev(p.img1), dev(p.img2), pv)
            for k in ("flow_fwd", "flow_bwd", "keep_fwd"):
                assert np.array_equal(host(g[k]), o[k]), (passes, v, k)
            assert np.array_equal(as_u32(g["cost_bwd"]), o["cost_bwd"]), (passes, v)
            assert tuple(int(x) for x in host(g["n_evals"])) == o["n_evals"], (passes, v)


def test_plus_batch_equals_single_pair_path():
    c = CONFIG_PARAMS[4]
    prm = ff.Params(levels=c.levels, iters=8, plus_iters=4, Rp_num=2, fine_iters=4)
    shapes = batch_shapes()[:5]
    b = BatchFlowFields(shapes, prm)
    imgs = []
    for k, shp in enumerate(shapes):
        p = make_pair(4, k, shape=shp)
        i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
        imgs.append((p, i1, i2))
        b.set_pair(k, i1, i2)
    b.run()
    torch.cuda.synchronize()
    for k, (p, i1, i2) in enumerate(imgs):
        g = ff.flow_fields(i1, i2, prm)
        for key in KEYS:
            assert torch.equal(b.out[k][key], g[key]), (k, key)
    p, i1, i2 = imgs[0]
    o = oracle.flow_fields(p.img1, p.img2, prm.levels, prm.iters, nthreads=NT, plus_iters=4, Rp_num=2, fine_iters=4)
    assert np.array_equal(b.out[0]["flow_fwd"].cpu().numpy(), o["flow_fwd"])
    assert tuple(int(v) for v in b.out[0]["n_evals"].cpu()) == o["n_evals"]


@pytest.mark.parametrize("sched", [(4, 2, 8, 0), (2, 3, 3, 2)])
def test_plus_learned_features_bit_exact(sched):
    from paper_1703_02563_amd import learned as Lm
    H, W, pad, L = 61, 95, 10, 3
    canvas = feature_canvas(31, H + 2 * pad, W + 2 * pad)
    F1 = canvas[pad:pad + H, pad:pad + W].copy()
    F2 = canvas[pad - 2:pad - 2 + H, pad + 3:pad + 3 + W].copy() + feature_canvas(32, H, W) * 0.05
    m1, m2 = feature_pyramid(F1, L), feature_pyramid(F2, L)
    P, Rp, T, Tf = sched
    prm = ff.Params(levels=L, iters=T, plus_iters=P, Rp_num=Rp, fine_iters=Tf)
    o = oracle.flow_fields_f32(m1, m2, L, T, nthreads=NT, plus_iters=P, Rp_num=Rp, fine_iters=Tf)
    g = Lm.flow_fields_f32([torch.from_numpy(a).cuda() for a in m1], [torch.from_numpy(a).cuda() for a in m2], prm)
    torch.cuda.synchronize()
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(g[k].cpu().numpy(), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(g[k].cpu().numpy().view(np.uint32), o[k]), k
    assert tuple(int(v) for v in g["n_evals"].cpu()) == o["n_evals"]


@pytest.mark.parametrize("config,radius2", [(1, 2), (1, 3), (2, 2)])
def test_two_backward_check_bit_exact(config, radius2):
    """flow_fields_two_backward = oracle fields of both runs (the second on
    the swapped images with seed 999 and patch radius radius2) and the
    oracle's mask against both backward fields."""
    p = make_pair(config)
    c = CONFIG_PARAMS[config]
    prm = ff.Params(levels=c.levels, iters=c.iters, R_num=c.R_num, R_den=c.R_den, eps=c.eps, seed=c.seed)
    g = ff.flow_fields_two_backward(dev(p.img1), dev(p.img2), prm, seed2=999, radius2=radius2)
    o1 = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, 3, c.R_num, c.R_den, c.eps, c.seed, nthreads=NT)
    o2 = oracle.flow_fields(p.img2, p.img1, c.levels, c.iters, radius2, c.R_num, c.R_den, c.eps, 999, nthreads=NT)
    keep = oracle.consistency2(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], o2["flow_fwd"],
                               o2["cost_fwd"], c.eps)
    assert np.array_equal(host(g["flow_bwd2"]), o2["flow_fwd"])
    assert np.array_equal(as_u32(g["cost_bwd2"]), o2["cost_fwd"])
    assert np.array_equal(host(g["keep_fwd"]), keep)
    assert np.array_equal(host(g["keep_bwd"]), o1["keep_bwd"])
    assert host(g["keep_fwd"]).sum() <= o1["keep_fwd"].sum()


@pytest.mark.parametrize("q,e,two", [(3, 1, True), (3, 5, False), (4, 2, True), (1, 1, False), (64, 3, True),
                                     (7, 0, False)])
def test_sparsify_bit_exact_on_random_fields(q, e, two):
    """Random fields (targets partly outside the image, many equal errors):
    selections, ties and dropped regions equal the oracle's."""
    rng = np.random.default_rng(q * 100 + e)
    H, W = 97, 131
    fa = rng.integers(-5, 6, size=(H, W, 2)).astype(np.int16)
    fb1 = rng.integers(-5, 6, size=(H, W, 2)).astype(np.int16)
    fb2 = rng.integers(-5, 6, size=(H, W, 2)).astype(np.int16) if two else None
    keep = (rng.random((H, W)) < 0.5).astype(np.uint8)
    got = ff.sparsify(dev(fa), dev(keep), dev(fb1), None if fb2 is None else dev(fb2), q, e)
    assert np.array_equal(host(got), oracle.sparsify(fa, keep, fb1, fb2, q, e))


def test_sparsify_bit_exact_on_oracle_fields():
    """The 1024x436 pair's fields from the oracle (both backward fields):
    the GPU selection equals the oracle's."""
    p = make_pair(2)
    c = CONFIG_PARAMS[2]
    o1 = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, nthreads=NT)
    o2 = oracle.flow_fields(p.img2, p.img1, c.levels, c.iters, radius=2, seed=c.seed + 1, nthreads=NT)
    keep = oracle.consistency2(o1["flow_fwd"], o1["cost_fwd"], o1["flow_bwd"], o1["cost_bwd"], o2["flow_fwd"],
                               o2["cost_fwd"], c.eps)
    for q, e in ((3, 1), (3, 3), (4, 4)):
        got = ff.sparsify(dev(o1["flow_fwd"]), dev(keep), dev(o1["flow_bwd"]), dev(o2["flow_fwd"]), q, e)
        exp = oracle.sparsify(o1["flow_fwd"], keep, o1["flow_bwd"], o2["flow_fwd"], q, e)
        assert np.array_equal(host(got), exp), (q, e)
        assert (exp >= 0).sum() > 0


def _random_filter_inputs(seed, H, W):
    rng = np.random.default_rng(seed)
    flow = rng.integers(-4, 5, size=(H, W, 2)).astype(np.int16)
    flow[: H // 2] = rng.integers(-1, 2, size=(H // 2, W, 2))  # smooth half: large regions
    cost = rng.integers(0, 1000, size=(H, W)).astype(np.uint32)
    cost[rng.random((H, W)) < 0.05] = oracle.UNSET
    keep = ((rng.random((H, W)) < 0.7) & (cost != oracle.UNSET)).astype(np.uint8)
    return flow, cost, keep


@pytest.mark.parametrize("seed,shape,s", [(1, (97, 131), 5), (2, (97, 131), 40), (3, (1, 300), 3), (4, (300, 1), 7),
                                          (5, (1, 1), 2), (6, (64, 64), 0), (7, (211, 157), 100)])
def test_region_filter_bit_exact_on_random_fields(seed, shape, s):
    flow, cost, keep = _random_filter_inputs(seed, *shape)
    got = ff.region_filter(dev(flow), dev(cost.view(np.int32)), dev(keep), s)
    assert np.array_equal(host(got), oracle.region_filter(flow, cost, keep, s))


def test_region_filter_serpentine_region():
    """One region winding through the whole image (long chains of unions)
    plus single-pixel islands next to removed outliers."""
    H, W = 64, 96
    keep = np.zeros((H, W), np.uint8)
    keep[::2] = 1
    for y in range(1, H, 2):
        keep[y, W - 1 if (y // 2) % 2 == 0 else 0] = 1  # connect rows alternately at the ends
    flow = np.zeros((H, W, 2), np.int16)
    cost = np.zeros((H, W), np.uint32)
    rng = np.random.default_rng(9)
    for y, x in zip(rng.integers(1, H - 1, 40) | 1, rng.integers(2, W - 2, 40)):
        keep[y, x] = 1  # islands inside the gaps; they touch the serpentine, so they join it
    for s in (10, H * W):
        got = ff.region_filter(dev(flow), dev(cost.view(np.int32)), dev(keep), s)
        assert np.array_equal(host(got), oracle.region_filter(flow, cost, keep, s)), s


def test_region_filter_bit_exact_on_oracle_fields():
    p = make_pair(2)
    c = CONFIG_PARAMS[2]
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, nthreads=NT)
    for s in (4, 50):
        exp = oracle.region_filter(o["flow_fwd"], o["cost_fwd"], o["keep_fwd"], s)
        got = ff.region_filter(dev(o["flow_fwd"]), dev(o["cost_fwd"].view(np.int32)), dev(o["keep_fwd"]), s)
        assert np.array_equal(host(got), exp), s
        assert exp.sum() < o["keep_fwd"].sum()


@pytest.mark.parametrize("sched", [SCHEDULES[0], SCHEDULES[1]])
def test_plus_graph_replay_repeats_eager_results(sched):
    """A HIP-graph capture of a Flow Fields+ call replays the eager results,
    with eager work of its own between the replays."""
    p = make_pair(1)
    prm = _params(1, sched)
    H, W = p.img1.shape
    f = ff.FlowFields(W, H, prm)
    i1, i2 = dev(p.img1), dev(p.img2)
    eager = {k: host(v).copy() for k, v in f(i1, i2).items()}
    f.capture(i1, i2)
    for rep in range(3):
        for k in ("flow_fwd", "cost_fwd", "keep_fwd", "n_evals"):
            f.out[k].fill_(5)
        ff.flow_fields(i2, i1, prm)
        torch.cuda.synchronize()
        got = {k: host(v).copy() for k, v in f.replay().items()}
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)


@pytest.mark.parametrize("level,sched", [(0, (4, 2, 8, 0)), (0, (4, 2, 8, 4)), (1, (3, 2, 2, 1)), (2, (2, 3, 3, 0))])
def test_run_level_plus_schedules_bit_exact(level, sched):
    """ff_run_level from a consistent state under a Flow Fields+ / Fast
    schedule equals the oracle's steps in the order Sec. 3.3 gives (Fast:
    fine_iters steps at R when the scale is the finest)."""
    P, Rp, T, Tf = sched
    H, W = 61, 83
    n = 1 << level
    prm = ff.Params(levels=level + 1, iters=T, plus_iters=P, Rp_num=Rp, fine_iters=Tf)
    ia, ib = random_images(870 + level, H, W)
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    flow, cost = _random_level_state(5 + level, H, W, n)
    for j, i in zip(*np.nonzero(cost != oracle.UNSET)):
        cost[j, i] = oracle.cost(Da, Db, n, 3, i * n, j * n, int(flow[j, i, 0]), int(flow[j, i, 1]))
    Pl, Tl = (0, Tf) if level == 0 and Tf > 0 else (P, T)
    ef, ec, ne = flow, cost, 0
    for t in range(Pl + Tl):
        ef, ec, k = oracle.propagate(Da, Db, n, t, ef, ec, nthreads=NT)
        ne += k
        if t != Pl - 1 and t != Pl + Tl - 1:
            Rn = oracle.rs_radius(n, Rp, 1) if t < Pl else oracle.rs_radius(n, 1, 1)
            ef, ec, k = oracle.random_search(Da, Db, n, Rn, prm.seed, 0, level, t, ef, ec, nthreads=NT)
            ne += k
    gf, gc = dev(flow), dev(cost.view(np.int32))
    cnt = counter()
    ff.run_level(dev(to_lib(Da, n)), dev(to_lib(Db, n)), level, prm, 0, 0, gf, gc, n_evals=cnt)
    assert np.array_equal(host(gf), ef)
    assert np.array_equal(as_u32(gc), ec)
    assert int(host(cnt)[0]) == ne


@pytest.mark.parametrize("radius,stepwise", [(3, False), (3, True), (2, False)])
def test_forward_only_equals_the_forward_part(radius, stepwise):
    """ff_flow_fields with every backward output NULL gives the full call's
    forward field, cost and evaluation count (blocked, step-wise and
    per-step radius paths)."""
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    prm = ff.Params(levels=c.levels, iters=c.iters, radius=radius, seed=c.seed)
    if stepwise:
        prm = with_tuning(prm, variant=[int(ff.lib().ff_level_variant_count()) - 1] * 7)
    full = ff.flow_fields(dev(p.img1), dev(p.img2), prm)
    fwd = ff.flow_fields(dev(p.img1), dev(p.img2), prm, backward=False)
    assert set(fwd) == {"flow_fwd", "cost_fwd", "n_evals"}
    assert torch.equal(fwd["flow_fwd"], full["flow_fwd"]) and torch.equal(fwd["cost_fwd"], full["cost_fwd"])
    ne = host(fwd["n_evals"])
    assert int(ne[0]) == int(host(full["n_evals"])[0]) and int(ne[1]) == 0
