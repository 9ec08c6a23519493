"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every kernel is compared element by element with the oracle on the same
seeded inputs: sizes that span several tiles with ragged tails, the
degenerate shapes (1x1, 1xN, Nx1, grids smaller than one coarse cell) and
the full-size workloads.  The evaluation counters must match as well.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1703_02563_amd as ff
from tuning_util import with_tuning
from ffgen import CONFIG_PARAMS, FF_SEED, make_pair, random_images

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def as_u32(t):
    return host(t).view(np.uint32)


def counter():
    return torch.zeros(1, dtype=torch.int64, device="cuda")


def phase_columns(Wp, n):
    """Stored column of every column c of a padded map row (phase order:
    c mod n, then c // n), as documented for ff_descriptors."""
    c = np.arange(Wp)
    r = c % n
    return r * (Wp // n) + np.minimum(r, Wp % n) + c // n


def to_lib(D, n):
    """Row-major [H][W][16] descriptors -> the library's descriptor map:
    replicated border of 4n pixels, rows in phase order."""
    P = 4 * n
    H, W = D.shape[:2]
    padded = D[np.clip(np.arange(-P, H + P), 0, H - 1)][:, np.clip(np.arange(-P, W + P), 0, W - 1)]
    out = np.empty_like(padded)
    out[:, phase_columns(W + 2 * P, n)] = padded
    return out


def wform_lib(B, n):
    """Blurred image [H][W] -> weight-class row map [H + 6n][W][16] as
    documented for ff_wform_map_bytes (numpy, from the oracle's blur)."""
    H, W = B.shape
    rows = B[np.clip(np.arange(-3 * n, H + 3 * n), 0, H - 1)]
    x = np.arange(W)

    def col(a):
        return rows[:, np.clip(x + n * a, 0, W - 1)]

    out = np.zeros((H + 6 * n, W, 16), np.uint8)
    for k, a in enumerate((-6, -5, 5, 6, -4, -3, 3, 4, -2, -1, 1, 2, 0)):
        out[..., k] = col(a)
    return out


def from_lib(M, n):
    """Descriptor map -> row-major [H][W][16] (drops the border)."""
    P = 4 * n
    Hp, Wp = M.shape[:2]
    padded = M[:, phase_columns(Wp, n)]
    return np.ascontiguousarray(padded[P:Hp - P, P:Wp - P])


SHAPES = [(37, 53), (1, 1), (1, 40), (33, 1), (120, 160), (9, 300)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_descriptors_bit_exact(shape, n):
    img, _ = random_images(100 + n, *shape, kind="uniform")
    blurred, desc, plain, wform = ff.descriptors(dev(img), n, rowmajor=True, wform=True)
    eb = oracle.blur(img, n)
    ed = oracle.descriptor(eb, n)
    assert np.array_equal(host(blurred), eb)
    assert np.array_equal(host(wform), wform_lib(eb, n))
    assert np.array_equal(host(plain), ed)
    assert np.array_equal(from_lib(host(desc), n), ed)
    assert np.array_equal(host(desc), to_lib(ed, n))  # the replicated border as well
    Wp = shape[1] + 8 * n
    assert sorted(phase_columns(Wp, n)) == list(range(Wp))  # a permutation


@pytest.mark.parametrize("shape", [(37, 53), (120, 160), (9, 300), (200, 131)])
@pytest.mark.parametrize("n", [3, 6, 12, 24, 32, 48, 64])
def test_blur_sub_and_large_scales_bit_exact(shape, n):
    """The box filter at the sub-scales n* = 3n/2 and at the largest scales
    (half-widths up to 32, the widest tile border the one-launch blur
    stages), on frames that span several 64 x 64 tiles with ragged edges;
    the row-major descriptors at the same scale."""
    img, _ = random_images(300 + n, *shape, kind="uniform")
    blurred, desc, plain = ff.descriptors(dev(img), n, rowmajor=True)
    eb = oracle.blur(img, n)
    assert np.array_equal(host(blurred), eb)
    assert np.array_equal(host(plain), oracle.descriptor(eb, n))
    if n & (n - 1) == 0:  # power-of-two scales: the phase-ordered map too
        assert np.array_equal(host(desc), to_lib(oracle.descriptor(eb, n), n))


def _descs(img, levels):
    return oracle.descriptors_all(img, levels)


@pytest.mark.parametrize("shape,nc", [((17, 23), 1), ((40, 60), 4), ((61, 95), 8), ((3, 5), 2), ((1, 1), 1),
                                      ((130, 257), 4), ((7, 200), 16)])
def test_init_nn_bit_exact(shape, nc):
    ia, ib = random_images(7 * nc + shape[0], *shape)
    L = nc.bit_length()
    Da, Db = _descs(ia, L), _descs(ib, L)
    idx, dist = oracle.nn(Da[0], Db[0], nc, nthreads=NT)
    eflow, ecost, ene = oracle.init_coarse(idx, Da[L - 1], Db[L - 1], nc)
    cnt = counter()
    flow, cost, key = ff.init_nn(dev(Da[0]), dev(Db[0]), dev(to_lib(Da[L - 1], nc)), dev(to_lib(Db[L - 1], nc)), nc,
                                 n_evals=cnt)
    k = host(key).view(np.uint64)
    assert np.array_equal((k & 0xFFFFFFFF).astype(np.int64), idx.astype(np.int64))
    assert np.array_equal((k >> 32).astype(np.int64), dist)
    assert np.array_equal(host(flow), eflow)
    assert np.array_equal(as_u32(cost), ecost)
    assert int(host(cnt)[0]) == ene


def test_init_nn_ties_smallest_index():
    ia, _ = random_images(5, 24, 36)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = np.full_like(Da, 100)          # every reference identical
    Db[20, 30] = Da[8, 12]               # two exact matches of one query
    Db[21, 3] = Da[8, 12]
    idx, dist = oracle.nn(Da, Db, 4)
    _, _, key = ff.init_nn(dev(Da), dev(Db), dev(to_lib(Da, 4)), dev(to_lib(Db, 4)), 4)
    k = host(key).view(np.uint64)
    assert np.array_equal((k & 0xFFFFFFFF).astype(np.int64), idx.astype(np.int64))
    assert idx[2, 3] == 20 * 36 + 30


def _random_level_state(seed, H, W, n, unset_frac=0.3):
    rng = np.random.default_rng(seed)
    Wn, Hn = -(-W // n), -(-H // n)
    ys, xs = np.mgrid[0:Hn, 0:Wn] * n
    tx = rng.integers(0, W, size=(Hn, Wn))
    ty = rng.integers(0, H, size=(Hn, Wn))
    # a few coherent patches so that "same flow" skips happen
    tx[: Hn // 2, : Wn // 2] = np.clip(xs[: Hn // 2, : Wn // 2] + 3, 0, W - 1)
    ty[: Hn // 2, : Wn // 2] = np.clip(ys[: Hn // 2, : Wn // 2] - 1, 0, H - 1)
    flow = np.stack([tx - xs, ty - ys], -1).astype(np.int16)
    cost = rng.integers(0, 60000, size=(Hn, Wn)).astype(np.uint32)
    un = rng.random((Hn, Wn)) < unset_frac
    cost[un] = oracle.UNSET
    flow[un] = 0
    return flow, cost


@pytest.mark.parametrize("shape,n", [((45, 70), 1), ((61, 83), 2), ((50, 50), 4), ((1, 31), 1), ((29, 1), 2)])
def test_seed_level_bit_exact(shape, n):
    H, W = shape
    ia, ib = random_images(300 + n, H, W)
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    cflow, ccost = _random_level_state(n, H, W, 2 * n)
    ef, ec, ene = oracle.seed_level(cflow, ccost, Da, Db, n)
    cnt = counter()
    f, c = ff.seed_level(dev(cflow), dev(ccost.view(np.int32)), dev(to_lib(Da, n)), dev(to_lib(Db, n)), n,
                         n_evals=cnt)
    assert np.array_equal(host(f), ef)
    assert np.array_equal(as_u32(c), ec)
    assert int(host(cnt)[0]) == ene


@pytest.mark.parametrize("shape,n", [((45, 70), 1), ((61, 83), 2), ((64, 96), 4), ((1, 31), 1), ((29, 1), 1),
                                     ((200, 300), 1)])
@pytest.mark.parametrize("pass_", [0, 1, 2, 3, 5])
def test_propagate_bit_exact(shape, n, pass_):
    H, W = shape
    ia, ib = random_images(400 + n + pass_, H, W)
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    flow, cost = _random_level_state(pass_, H, W, n)
    ef, ec, ene = oracle.propagate(Da, Db, n, pass_, flow, cost, nthreads=NT)
    gf, gc, cnt = dev(flow), dev(cost.view(np.int32)), counter()
    ff.propagate_level(dev(to_lib(Da, n)), dev(to_lib(Db, n)), n, pass_, gf, gc, n_evals=cnt)
    assert np.array_equal(host(gf), ef)
    assert np.array_equal(as_u32(gc), ec)
    assert int(host(cnt)[0]) == ene


@pytest.mark.parametrize("shape,n,Rn", [((45, 70), 1, 1), ((61, 83), 2, 3), ((64, 96), 4, 6), ((1, 31), 1, 1),
                                        ((200, 300), 1, 2), ((30, 40), 2, 0)])
def test_random_search_bit_exact(shape, n, Rn):
    H, W = shape
    ia, ib = random_images(500 + n, H, W)
    Da = oracle.descriptor(oracle.blur(ia, n), n)
    Db = oracle.descriptor(oracle.blur(ib, n), n)
    flow, cost = _random_level_state(Rn, H, W, n)
    for stream_id, level, pass_ in [(0, 0, 0), (1, 2, 3), (0, 4, 1)]:
        ef, ec, ene = oracle.random_search(Da, Db, n, Rn, FF_SEED, stream_id, level, pass_, flow, cost,
                                           nthreads=NT)
        gf, gc, cnt = dev(flow), dev(cost.view(np.int32)), counter()
        ff.random_search(dev(to_lib(Da, n)), dev(to_lib(Db, n)), n, Rn, FF_SEED, stream_id, level, pass_, gf, gc,
                         n_evals=cnt)
        assert np.array_equal(host(gf), ef)
        assert np.array_equal(as_u32(gc), ec)
        assert int(host(cnt)[0]) == ene


def test_consistency_bit_exact():
    p = make_pair(1)
    o = oracle.flow_fields(p.img1, p.img2, 3, 4, nthreads=NT)
    ka, kb = ff.consistency_filter(dev(o["flow_fwd"]), dev(o["cost_fwd"].view(np.int32)), dev(o["flow_bwd"]),
                                   dev(o["cost_bwd"].view(np.int32)), 1.0)
    assert np.array_equal(host(ka), o["keep_fwd"])
    assert np.array_equal(host(kb), o["keep_bwd"])
    for eps in (0.5, 1.5, 3.0):
        e = oracle.consistency(o["flow_fwd"], o["cost_fwd"], o["flow_bwd"], o["cost_bwd"], eps)
        g, _ = ff.consistency_filter(dev(o["flow_fwd"]), dev(o["cost_fwd"].view(np.int32)), dev(o["flow_bwd"]),
                                     dev(o["cost_bwd"].view(np.int32)), eps, both=False)
        assert np.array_equal(host(g), e)


def _compare_full(img1, img2, params: ff.Params):
    o = oracle.flow_fields(img1, img2, params.levels, params.iters, params.radius, params.R_num, params.R_den,
                           params.eps, params.seed, nthreads=NT, plus_iters=params.plus_iters, Rp_num=params.Rp_num,
                           fine_iters=params.fine_iters)
    g = ff.flow_fields(dev(img1), dev(img2), params)
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(host(g[k]), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(as_u32(g[k]), o[k]), k
    assert tuple(int(v) for v in host(g["n_evals"])) == o["n_evals"]
    return o


@pytest.mark.parametrize("shape,L,T,R", [((1, 1), 1, 1, (1, 1)), ((1, 37), 2, 2, (1, 1)), ((23, 1), 3, 3, (1, 1)),
                                         ((5, 7), 4, 2, (1, 1)), ((31, 45), 3, 4, (3, 2)), ((48, 64), 1, 3, (1, 1)),
                                         ((66, 97), 4, 5, (2, 1)), ((40, 50), 2, 4, (0, 1))])
def test_flow_fields_small_shapes(shape, L, T, R):
    ia, ib = random_images(600 + L * T, *shape)
    _compare_full(ia, ib, ff.Params(levels=L, iters=T, R_num=R[0], R_den=R[1]))


def test_flow_fields_radius_variants():
    ia, ib = random_images(700, 40, 56)
    for r in (0, 1, 2, 5):
        _compare_full(ia, ib, ff.Params(levels=2, iters=3, radius=r))


@pytest.mark.parametrize("config", [1, 2, 3])
def test_flow_fields_configs_bit_exact(config):
    p = make_pair(config)
    c = CONFIG_PARAMS[config]
    o = _compare_full(p.img1, p.img2, ff.Params(levels=c.levels, iters=c.iters, R_num=c.R_num, R_den=c.R_den,
                                                eps=c.eps, seed=c.seed))
    print(f"config {config}: n_evals {o['n_evals']}", flush=True)


def test_flow_fields_repeat_is_deterministic():
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    prm = ff.Params(levels=c.levels, iters=c.iters)
    f = ff.FlowFields(160, 120, prm)
    a = {k: host(v).copy() for k, v in f(dev(p.img1), dev(p.img2)).items()}
    b = {k: host(v).copy() for k, v in f(dev(p.img1), dev(p.img2)).items()}
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("config", [1, 2])
def test_flow_fields_graph_replay_repeats_eager_results(config):
    """One ff_flow_fields call captured into a HIP graph: every replay gives
    the eager call's outputs (fields, costs, masks, evaluation counts), with
    the outputs clobbered and eager work on the device between replays."""
    p = make_pair(config)
    c = CONFIG_PARAMS[config]
    H, W = p.img1.shape
    prm = ff.Params(levels=c.levels, iters=c.iters, R_num=c.R_num, R_den=c.R_den, eps=c.eps, seed=c.seed)
    f = ff.FlowFields(W, H, prm)
    i1, i2 = dev(p.img1), dev(p.img2)
    eager = {k: host(v).copy() for k, v in f(i1, i2).items()}
    f.capture(i1, i2)
    for rep in range(3):
        for k in ("flow_fwd", "flow_bwd", "cost_fwd", "keep_fwd", "n_evals"):
            f.out[k].fill_(3)
        ff.flow_fields(i2, i1, prm)  # eager work of its own between replays
        torch.cuda.synchronize()
        got = {k: host(v).copy() for k, v in f.replay().items()}
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)


@pytest.mark.parametrize("config", [1, 2])
def test_level_kernel_variants_bit_exact(config):
    """Every launch variant of the level kernel gives the same field."""
    p = make_pair(config)
    c = CONFIG_PARAMS[config]
    prm = ff.Params(levels=c.levels, iters=c.iters, R_num=c.R_num, R_den=c.R_den)
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, c.radius, c.R_num, c.R_den, c.eps, c.seed,
                           nthreads=NT)
    for v in range(int(ff.lib().ff_level_variant_count())):
        g = ff.flow_fields(dev(p.img1), dev(p.img2), with_tuning(prm, variant=[v] * 7))
        for k in ("flow_fwd", "flow_bwd", "keep_fwd"):
            assert np.array_equal(host(g[k]), o[k]), (v, k)
        assert np.array_equal(as_u32(g["cost_fwd"]), o["cost_fwd"]), v
        assert tuple(int(x) for x in host(g["n_evals"])) == o["n_evals"], v


@pytest.mark.parametrize("shape,level,T,R", [((61, 83), 0, 6, (1, 1)), ((61, 83), 1, 4, (3, 2)),
                                             ((130, 200), 2, 6, (1, 1)), ((45, 70), 0, 9, (2, 1)),
                                             ((33, 1), 0, 3, (1, 1)), ((200, 260), 0, 6, (1, 1))])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("variant", [None, 18, 20, 23])
def test_run_level_bit_exact(shape, level, T, R, mode, variant):
    """ff_run_level equals the oracle's step sequence for that scale (the
    built-in table, and weight-class variants given their row maps)."""
    H, W = shape
    n = 1 << level
    prm = ff.Params(levels=level + 1, iters=T, R_num=R[0], R_den=R[1])
    ia, ib = random_images(800 + level * 10 + mode, H, W)
    Ba, Bb = oracle.blur(ia, n), oracle.blur(ib, n)
    Da = oracle.descriptor(Ba, n)
    Db = oracle.descriptor(Bb, n)
    wf = {}
    if variant is not None:
        prm = with_tuning(prm, variant=[variant] * 7)
        wf = dict(wform_a=dev(wform_lib(Ba, n)), wform_b=dev(wform_lib(Bb, n)))
    Wn, Hn = -(-W // n), -(-H // n)
    key = cflow = ccost = None
    if mode == 0:
        # a consistent state (cost = E_n of the flow), as ff_run_level requires
        flow, cost = _random_level_state(3, H, W, n)
        for j, i in zip(*np.nonzero(cost != oracle.UNSET)):
            cost[j, i] = oracle.cost(Da, Db, n, 3, i * n, j * n, int(flow[j, i, 0]), int(flow[j, i, 1]))
        ne0 = 0
    elif mode == 1:
        Da1 = oracle.descriptor(oracle.blur(ia, 1), 1)
        Db1 = oracle.descriptor(oracle.blur(ib, 1), 1)
        idx, _ = oracle.nn(Da1, Db1, n, nthreads=NT)
        flow, cost, ne0 = oracle.init_coarse(idx, Da, Db, n)
        key = dev(idx.astype(np.int64))
    else:
        cflow, ccost = _random_level_state(4, H, W, 2 * n)
        flow, cost, ne0 = oracle.seed_level(cflow, ccost, Da, Db, n)
    ef, ec, ne = flow, cost, ne0
    Rn = oracle.rs_radius(n, *R)
    for t in range(T):
        ef, ec, k = oracle.propagate(Da, Db, n, t, ef, ec, nthreads=NT)
        ne += k
        if t < T - 1:
            ef, ec, k = oracle.random_search(Da, Db, n, Rn, prm.seed, 0, level, t, ef, ec, nthreads=NT)
            ne += k
    if mode == 0:
        gf, gc = dev(flow), dev(cost.view(np.int32))
    else:
        gf = torch.empty((Hn, Wn, 2), dtype=torch.int16, device="cuda")
        gc = torch.empty((Hn, Wn), dtype=torch.int32, device="cuda")
    cnt = counter()
    ff.run_level(dev(to_lib(Da, n)), dev(to_lib(Db, n)), level, prm, 0, mode, gf, gc, nn_key=key,
                 coarse_flow=None if cflow is None else dev(cflow),
                 coarse_cost=None if ccost is None else dev(ccost.view(np.int32)), n_evals=cnt, **wf)
    assert np.array_equal(host(gf), ef)
    assert np.array_equal(as_u32(gc), ec)
    assert int(host(cnt)[0]) == ne


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_run_length_does_not_change_results(passes):
    """Shorter runs of steps per blocked launch give the same field."""
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    prm = ff.Params(levels=c.levels, iters=c.iters)
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, nthreads=NT)
    g = ff.flow_fields(dev(p.img1), dev(p.img2), with_tuning(prm, passes=[passes] * 7))
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(host(g[k]), o[k]), k
    assert np.array_equal(as_u32(g["cost_fwd"]), o["cost_fwd"])
    assert tuple(int(x) for x in host(g["n_evals"])) == o["n_evals"]


@pytest.mark.parametrize("table", [([4, 7, 6, 6, 6, 3, 3], [1, 2, 2, 3, 3, 0, 0]),
                                   ([2, 5, 3, 7, 6, 3, 3], [1, 1, 1, 1, 1, 1, 1]),
                                   ([0, 1, 4, 2, 8, 3, 3], [3, 2, 0, 1, 2, 0, 0]),
                                   ([16, 17, 13, 14, 16, 3, 3], [7, 7, 7, 7, 7, 0, 0]),
                                   ([17, 16, 14, 13, 12, 11, 15], [4, 3, 6, 5, 2, 1, 0]),
                                   ([18, 19, 22, 23, 23, 3, 3], [2, 2, 3, 2, 2, 0, 0]),
                                   ([20, 21, 18, 22, 24, 23, 19], [1, 1, 2, 3, 0, 1, 2])])
@pytest.mark.parametrize("case", [(2, 0), (5, 16)])
def test_mixed_variant_and_run_length_tables_bit_exact(table, case):
    """Launch tables mixing variants and run lengths per scale (as the
    autotuner writes them) on 1024x436 pairs: every scale that takes several
    launches alternates its two grid buffers."""
    cfg, k = case
    p = make_pair(cfg, k)
    c = CONFIG_PARAMS[2]
    prm = ff.Params(levels=c.levels, iters=c.iters)
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, nthreads=NT)
    prm = with_tuning(prm, variant=table[0], passes=table[1])
    for _ in range(2):
        g = ff.flow_fields(dev(p.img1), dev(p.img2), prm)
        for key in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
            assert np.array_equal(host(g[key]), o[key]), key
        assert np.array_equal(as_u32(g["cost_bwd"]), o["cost_bwd"])
        assert tuple(int(x) for x in host(g["n_evals"])) == o["n_evals"]


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("passes", [1, 2])
@pytest.mark.parametrize("variant", [None, 18])
def test_run_level_multi_launch_bit_exact(mode, passes, variant):
    """ff_run_level split into several launches (odd and even counts, a
    continuing first run included) equals the oracle's step sequence."""
    H, W, level, T = 130, 200, 0, 5
    n = 1
    prm = ff.Params(levels=1, iters=T)
    ia, ib = random_images(950 + mode + passes, H, W)
    Ba, Bb = oracle.blur(ia, n), oracle.blur(ib, n)
    Da = oracle.descriptor(Ba, n)
    Db = oracle.descriptor(Bb, n)
    wf = {}
    if variant is not None:
        prm = with_tuning(prm, variant=[variant] * 7)
        wf = dict(wform_a=dev(wform_lib(Ba, n)), wform_b=dev(wform_lib(Bb, n)))
    if mode == 0:
        flow, cost = _random_level_state(5, H, W, n)
        for j, i in zip(*np.nonzero(cost != oracle.UNSET)):
            cost[j, i] = oracle.cost(Da, Db, n, 3, i * n, j * n, int(flow[j, i, 0]), int(flow[j, i, 1]))
        ne = 0
        gf, gc = dev(flow), dev(cost.view(np.int32))
        cflow = ccost = None
    else:
        cflow, ccost = _random_level_state(6, H, W, 2)
        flow, cost, ne = oracle.seed_level(cflow, ccost, Da, Db, n)
        gf = torch.empty((H, W, 2), dtype=torch.int16, device="cuda")
        gc = torch.empty((H, W), dtype=torch.int32, device="cuda")
    ef, ec = flow, cost
    for t in range(T):
        ef, ec, k = oracle.propagate(Da, Db, n, t, ef, ec, nthreads=NT)
        ne += k
        if t < T - 1:
            ef, ec, k = oracle.random_search(Da, Db, n, 1, prm.seed, 0, level, t, ef, ec, nthreads=NT)
            ne += k
    cnt = counter()
    ff.run_level(dev(to_lib(Da, n)), dev(to_lib(Db, n)), level, with_tuning(prm, passes=[passes] * 7), 0, mode, gf,
                 gc, coarse_flow=None if cflow is None else dev(cflow),
                 coarse_cost=None if ccost is None else dev(ccost.view(np.int32)), n_evals=cnt, **wf)
    assert np.array_equal(host(gf), ef)
    assert np.array_equal(as_u32(gc), ec)
    assert int(host(cnt)[0]) == ne


def _tie_state(bands, cells):
    """Tie cases like those of the oracle pins, on a 48 x 24 pair: image b is
    a blurred image constant on the bands x < 24 and x >= 24 (its patch costs
    depend only on the band a target's patch and descriptors reach); a few
    set cells with consistent costs."""
    ia, _ = random_images(77, 24, 48)
    Ba = oracle.blur(ia, 1)
    Bb = np.empty((24, 48), np.uint8)
    Bb[:, :24] = bands[0]
    Bb[:, 24:] = bands[1]
    Da, Db = oracle.descriptor(Ba, 1), oracle.descriptor(Bb, 1)
    flow = np.zeros((24, 48, 2), np.int16)
    cost = np.full((24, 48), oracle.UNSET, np.uint32)
    for (i, j), f in cells.items():
        flow[j, i] = f
        cost[j, i] = oracle.cost(Da, Db, 1, 3, i, j, f[0], f[1])
    return Ba, Bb, Da, Db, flow, cost


@pytest.mark.parametrize("blocked", [False, True, "wform"])
def test_propagation_ties_bit_exact(blocked):
    """Equal errors of the horizontal and vertical source (the horizontal
    one wins), a held flow of equal error (kept) and strict differences
    either way, for cell (23, 10) (left source (22, 10), top (23, 9)),
    through the per-step kernel, the blocked descriptor kernel and the
    weight-class kernel (every cell and target here 3 px inside)."""
    fh, fv, fr = (-8, 2), (-9, -4), (8, 3)  # targets (15, 12), (14, 6) in the left band, (31, 13) in the right
    cases = [((100, 100), {(22, 10): fh, (23, 9): fv}),
             ((100, 100), {(22, 10): fh, (23, 9): fv, (23, 10): (-7, 1)}),
             ((100, 250), {(22, 10): fr, (23, 9): fh}), ((100, 250), {(22, 10): fh, (23, 9): fr}),
             ((250, 100), {(22, 10): fr, (23, 9): fh}), ((250, 100), {(22, 10): fh, (23, 9): fr})]
    prm = ff.Params(levels=1, iters=1)
    for bands, cells in cases:
        Ba, Bb, Da, Db, flow, cost = _tie_state(bands, cells)
        ef, ec, ne = oracle.propagate(Da, Db, 1, 0, flow, cost)
        if bands[0] == bands[1] and len(cells) == 2:
            assert tuple(ef[10, 23]) == fh  # the pinned rule on this case
        gf, gc, cnt = dev(flow), dev(cost.view(np.int32)), counter()
        if blocked == "wform":
            ff.run_level(dev(to_lib(Da, 1)), dev(to_lib(Db, 1)), 0, with_tuning(prm, variant=[18] * 7), 0, 0, gf, gc,
                         n_evals=cnt, wform_a=dev(wform_lib(Ba, 1)), wform_b=dev(wform_lib(Bb, 1)))
        elif blocked:
            ff.run_level(dev(to_lib(Da, 1)), dev(to_lib(Db, 1)), 0, prm, 0, 0, gf, gc, n_evals=cnt)
        else:
            ff.propagate_level(dev(to_lib(Da, 1)), dev(to_lib(Db, 1)), 1, 0, gf, gc, n_evals=cnt)
        assert np.array_equal(host(gf), ef), cells
        assert np.array_equal(as_u32(gc), ec), cells
        assert int(host(cnt)[0]) == ne


def test_two_streams_with_different_tables_run_concurrently():
    """Launch tables travel with each call: two threads enqueue calls with
    different tables on two streams at once, and both results are the
    oracle's."""
    import threading
    p = make_pair(1)
    c = CONFIG_PARAMS[1]
    o = oracle.flow_fields(p.img1, p.img2, c.levels, c.iters, c.radius, c.R_num, c.R_den, c.eps, c.seed, nthreads=NT)
    base = ff.Params(levels=c.levels, iters=c.iters, R_num=c.R_num, R_den=c.R_den)
    prms = [with_tuning(base, variant=[16, 17, 14, 15, 15, 3, 3], passes=[2, 2, 3, 2, 2, 0, 0]),
            with_tuning(base, variant=[2, 5, 3, 7, 6, 3, 3], passes=[1, 1, 1, 1, 1, 1, 1])]
    i1, i2 = dev(p.img1), dev(p.img2)
    runners = [ff.FlowFields(160, 120, prm) for prm in prms]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    errors = []

    def work(k):
        try:
            with torch.cuda.stream(streams[k]):
                for _ in range(20):
                    runners[k](i1, i2)
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors
    for r in runners:
        for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
            assert np.array_equal(host(r.out[k]), o[k]), k
        assert np.array_equal(as_u32(r.out["cost_fwd"]), o["cost_fwd"])
        assert tuple(int(x) for x in host(r.out["n_evals"])) == o["n_evals"]


@pytest.mark.parametrize("radius", [3, 2, 1])
def test_run_level_work_counters(radius):
    """ff_run_level's counters of computed evaluations: never above the
    schedule's count, owned cells <= all cells, and for the per-step
    kernels (radius 1 here; no halo) the two are equal; the blocked kernels
    (radius 3 and 2) compute most of the schedule's evaluations (a
    consistent state fixes only the repeated vertical sources)."""
    H, W, T = 130, 200, 5
    prm = ff.Params(levels=1, iters=T, radius=radius)
    ia, ib = random_images(77, H, W)
    Da = oracle.descriptor(oracle.blur(ia, 1), 1)
    Db = oracle.descriptor(oracle.blur(ib, 1), 1)
    cflow, ccost = _random_level_state(6, H, W, 2)
    gf = torch.empty((H, W, 2), dtype=torch.int16, device="cuda")
    gc = torch.empty((H, W), dtype=torch.int32, device="cuda")
    cnt = counter()
    work = torch.zeros(2, dtype=torch.int64, device="cuda")
    ff.run_level(dev(to_lib(Da, 1)), dev(to_lib(Db, 1)), 0, prm, 0, 2, gf, gc, coarse_flow=dev(cflow),
                 coarse_cost=dev(ccost.view(np.int32)), n_evals=cnt, n_work=work)
    ne = int(host(cnt)[0])
    owned, every = (int(v) for v in host(work))
    assert 0 < owned <= ne and owned <= every
    if radius not in (2, 3):
        assert owned == every
    else:
        assert every > owned and owned > 0.8 * ne


@pytest.mark.parametrize("shape,level,T", [((61, 83), 0, 6), ((130, 200), 1, 5), ((45, 70), 0, 4)])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("with_wform", [True, False])
def test_run_level_pair_bit_exact(shape, level, T, mode, with_wform):
    """ff_run_level_pair: both directions of one scale in one set of launches
    (direction 0 image a's cells in image b, stream id 0; direction 1 the
    reverse, stream id 1), each equal to the oracle's step sequence, with
    per-direction evaluation counts."""
    H, W = shape
    n = 1 << level
    prm = ff.Params(levels=level + 1, iters=T)
    ia, ib = random_images(1300 + level * 10 + mode, H, W)
    B = [oracle.blur(im, n) for im in (ia, ib)]
    D = [oracle.descriptor(b, n) for b in B]
    Wn, Hn = -(-W // n), -(-H // n)
    Rn = oracle.rs_radius(n, prm.R_num, prm.R_den)
    flows, costs, keys, cflows, ccosts, expect = [], [], [], [], [], []
    for dr in range(2):
        Da, Db = D[dr], D[dr ^ 1]
        if mode == 0:
            flow, cost = _random_level_state(30 + dr, H, W, n)
            for j, i in zip(*np.nonzero(cost != oracle.UNSET)):
                cost[j, i] = oracle.cost(Da, Db, n, 3, i * n, j * n, int(flow[j, i, 0]), int(flow[j, i, 1]))
            ne = 0
            flows.append(dev(flow))
            costs.append(dev(cost.view(np.int32)))
        else:
            if mode == 1:
                D1 = [oracle.descriptor(oracle.blur(im, 1), 1) for im in (ia, ib)]
                idx, _ = oracle.nn(D1[dr], D1[dr ^ 1], n, nthreads=NT)
                flow, cost, ne = oracle.init_coarse(idx, Da, Db, n)
                keys.append(dev(idx.astype(np.int64)))
            else:
                cf, cc = _random_level_state(40 + dr, H, W, 2 * n)
                flow, cost, ne = oracle.seed_level(cf, cc, Da, Db, n)
                cflows.append(dev(cf))
                ccosts.append(dev(cc.view(np.int32)))
            flows.append(torch.empty((Hn, Wn, 2), dtype=torch.int16, device="cuda"))
            costs.append(torch.empty((Hn, Wn), dtype=torch.int32, device="cuda"))
        for t in range(T):
            flow, cost, k = oracle.propagate(Da, Db, n, t, flow, cost, nthreads=NT)
            ne += k
            if t < T - 1:
                flow, cost, k = oracle.random_search(Da, Db, n, Rn, prm.seed, dr, level, t, flow, cost, nthreads=NT)
                ne += k
        expect.append((flow, cost, ne))
    wf = dict(wform_a=dev(wform_lib(B[0], n)), wform_b=dev(wform_lib(B[1], n))) if with_wform else {}
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    work = torch.zeros(2, dtype=torch.int64, device="cuda")
    ff.run_level_pair(dev(to_lib(D[0], n)), dev(to_lib(D[1], n)), level, prm, mode, flows, costs,
                      nn_keys=keys or None, coarse_flows=cflows or None, coarse_costs=ccosts or None, n_evals=cnt,
                      n_work=work, **wf)
    for dr in range(2):
        ef, ec, ne = expect[dr]
        assert np.array_equal(host(flows[dr]), ef), dr
        assert np.array_equal(as_u32(costs[dr]), ec), dr
        assert int(host(cnt)[dr]) == ne, dr
    owned, every = (int(v) for v in host(work))
    assert 0 < owned <= every and owned <= int(host(cnt).sum())
