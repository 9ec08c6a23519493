"""Learned-descriptor form on the GPU: convolution kernels against float64
torch.nn.functional.conv2d and its autograd, the whole network's gradient
against the float64 reference (bf16 rounding emulated where the kernels
round) and float64 finite differences, Adam against its formula, the
quantiser and the learned-feature Flow Fields against the oracle bit for
bit, and a short training run."""
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import paper_1703_02563_amd as ff
from tuning_util import with_tuning
from descnet_ref import LAYERS, bf16, forward, reference_chain, torch_weight
from paper_1703_02563_amd import learned as Lm
from test_learned_oracle import feature_canvas, feature_pyramid

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


def bits(t64):
    """float64 CPU tensor of bf16-representable values -> bf16 bit patterns on the GPU."""
    return Lm._bf16_bits(t64.float().cuda())


def _rand(shape, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return bf16(torch.randn(shape, generator=g, dtype=torch.float64) * scale)


# float32 accumulation of K bf16 x bf16 products (exact in float32):
# |err| <= K * 2^-24 * sum|products|
def _bound(x, w, K):
    return K * 2.0 ** -24 * F.conv2d(x.abs(), w.abs(), padding=1) + 1e-6


@pytest.mark.parametrize("cin,cout", [(1, 32), (32, 32), (32, 16), (16, 32)])
@pytest.mark.parametrize("B,H,W", [(1, 37, 53), (2, 16, 70), (1, 1, 1)])
def test_conv_forward_matches_f64(cin, cout, B, H, W):
    x = _rand((B, H, W, cin), 10 + cin + H)
    w = _rand((cout, 9, cin), 20 + cout, (2.0 / (9 * cin)) ** 0.5)
    b = torch.randn(cout, generator=torch.Generator().manual_seed(3), dtype=torch.float64) * 0.1
    # every device argument is a named tensor: a temporary would be freed and
    # its memory reused for the next argument before the kernel runs
    xd, wd, bd = bits(x), bits(w), b.float().cuda()
    for relu in (0, 1):
        out = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
        ff.ffi.check(ff.lib().ff_conv3x3_fwd(Lm._ptr(xd), B, H, W, cin, cout, Lm._ptr(wd), Lm._ptr(bd), relu,
                                             Lm._ptr(out), None, Lm._stream()), "ff_conv3x3_fwd")
        xt, wt = x.permute(0, 3, 1, 2), torch_weight(w)
        ref = F.conv2d(xt, wt, b.float().double(), padding=1)
        if relu:
            ref = torch.relu(ref)
        tol = _bound(xt, wt, 9 * cin)
        got = out.cpu().double().permute(0, 3, 1, 2)
        assert torch.all((got - ref).abs() <= tol), float(((got - ref).abs() - tol).max())


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 16)])
def test_conv_data_and_weight_gradients_match_f64_autograd(cin, cout):
    B, H, W = 2, 23, 41
    x = _rand((B, H, W, cin), 5)
    w = _rand((cout, 9, cin), 6, (2.0 / (9 * cin)) ** 0.5)
    go = _rand((B, H, W, cout), 7)
    xt = x.permute(0, 3, 1, 2).clone().requires_grad_(True)
    wt = torch_weight(w).clone().requires_grad_(True)
    bt = torch.zeros(cout, dtype=torch.float64, requires_grad=True)
    (F.conv2d(xt, wt, bt, padding=1) * go.permute(0, 3, 1, 2)).sum().backward()
    # data gradient
    xd, wd, god, go32 = bits(x), bits(w), bits(go), go.float().cuda()
    flip = torch.empty((cin, 9, cout), dtype=torch.int16, device="cuda")
    gin = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    ff.ffi.check(ff.lib().ff_conv3x3_bwd_data(Lm._ptr(god), B, H, W, cin, cout, Lm._ptr(wd), Lm._ptr(flip),
                                              Lm._ptr(gin), None, Lm._stream()), "ff_conv3x3_bwd_data")
    ref = xt.grad.permute(0, 2, 3, 1)
    tol = 9 * cout * 2.0 ** -24 * F.conv2d(go.abs().permute(0, 3, 1, 2),
                                            torch_weight(w).abs().flip(2, 3).transpose(0, 1),
                                            padding=1).permute(0, 2, 3, 1) + 1e-6
    assert torch.all((gin.cpu().double() - ref).abs() <= tol)
    # weight and bias gradients (float32 sums over all pixels)
    nbytes = int(ff.lib().ff_conv3x3_wgrad_scratch_bytes(B, H, cin, cout))
    scratch = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    gw = torch.empty((cout, 9, cin), dtype=torch.float32, device="cuda")
    gb = torch.empty(cout, dtype=torch.float32, device="cuda")
    ff.ffi.check(ff.lib().ff_conv3x3_bwd_weight(Lm._ptr(xd), Lm._ptr(go32), B, H, W, cin, cout,
                                                Lm._ptr(scratch), nbytes, Lm._ptr(gw), Lm._ptr(gb), Lm._stream()),
                 "ff_conv3x3_bwd_weight")
    gw_ref = wt.grad.permute(0, 2, 3, 1).reshape(cout, 9, cin)
    P = B * H * W
    absw = torch.zeros_like(gw_ref)  # sum |g * x| per weight, the accumulation error scale
    xa = F.pad(x.abs().permute(0, 3, 1, 2), (1, 1, 1, 1))
    for tap in range(9):
        ky, kx = tap // 3, tap % 3
        xs = xa[:, :, ky:ky + H, kx:kx + W]
        absw[:, tap, :] = torch.einsum("bchw,bdhw->dc", xs, go.abs().permute(0, 3, 1, 2))
    # matrix-core products of x with go split into two bf16 parts (within
    # 2^-18 |go| of go), float32 accumulation of at most about 2.2 P terms
    # per output (two products of 16 pixels per MFMA step, then the
    # per-wave partials): |error| <= (2^-18 + 3.1 P 2^-24) sum |go x|
    wg = 2.0 ** -18 + 3.1 * P * 2.0 ** -24
    assert torch.all((gw.cpu().double() - gw_ref).abs() <= wg * absw + 1e-6)
    assert torch.allclose(gb.cpu().double(), bt.grad, rtol=0, atol=wg * float(go.abs().sum()) + 1e-6)


def test_wgrad_is_deterministic():
    B, H, W, cin, cout = 4, 64, 96, 32, 32
    x = bits(_rand((B, H, W, cin), 8))
    go = _rand((B, H, W, cout), 9).float().cuda()
    nbytes = int(ff.lib().ff_conv3x3_wgrad_scratch_bytes(B, H, cin, cout))
    outs = []
    for _ in range(2):
        scratch = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        gw = torch.empty((cout, 9, cin), dtype=torch.float32, device="cuda")
        ff.ffi.check(ff.lib().ff_conv3x3_bwd_weight(Lm._ptr(x), Lm._ptr(go), B, H, W, cin, cout, Lm._ptr(scratch),
                                                    nbytes, Lm._ptr(gw), None, Lm._stream()), "wgrad")
        outs.append(gw.cpu())
    assert torch.equal(outs[0], outs[1])


def _net_and_crop(seed=0, normalize=True):
    net = Lm.DescNet(seed=seed, normalize=normalize)
    g = torch.Generator().manual_seed(seed + 1)
    for k in range(3):  # non-zero biases exercise the bias gradient
        net.b[k] = (torch.randn(net.b[k].shape, generator=g) * 0.1).cuda()
    img = (torch.rand((1, 48, 64), generator=g) * 255).round().to(torch.uint8)
    return net, img


U32 = 2.0 ** -24  # float32 unit roundoff
UBF = 2.0 ** -8   # bounds |bf16(s) - bf16(t)| <= (1 + 2^-8)|s - t| + 2^-8 |t| (round to nearest even, 2^-9 each)


def _nchw(t):
    return t.permute(0, 3, 1, 2)


@pytest.mark.parametrize("seed", [0, 1])
def test_network_forward_and_gradients_elementwise(seed):
    """The whole network on the GPU (conv kernels, ReLU backward, bf16
    roundings of activations and upstream gradients) against the float64
    chain, element by element: every layer's error bound is propagated from
    the previous layer's (conv of the error with |w|), plus float32
    accumulation of K terms (K u sum|terms|; the weight gradient's upstream
    factor also split into two bf16 parts), plus bf16 rounding of either
    side (2^-8 relative), plus the full value where the two sides' ReLU
    masks differ."""
    net, img = _net_and_crop(seed=seed, normalize=False)
    x_bits = net.input_from_images(img.cuda())
    out, acts = net.forward(x_bits, keep=True)
    probe = torch.randn((1, 48, 64, 16), generator=torch.Generator().manual_seed(5 + seed), dtype=torch.float64)
    probe = probe.float().double()  # the kernels receive float32
    gws, gbs = net.backward(acts, probe.float().cuda())
    x = _nchw(Lm.bf16_bits_to_f32(x_bits).cpu().double())
    ws = [w.cpu().double() for w in net.w]
    ws = [bf16(w) for w in ws]  # the kernels multiply the bf16 copies
    bs = [b.cpu().double() for b in net.b]
    a, ys, gw_ref, gb_ref, gy = reference_chain(x, ws, bs, _nchw(probe))
    P = float(x.numel())  # pixels summed by the weight gradient
    # forward
    da = [torch.zeros_like(x)]
    for k, (cin, cout, relu) in enumerate(LAYERS):
        wt = torch_weight(ws[k]).abs()
        e = F.conv2d(da[k], wt, padding=1) + (9 * cin + 1) * U32 * (
            F.conv2d(a[k].abs() + da[k], wt, padding=1) + bs[k].abs()[None, :, None, None])
        if relu:
            d = e * (1 + UBF) + UBF * torch.relu(ys[k])
            got = _nchw(Lm.bf16_bits_to_f32(acts[k + 1]).cpu().double())
            assert torch.all((got - a[k + 1]).abs() <= d), (k, float(((got - a[k + 1]).abs() - d).max()))
            da.append(d)
        else:
            got = _nchw(out.cpu().double())
            assert torch.all((got - ys[k]).abs() <= e + 1e-30), float(((got - ys[k]).abs() - e).max())
    # backward: dg = bound of the GPU's upstream gradient of layer k's output
    dg = torch.zeros_like(gy[2])
    for k in (2, 1, 0):
        cin, cout, _ = LAYERS[k]
        ga, ea = a[k].abs(), da[k]
        g_abs = gy[k].abs()
        shape = torch_weight(ws[k]).shape
        cw = torch.nn.grad.conv2d_weight
        # weight gradient: the upstream gradient split into two bf16 parts
        # (within 2^-18 of it) times the bf16 activations on matrix cores,
        # float32 accumulation of at most about 2.2 P terms
        wg = 2.0 ** -18 + 3.1 * P * U32
        bw = cw(ea, shape, g_abs + dg, padding=1) + cw(ga, shape, dg, padding=1) + \
            wg * cw(ga + ea, shape, g_abs + dg, padding=1)
        got_w = torch_weight(gws[k].cpu().double().reshape(ws[k].shape))
        assert torch.all((got_w - gw_ref[k]).abs() <= bw + 1e-12), (k, float(((got_w - gw_ref[k]).abs() - bw).max()))
        bb = dg.sum((0, 2, 3)) + wg * (g_abs + dg).sum((0, 2, 3))
        assert torch.all((gbs[k].cpu().double() - gb_ref[k]).abs() <= bb + 1e-12), k
        if k == 0:
            break
        # the kernels round the upstream gradient to bf16, take the data
        # gradient with float32 accumulation, then mask by the ReLU of a[k]
        d16 = dg * (1 + UBF) + UBF * g_abs
        wt = torch_weight(ws[k]).abs()
        ci = torch.nn.grad.conv2d_input
        gin_ref = ci(a[k].shape, torch_weight(ws[k]), gy[k], padding=1)
        e = ci(a[k].shape, wt, d16, padding=1) + (9 * cout + 1) * U32 * ci(a[k].shape, wt, g_abs + d16, padding=1)
        mask_gpu = _nchw(Lm.bf16_bits_to_f32(acts[k]).cpu().double()) > 0
        mask_ref = ys[k - 1] > 0
        dg = torch.where(mask_gpu == mask_ref, e, gin_ref.abs() + e)
        dg = torch.where(mask_gpu | mask_ref, dg, torch.zeros_like(dg))


def test_l2norm_forward_and_backward():
    from descnet_ref import l2norm
    g0 = torch.Generator().manual_seed(6)
    f = torch.randn((2, 13, 17, 16), generator=g0) * 3
    f[0, 0, 0] = 0.0  # zero feature: finite thanks to delta
    g = torch.randn((2, 13, 17, 16), generator=g0)
    fd, gd = f.cuda(), g.cuda()
    y = torch.empty_like(fd)
    inv = torch.empty((2, 13, 17), device="cuda")
    ff.ffi.check(ff.lib().ff_l2norm16_fwd(Lm._ptr(fd), 2 * 13 * 17, 1e-4, Lm._ptr(y), Lm._ptr(inv), Lm._stream()),
                 "l2norm fwd")
    gin = torch.empty_like(fd)
    ff.ffi.check(ff.lib().ff_l2norm16_bwd(Lm._ptr(y), Lm._ptr(inv), Lm._ptr(gd), 2 * 13 * 17, Lm._ptr(gin),
                                          Lm._stream()), "l2norm bwd")
    f64 = f.double().permute(0, 3, 1, 2).requires_grad_(True)
    ref = l2norm(f64, float(np.float32(1e-4)))
    (ref * g.double().permute(0, 3, 1, 2)).sum().backward()
    assert torch.allclose(y.cpu().double(), ref.detach().permute(0, 2, 3, 1), rtol=0, atol=2e-6)
    assert torch.allclose(gin.cpu().double(), f64.grad.permute(0, 2, 3, 1), rtol=1e-4, atol=1e-4)


def test_adam_step_matches_formula():
    n = 1000
    g = torch.Generator().manual_seed(2)
    p0 = torch.randn(n, generator=g)
    grads = [torch.randn(n, generator=g) for _ in range(3)]
    p = p0.clone().cuda()
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    pr, mr, vr = p0.double().numpy(), np.zeros(n), np.zeros(n)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for t, gr in enumerate(grads, start=1):
        grd = gr.cuda()
        ff.ffi.check(ff.lib().ff_adam_step(Lm._ptr(p), Lm._ptr(grd), Lm._ptr(m), Lm._ptr(v), n, lr, b1, b2, eps,
                                           t, None, Lm._stream()), "adam")
        gd = gr.double().numpy()
        mr = b1 * mr + (1 - b1) * gd
        vr = b2 * vr + (1 - b2) * gd * gd
        pr = pr - lr * (mr / (1 - b1 ** t)) / (np.sqrt(vr / (1 - b2 ** t)) + eps)
    assert np.allclose(p.cpu().double().numpy(), pr, rtol=0, atol=1e-6)


def test_quantize_matches_oracle():
    f = feature_canvas(3, 40, 60)
    q = Lm.quantize_u8(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.array_equal(q, oracle.quantize_u8(f))


@pytest.mark.parametrize("tiles", [None, 0, 1, 2, 3, 4])
@pytest.mark.parametrize("shape,L,T,passes", [((40, 56), 3, 4, 0), ((33, 1), 2, 3, 0), ((1, 1), 1, 1, 0),
                                              ((120, 160), 3, 4, 0), ((61, 95), 4, 5, 0), ((61, 95), 4, 5, 1),
                                              ((120, 160), 3, 4, 2), ((150, 211), 5, 4, 0)])
def test_learned_flow_fields_bit_exact(shape, L, T, passes, tiles):
    """Float-feature fields equal the oracle for the default variant table
    and with every scale on one variant (16x16 or 8x8 tiles, windows with a
    halo of 2, 4 or 6: with run length 0 the wider windows run two or three
    steps per launch)."""
    H, W = shape
    pad = 10
    canvas = feature_canvas(11 + H, H + 2 * pad, W + 2 * pad)
    F1 = canvas[pad:pad + H, pad:pad + W].copy()
    F2 = canvas[pad - 3:pad - 3 + H, pad + 2:pad + 2 + W].copy() + feature_canvas(12, H, W) * 0.05
    m1, m2 = feature_pyramid(F1, L), feature_pyramid(F2, L)
    prm = with_tuning(ff.Params(levels=L, iters=T), passes_f32=[passes] * 7,
                      **({} if tiles is None else {"variant_f32": [tiles] * 7}))
    o = oracle.flow_fields_f32(m1, m2, L, T, nthreads=NT)
    g = Lm.flow_fields_f32([torch.from_numpy(a).cuda() for a in m1], [torch.from_numpy(a).cuda() for a in m2], prm)
    torch.cuda.synchronize()
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(g[k].cpu().numpy(), o[k]), k
    for k in ("cost_fwd", "cost_bwd"):
        assert np.array_equal(g[k].cpu().numpy().view(np.uint32), o[k]), k
    assert tuple(int(v) for v in g["n_evals"].cpu()) == o["n_evals"]


def test_training_reduces_the_triplet_loss():
    from ffgen import make_pair
    net = Lm.DescNet(seed=0)
    prm = ff.Params(levels=3, iters=4)
    batch = []
    for k in range(4):
        p = make_pair(5, k, shape=(96, 128))
        i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
        o = ff.flow_fields(i1, i2, prm)
        batch.append((i1, i2, o["flow_fwd"], o["keep_fwd"]))
    rng = np.random.default_rng(0)
    losses = [Lm.train_step(net, batch, rng, samples=512, lr=3e-3) for _ in range(40)]
    assert np.isfinite(losses).all()
    assert np.mean(losses[-5:]) < 0.8 * np.mean(losses[:5]), losses


def test_learned_path_end_to_end_matches_oracle_on_the_network_features():
    """Scale images -> DescNet -> learned Flow Fields: the schedule on the
    GPU's own features is bit-exact to the oracle run on the same features."""
    from ffgen import make_pair
    net = Lm.DescNet(seed=3)
    p = make_pair(1, 0)
    prm = ff.Params(levels=3, iters=4)
    i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
    scales = Lm.scale_images(i1, i2, 3)
    feats = Lm.learned_features(net, scales)
    g = Lm.learned_flow_fields(net, i1, i2, prm, scales=scales)
    torch.cuda.synchronize()
    # the scale images are the plain path's blur, which the oracle pins
    sc = scales.cpu().numpy()
    for lv in range(3):
        assert np.array_equal(sc[lv], oracle.blur(p.img1, 1 << lv))
        assert np.array_equal(sc[3 + lv], oracle.blur(p.img2, 1 << lv))
    fc = feats.cpu().numpy()
    o = oracle.flow_fields_f32([fc[lv] for lv in range(3)], [fc[3 + lv] for lv in range(3)], 3, 4, nthreads=NT)
    for k in ("flow_fwd", "flow_bwd", "keep_fwd", "keep_bwd"):
        assert np.array_equal(g[k].cpu().numpy(), o[k]), k
    assert tuple(int(v) for v in g["n_evals"].cpu()) == o["n_evals"]


def test_triplet_hinge_kernel_and_gradient_match_autograd():
    """ff_triplet_hinge + ff_cost_f32_bwd give the loss and feature gradients
    of relu(margin + (C_pos - C_neg) / 49) summed and weighted: the loss and
    the cost gradient against float64 sums of the same costs, the feature
    gradients against the oracle's float64 gradient formula."""
    H, W = 40, 56
    g0 = torch.Generator().manual_seed(9)
    f1 = torch.randn((H, W, 16), generator=g0).cuda()
    f2 = torch.randn((H, W, 16), generator=g0).cuda()
    rng = np.random.default_rng(3)
    m = 300
    xs, ys = rng.integers(0, W, m), rng.integers(0, H, m)
    pos = np.stack([xs, ys, rng.integers(-xs, W - xs), rng.integers(-ys, H - ys)], 1)
    neg = np.stack([xs, ys, rng.integers(-xs, W - xs), rng.integers(-ys, H - ys)], 1)
    entries = torch.from_numpy(np.concatenate([pos, neg]).astype(np.int32)).cuda()
    margin, weight = 1.0, 1.0 / m
    cost = Lm.cost_f32(f1, f2, entries)
    loss, gcost = Lm.triplet_hinge(cost, m, margin, 1.0 / 49.0, weight)
    c = cost.double().cpu()
    h = margin + (c[:m] - c[m:]) / 49.0
    assert abs(float(loss) - float(torch.relu(h).sum()) * weight) <= 1e-5 * max(1.0, abs(float(loss)))
    on = (h > 0).double() * weight / 49.0
    assert torch.allclose(gcost.double().cpu(), torch.cat([on, -on]), rtol=1e-6, atol=0)
    assert 0 < int((h > 0).sum()) < m  # both branches exercised
    g1, g2 = Lm.cost_f32_grad(f1, f2, entries, gcost)
    # feature gradients of the hinge from the float64 formula of the oracle
    # (not the kernel): +-2 g (f1 - f2) per patch position, with g the
    # hinge's gradient of each cost; every contribution is computed in
    # float32 (2 roundings) and summed in 2^-32 fixed point
    from oracle.float_cost import grad_f64
    ent = entries.cpu().numpy().astype(np.int64)
    g64 = gcost.double().cpu().numpy()  # the float32 values the kernel scales by (checked above)
    e1, e2, s1, s2 = grad_f64(f1.cpu().double().numpy(), f2.cpu().double().numpy(), ent, g64)
    terms = 2 * m * 49
    for got, ref, absum in ((g1, e1, s1), (g2, e2, s2)):
        err = np.abs(got.cpu().double().numpy() - ref)
        assert np.all(err <= 4 * 2.0 ** -24 * absum + terms * 2.0 ** -33), float(err.max())


def test_quantize_pair_matches_oracle():
    f1 = feature_canvas(3, 40, 60)
    f2 = feature_canvas(4, 40, 60) * 2.5 - 1.0
    q1, q2 = Lm.quantize_pair_u8(torch.from_numpy(f1).cuda(), torch.from_numpy(f2).cuda())
    e1, e2 = oracle.quantize_pair_u8(f1, f2)
    assert np.array_equal(q1.cpu().numpy(), e1) and np.array_equal(q2.cpu().numpy(), e2)


@pytest.mark.parametrize("shape,L,T", [((120, 160), 3, 4), ((150, 211), 5, 4)])
def test_learned_level_kernel_costs_within_float64_bound(shape, L, T):
    """Independently of the summation order the kernels and the oracle
    share: every set cell's stored float32 cost lies within 784 * 2^-24
    (relative) of the float64 patch cost of its flow (non-negative terms:
    the float32 sum of 784 terms is within 784 u of the exact sum)."""
    from oracle.float_cost import cost_f64
    H, W = shape
    pad = 10
    canvas = feature_canvas(31 + H, H + 2 * pad, W + 2 * pad)
    F1 = canvas[pad:pad + H, pad:pad + W].copy()
    F2 = canvas[pad - 3:pad - 3 + H, pad + 2:pad + 2 + W].copy() + feature_canvas(32, H, W) * 0.05
    m1, m2 = feature_pyramid(F1, L), feature_pyramid(F2, L)
    g = Lm.flow_fields_f32([torch.from_numpy(a).cuda() for a in m1], [torch.from_numpy(a).cuda() for a in m2],
                           ff.Params(levels=L, iters=T))
    torch.cuda.synchronize()
    for fa, fb, fk, ck in ((F1, F2, "flow_fwd", "cost_fwd"), (F2, F1, "flow_bwd", "cost_bwd")):
        flow = g[fk].cpu().numpy()
        bits_ = g[ck].cpu().numpy().view(np.uint32)
        ys, xs = np.nonzero(bits_ != oracle.UNSET)
        assert len(ys) > 0.9 * H * W
        ent = np.stack([xs, ys, flow[ys, xs, 0], flow[ys, xs, 1]], 1)
        ref = cost_f64(fa, fb, ent, 1, 3)
        got = bits_[ys, xs].view(np.float32).astype(np.float64)
        assert np.all(np.abs(got - ref) <= 784 * 2.0 ** -24 * ref + 1e-30), float(np.max(np.abs(got - ref) / ref))


def test_cost_grad_overflow_gives_nan_not_a_wrapped_sum():
    """The fixed-point accumulators cover |sum| < 2^31: a single term of 2^31
    or more, and sums of smaller terms that pass 2^31, make every gradient
    output NaN; the next call within range clears the overflow count."""
    H, W = 12, 14
    f1 = torch.zeros((H, W, 16), device="cuda")
    f2 = torch.zeros((H, W, 16), device="cuda")
    f1[..., 0] = 1.0  # f1 - f2 = 1 in channel 0 everywhere
    one = torch.tensor([[3, 4, 2, 1]], dtype=torch.int32, device="cuda")
    acc = Lm.acc_scratch(W, H, "cuda")
    # one term 2 g (f1 - f2) = 2^31: out of range
    g1, g2 = Lm.cost_f32_grad(f1, f2, one, torch.tensor([2.0 ** 30], device="cuda"), acc=acc)
    assert torch.isnan(g1).all() and torch.isnan(g2).all()
    # terms of 2^30 each, three on the same pixels: the sum passes 2^31
    three = one.repeat(3, 1)
    g1, g2 = Lm.cost_f32_grad(f1, f2, three, torch.full((3,), 2.0 ** 29, device="cuda"), acc=acc)
    assert torch.isnan(g1).all() and torch.isnan(g2).all()
    # within range on the same scratch: finite, exact sums of the terms
    g1, g2 = Lm.cost_f32_grad(f1, f2, three, torch.full((3,), 2.0 ** 20, device="cuda"), acc=acc)
    assert torch.isfinite(g1).all() and torch.isfinite(g2).all()
    assert float(g1[..., 0].max()) == 3 * 2.0 ** 21 and float(g2[..., 0].min()) == -3 * 2.0 ** 21
    assert float(g1[..., 1:].abs().max()) == 0.0


@pytest.mark.parametrize("shape", [(1, 48, 64), (3, 37, 61), (2, 5, 3), (1, 1, 1), (1, 4, 121), (2, 436, 1024)])
@pytest.mark.parametrize("normalize", [True, False])
def test_fused_network_equals_the_layer_launches(shape, normalize):
    """ff_descnet_fwd (the whole network in one launch, activations on chip)
    gives the features of the three convolution launches and the
    normalisation launch bit for bit: ragged tiles (60 x 4 output pixels per
    workgroup), tiny and full-size frames, with non-zero biases."""
    B, H, W = shape
    net = Lm.DescNet(seed=3, normalize=normalize)
    g = torch.Generator().manual_seed(11)
    for k in range(3):
        net.b[k] = (torch.randn(net.b[k].shape, generator=g) * 0.1).cuda()
    img = (torch.rand((B, H, W), generator=g) * 255).round().to(torch.uint8).cuda()
    x = net.input_from_images(img)
    ref = net.forward(x)
    got = net.infer(x)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
