"""Pin of the float64 descriptor-network reference: autograd of the conv2d
formulation (with and without the per-pixel normalisation of the output)
against float64 central differences on a 64x48 crop, and the closed form of
the normalisation's gradient."""
import numpy as np
import pytest
import torch

from descnet_ref import LAYERS, forward


@pytest.mark.parametrize("delta", [None, 1e-4])
def test_reference_gradient_matches_central_differences(delta):
    g = torch.Generator().manual_seed(0)
    x = torch.rand((1, 48, 64, 1), generator=g, dtype=torch.float64) - 0.5
    ws = [torch.randn((cout, 9, cin), generator=g, dtype=torch.float64) * (2.0 / (9 * cin)) ** 0.5
          for cin, cout, _ in LAYERS]
    bs = [torch.randn(cout, generator=g, dtype=torch.float64) * 0.1 for _, cout, _ in LAYERS]
    probe = torch.randn((1, 48, 64, 16), generator=g, dtype=torch.float64)

    def loss(ws_, bs_):
        return (forward(x, ws_, bs_, delta=delta) * probe).sum()

    wr = [w.clone().requires_grad_(True) for w in ws]
    br = [b.clone().requires_grad_(True) for b in bs]
    loss(wr, br).backward()
    rng = np.random.default_rng(1)
    h = 1e-6
    for k in range(3):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in ws[k].shape)
            wp = [w.clone() for w in ws]
            wm = [w.clone() for w in ws]
            wp[k][idx] += h
            wm[k][idx] -= h
            num = float((loss(wp, bs) - loss(wm, bs)) / (2 * h))
            ana = float(wr[k].grad[idx])
            assert abs(num - ana) <= 1e-5 * max(1.0, abs(num)), (k, idx, num, ana)
        c = int(rng.integers(0, bs[k].shape[0]))
        bp = [b.clone() for b in bs]
        bm = [b.clone() for b in bs]
        bp[k][c] += h
        bm[k][c] -= h
        num = float((loss(ws, bp) - loss(ws, bm)) / (2 * h))
        assert abs(num - float(br[k].grad[c])) <= 1e-5 * max(1.0, abs(num))


def test_normalisation_gradient_closed_form():
    """d/df of <g, f / sqrt(|f|^2 + delta)> = r (g - y <g, y>), r = 1/sqrt(|f|^2 + delta)."""
    from descnet_ref import l2norm
    g0 = torch.Generator().manual_seed(4)
    f = torch.randn((3, 16, 5, 7), generator=g0, dtype=torch.float64).requires_grad_(True)
    g = torch.randn((3, 16, 5, 7), generator=g0, dtype=torch.float64)
    (l2norm(f, 1e-4) * g).sum().backward()
    r = 1.0 / torch.sqrt((f.detach() ** 2).sum(1, keepdim=True) + 1e-4)
    y = f.detach() * r
    closed = r * (g - y * (g * y).sum(1, keepdim=True))
    assert torch.allclose(f.grad, closed, rtol=1e-12, atol=1e-12)
    assert torch.allclose((y * y).sum(1), 1.0 - 1e-4 * r[:, 0] ** 2, rtol=1e-12)


def test_reference_chain_matches_central_differences():
    """reference_chain (the float64 chain the GPU network is compared with,
    element by element) is the exact derivative: 32 weights and 8 biases
    per layer against float64 central differences of the network with its
    bf16 activation roundings held fixed at their values (the kernels'
    backward treats those roundings as identity), within 1e-6 relative."""
    import numpy as np
    import torch.nn.functional as F

    from descnet_ref import LAYERS, bf16, reference_chain, torch_weight
    g = torch.Generator().manual_seed(2)
    x = bf16(torch.rand((1, 1, 48, 64), generator=g, dtype=torch.float64) - 0.5)
    ws = [bf16(torch.randn((cout, 9, cin), generator=g, dtype=torch.float64) * (2.0 / (9 * cin)) ** 0.5)
          for cin, cout, _ in LAYERS]
    bs = [(torch.randn(cout, generator=g, dtype=torch.float64) * 0.1).float().double() for _, cout, _ in LAYERS]
    probe = torch.randn((1, 16, 48, 64), generator=g, dtype=torch.float64)
    a, ys, gw_ref, gb_ref, _ = reference_chain(x, ws, bs, probe)
    offs = [a[k + 1] - torch.relu(ys[k]) for k in range(2)]  # frozen rounding offsets

    masks0 = [ys[k] > 0 for k in range(2)]

    def f(wl, bl):
        """Value, and whether every ReLU is on the same side as at the base
        point (the network is then linear in one parameter between the two
        points, and the central difference is exact up to rounding)."""
        h, same = x, True
        for k, (cin, cout, relu) in enumerate(LAYERS):
            h = F.conv2d(h, torch_weight(wl[k]), bl[k], padding=1)
            if relu:
                same = same and bool(torch.equal(h > 0, masks0[k]))
                h = torch.relu(h) + offs[k]
        return float((h * probe).sum()), same

    def central(plus, minus):
        (fp, sp), (fm, sm) = plus, minus
        return (fp - fm) / (2 * h), sp and sm

    rng = np.random.default_rng(9)
    h = 1e-5
    for k in range(3):
        done = 0
        while done < 32:  # samples whose difference crosses a ReLU kink are drawn again
            idx = tuple(int(rng.integers(0, s)) for s in ws[k].shape)
            wp, wm = [w.clone() for w in ws], [w.clone() for w in ws]
            wp[k][idx] += h
            wm[k][idx] -= h
            num, smooth = central(f(wp, bs), f(wm, bs))
            if not smooth:
                continue
            co, tap, ci = idx
            ana = float(gw_ref[k][co, ci, tap // 3, tap % 3])
            assert abs(num - ana) <= 1e-6 * max(abs(ana), 1.0), (k, idx, num, ana)
            done += 1
        done = 0
        while done < 8:
            c = int(rng.integers(0, bs[k].shape[0]))
            bp, bm = [b.clone() for b in bs], [b.clone() for b in bs]
            bp[k][c] += h
            bm[k][c] -= h
            num, smooth = central(f(ws, bp), f(ws, bm))
            if not smooth:
                continue
            assert abs(num - float(gb_ref[k][c])) <= 1e-6 * max(abs(float(gb_ref[k][c])), 1.0), (k, c)
            done += 1
