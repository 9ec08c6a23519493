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
