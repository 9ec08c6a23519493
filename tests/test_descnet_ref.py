"""Pin of the float64 descriptor-network reference: autograd of the conv2d
formulation against float64 central differences on a 64x48 crop."""
import numpy as np
import torch

from descnet_ref import LAYERS, forward


def test_reference_gradient_matches_central_differences():
    g = torch.Generator().manual_seed(0)
    x = torch.rand((1, 48, 64, 1), generator=g, dtype=torch.float64) - 0.5
    ws = [torch.randn((cout, 9, cin), generator=g, dtype=torch.float64) * (2.0 / (9 * cin)) ** 0.5
          for cin, cout, _ in LAYERS]
    bs = [torch.randn(cout, generator=g, dtype=torch.float64) * 0.1 for _, cout, _ in LAYERS]
    probe = torch.randn((1, 48, 64, 16), generator=g, dtype=torch.float64)

    def loss(ws_, bs_):
        return (forward(x, ws_, bs_) * probe).sum()

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
