"""Pins of the float patch-cost oracle (learned-feature data term).

The cost is pinned against an independent formulation with a library
routine (torch.nn.functional.unfold over edge-replicated maps, float64) and
closed forms; the gradient against torch autograd of that formulation and
against float64 central finite differences.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle.float_cost import cost_f64, grad_f64


def _feats(seed, H, W, C=16):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(H, W, C)), rng.normal(size=(H, W, C))


def _unfold_cost(f1, f2, entries, n, r):
    """Same cost from unfold: pad both maps by replication far enough that no
    read is clamped, take the (2r+1)^2 dilated patches of every pixel, pick the
    entries' pixels and targets."""
    t1 = f1.permute(2, 0, 1)[None]
    t2 = f2.permute(2, 0, 1)[None]
    H, W = f1.shape[:2]
    pad = r * n + max(abs(int(e[2])) + abs(int(e[3])) for e in entries) + 1
    P1 = F.pad(t1, (pad, pad, pad, pad), mode="replicate")
    P2 = F.pad(t2, (pad, pad, pad, pad), mode="replicate")
    k = 2 * r + 1
    U1 = F.unfold(P1, kernel_size=k, dilation=n)   # [1, C*k*k, L]
    U2 = F.unfold(P2, kernel_size=k, dilation=n)
    Wp = W + 2 * pad - n * (k - 1)
    out = []
    for x, y, fx, fy in entries:
        # patch whose centre is pixel (x, y): its top-left in padded coords
        i1 = (y + pad - r * n) * Wp + (x + pad - r * n)
        i2 = (y + fy + pad - r * n) * Wp + (x + fx + pad - r * n)
        d = U1[0, :, i1] - U2[0, :, i2]
        out.append((d * d).sum())
    return torch.stack(out)


def _entries(seed, H, W, count, fmax):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, W, count)
    y = rng.integers(0, H, count)
    fx = rng.integers(-fmax, fmax + 1, count)
    fy = rng.integers(-fmax, fmax + 1, count)
    return np.stack([x, y, fx, fy], 1).astype(np.int32)


@pytest.mark.parametrize("n,r", [(1, 3), (2, 3), (1, 1), (4, 2)])
def test_cost_matches_unfold_formulation(n, r):
    # targets that leave the frame: the unfold path clamps through replicate padding
    H, W = 20, 27
    f1, f2 = _feats(n + r, H, W)
    ent = _entries(3, H, W, 40, 6)
    c = cost_f64(f1, f2, ent, n, r)
    ref = _unfold_cost(torch.from_numpy(f1), torch.from_numpy(f2), ent, n, r).numpy()
    np.testing.assert_allclose(c, ref, rtol=1e-12, atol=1e-12)


def test_cost_closed_forms():
    H, W = 9, 11
    f1 = np.full((H, W, 16), 1.5)
    f2 = np.full((H, W, 16), -0.5)
    ent = np.array([[4, 4, 1, -2], [0, 0, -3, 5]], np.int32)
    assert np.allclose(cost_f64(f1, f2, ent, 1, 3), 49 * 16 * 4.0)
    g, _ = _feats(1, H, W)
    assert np.allclose(cost_f64(g, g, np.array([[5, 3, 0, 0]]), 2, 3), 0.0)
    g1, g2, _, _ = grad_f64(g, g, np.array([[5, 3, 0, 0]]), [1.0], 2, 3)
    assert np.allclose(g1, 0) and np.allclose(g2, 0)


@pytest.mark.parametrize("n", [1, 2])
def test_gradient_matches_autograd_of_unfold(n):
    H, W, r = 16, 19, 3
    f1, f2 = _feats(10 + n, H, W)
    ent = _entries(4 + n, H, W, 25, 5)
    gout = np.random.default_rng(5).normal(size=len(ent))
    t1 = torch.from_numpy(f1).requires_grad_(True)
    t2 = torch.from_numpy(f2).requires_grad_(True)
    (_unfold_cost(t1, t2, ent, n, r) * torch.from_numpy(gout)).sum().backward()
    g1, g2, _, _ = grad_f64(f1, f2, ent, gout, n, r)
    np.testing.assert_allclose(g1, t1.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g2, t2.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_gradient_matches_central_differences():
    """64x48 crop (the size of the learned-descriptor gradient check)."""
    H, W, n, r = 48, 64, 1, 3
    f1, f2 = _feats(21, H, W)
    ent = _entries(22, H, W, 30, 12)
    gout = np.random.default_rng(23).normal(size=len(ent))
    g1, g2, _, _ = grad_f64(f1, f2, ent, gout, n, r)
    rng = np.random.default_rng(24)
    h = 1e-6
    for which, base, grad in ((0, f1, g1), (1, f2, g2)):
        # probe elements that receive gradient and a few that do not
        hot = np.argwhere(np.abs(grad) > 0)
        picks = [tuple(hot[i]) for i in rng.choice(len(hot), 25, replace=False)]
        picks += [tuple(rng.integers(0, s) for s in base.shape) for _ in range(5)]
        for idx in picks:
            plus, minus = base.copy(), base.copy()
            plus[idx] += h
            minus[idx] -= h
            a = (f1, plus) if which else (plus, f2)
            b = (f1, minus) if which else (minus, f2)
            num = (np.dot(cost_f64(*a, ent, n, r), gout) - np.dot(cost_f64(*b, ent, n, r), gout)) / (2 * h)
            assert abs(num - grad[idx]) <= 1e-5 * max(1.0, abs(num)), (which, idx, num, grad[idx])
