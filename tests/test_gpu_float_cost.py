"""Float patch cost kernels (forward and hand-written backward) against the
float64 oracle, float64 central finite differences, and determinism."""
import numpy as np
import pytest
import torch

from oracle.float_cost import cost_f64, grad_f64
from paper_1703_02563_amd.learned import cost_f32, cost_f32_grad, patch_cost

pytestmark = pytest.mark.gpu

# float32 accumulation of at most 49*16 non-negative terms, one rounding
# each: relative error <= 784 * 2^-24 < 5e-5 of the sum
COST_RTOL = 5e-5
# gradients: each term is formed in float64 and rounded to 2^-32 units,
# the fixed-point sum is exact and the final conversion rounds once to
# float32: |err| <= 2^-24 |g| + terms * 2^-33
GRAD_RTOL, GRAD_ATOL = 2 ** -23, 1e-7


def _case(seed, H, W, count, fmax, scale=1.0):
    rng = np.random.default_rng(seed)
    f1 = (rng.normal(size=(H, W, 16)) * scale).astype(np.float32)
    f2 = (rng.normal(size=(H, W, 16)) * scale).astype(np.float32)
    ent = np.stack([rng.integers(0, W, count), rng.integers(0, H, count), rng.integers(-fmax, fmax + 1, count),
                    rng.integers(-fmax, fmax + 1, count)], 1).astype(np.int32)
    g = rng.normal(size=count).astype(np.float32)
    return f1, f2, ent, g


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("H,W,count,n,r", [(48, 64, 500, 1, 3), (37, 53, 333, 2, 3), (20, 30, 101, 1, 1),
                                          (120, 160, 4000, 4, 3), (1, 7, 9, 1, 3), (64, 48, 1, 1, 0)])
def test_cost_forward_matches_f64(H, W, count, n, r):
    f1, f2, ent, _ = _case(H + count, H, W, count, 12)
    ref = cost_f64(f1, f2, ent, n, r)
    got = cost_f32(cuda(f1), cuda(f2), cuda(ent), n, r).cpu().numpy()
    assert np.all(np.abs(got - ref) <= COST_RTOL * ref + 1e-6)


@pytest.mark.parametrize("H,W,count,n,r", [(48, 64, 400, 1, 3), (37, 53, 300, 2, 3), (20, 30, 101, 1, 1),
                                          (1, 7, 9, 1, 3), (64, 48, 50, 1, 0)])
def test_cost_forward_bit_exact_vs_oracle(H, W, count, n, r):
    """Same fixed summation order as the oracle's single-precision cost:
    identical bits, entry by entry (borders and out-of-image targets
    included)."""
    import oracle
    f1, f2, ent, _ = _case(3 * H + count, H, W, count, 12)
    got = cost_f32(cuda(f1), cuda(f2), cuda(ent), n, r).cpu().numpy()
    ref = np.array([oracle.cost_f32(f1, f2, n, r, *map(int, e)) for e in ent], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("H,W,count,n,r", [(48, 64, 300, 1, 3), (37, 53, 200, 2, 3), (120, 160, 2000, 1, 3),
                                          (9, 11, 40, 1, 2)])
def test_cost_backward_matches_f64(H, W, count, n, r):
    f1, f2, ent, g = _case(7 * H + count, H, W, count, 10)
    e1, e2, a1, a2 = grad_f64(f1, f2, ent, g, n, r)
    g1, g2 = cost_f32_grad(cuda(f1), cuda(f2), cuda(ent), cuda(g), n, r)
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    terms = count * (2 * r + 1) ** 2
    assert np.all(np.abs(g1 - e1) <= GRAD_RTOL * np.abs(e1) + terms * 2.0 ** -33 + GRAD_ATOL)
    assert np.all(np.abs(g2 - e2) <= GRAD_RTOL * np.abs(e2) + terms * 2.0 ** -33 + GRAD_ATOL)


def test_autograd_against_central_differences_64x48():
    """Analytic GPU gradient vs float64 central differences of the oracle."""
    H, W, n, r = 48, 64, 1, 3
    f1, f2, ent, gout = _case(31, H, W, 64, 12)
    t1 = cuda(f1).requires_grad_(True)
    t2 = cuda(f2).requires_grad_(True)
    loss = (patch_cost(t1, t2, cuda(ent), n, r) * cuda(gout)).sum()
    loss.backward()
    g1, g2 = t1.grad.cpu().numpy(), t2.grad.cpu().numpy()
    f1d, f2d = f1.astype(np.float64), f2.astype(np.float64)
    rng = np.random.default_rng(32)
    h = 1e-4
    for which, base, grad in ((0, f1d, g1), (1, f2d, g2)):
        hot = np.argwhere(np.abs(grad) > 0)
        for i in rng.choice(len(hot), 40, replace=False):
            idx = tuple(hot[i])
            plus, minus = base.copy(), base.copy()
            plus[idx] += h
            minus[idx] -= h
            a = (f1d, plus) if which else (plus, f2d)
            b = (f1d, minus) if which else (minus, f2d)
            num = (np.dot(cost_f64(*a, ent, n, r), gout) - np.dot(cost_f64(*b, ent, n, r), gout)) / (2 * h)
            assert abs(num - grad[idx]) <= 1e-4 * max(1.0, abs(num)), (which, idx, num, grad[idx])


def test_backward_is_deterministic():
    f1, f2, ent, g = _case(41, 96, 128, 5000, 4)   # many entries hit the same pixels
    a = [x.cpu().numpy() for x in cost_f32_grad(cuda(f1), cuda(f2), cuda(ent), cuda(g), 1, 3)]
    b = [x.cpu().numpy() for x in cost_f32_grad(cuda(f1), cuda(f2), cuda(ent), cuda(g), 1, 3)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_empty_entries():
    f1, f2, _, _ = _case(1, 8, 8, 1, 1)
    e = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    assert cost_f32(cuda(f1), cuda(f2), e).numel() == 0
    g1, g2 = cost_f32_grad(cuda(f1), cuda(f2), e, torch.zeros(0, device="cuda"))
    assert float(g1.abs().sum()) == 0.0 and float(g2.abs().sum()) == 0.0
