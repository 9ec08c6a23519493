"""The region filter entry point that allocates nothing (its scratch is the
library's static per-GPU array) against ff_region_filter, through the C ABI:
two calls in a row on one GPU, the second on a smaller image, so the second
call runs on the array the first one left behind."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_1703_02563_amd import ffi

pytestmark = pytest.mark.gpu


def _field(seed, H, W):
    rng = np.random.default_rng(seed)
    flow = np.zeros((H, W, 2), np.int16)
    # piecewise-constant flow with noise, so regions of many sizes form
    for _ in range(12):
        x0, y0 = rng.integers(0, W), rng.integers(0, H)
        w, h = rng.integers(1, max(2, W // 3)), rng.integers(1, max(2, H // 3))
        flow[y0:y0 + h, x0:x0 + w] = rng.integers(-20, 21, size=2)
    flow += rng.integers(-1, 2, size=flow.shape).astype(np.int16) * (rng.random((H, W, 1)) < 0.3)
    cost = rng.integers(0, 1000, size=(H, W)).astype(np.uint32)
    cost[rng.random((H, W)) < 0.05] = 0xFFFFFFFF
    keep = (rng.random((H, W)) < 0.8).astype(np.uint8)
    keep[cost == 0xFFFFFFFF] = 0
    return flow, cost, keep


def _both(flow, cost, keep, s):
    lib = ffi.lib()
    H, W = keep.shape
    dev = torch.device("cuda:0")
    f = torch.from_numpy(flow).to(dev)
    c = torch.from_numpy(cost.view(np.int32)).to(dev)
    k = torch.from_numpy(keep).to(dev)
    ref = torch.empty((H, W), dtype=torch.uint8, device=dev)
    got = torch.full((H, W), 7, dtype=torch.uint8, device=dev)
    nbytes = int(lib.ff_region_filter_scratch_bytes(W, H))
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    ffi.check(lib.ff_region_filter(P(f), P(c), P(k), W, H, s, P(scratch), nbytes, P(ref), stream),
              "ff_region_filter")
    ffi.check(lib.ff_region_filter_noalloc(P(f), P(c), P(k), W, H, s, P(got), stream), "ff_region_filter_noalloc")
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_region_filter_equals_scratch_variant_two_calls():
    # first a large image, then a smaller one on the array the first call left
    for seed, (H, W), s in ((1, (436, 1024), 50), (2, (97, 131), 20)):
        flow, cost, keep = _field(seed, H, W)
        ref, got = _both(flow, cost, keep, s)
        assert np.array_equal(got, ref), (H, W)
        assert np.array_equal(got, oracle.region_filter(flow, cost, keep, s)), (H, W)


def test_noalloc_region_filter_at_the_size_limit_and_beyond():
    lib = ffi.lib()
    maxpx = int(lib.ff_region_filter_noalloc_max_pixels())
    assert maxpx == 1 << 21
    H, W = 1024, maxpx // 1024  # exactly the limit
    flow, cost, keep = _field(3, H, W)
    ref, got = _both(flow, cost, keep, 30)
    assert np.array_equal(got, ref)
    fake = C.c_void_p(0x1000)
    assert lib.ff_region_filter_noalloc(fake, fake, fake, W + 1, H, 30, C.c_void_p(0x2000), None) == \
        ffi.FF_ERR_WORKSPACE
