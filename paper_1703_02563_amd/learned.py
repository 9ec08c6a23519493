"""Learned-feature data term: float patch cost behind torch.autograd.

PatchCost wraps ff_cost_f32_fwd / ff_cost_f32_bwd (hand-written HIP
kernels): forward gives the squared-difference cost of the subsampled patch
for every entry (x, y, fx, fy); backward gives the gradients with respect to
both feature maps (deterministic, fixed-point accumulation).
"""
from __future__ import annotations

import torch

from .ffi import check, lib
from .flowfields import _ptr, _stream


def cost_f32(f1: torch.Tensor, f2: torch.Tensor, entries: torch.Tensor, n: int = 1, radius: int = 3):
    H, W, C = f1.shape
    if C != 16 or tuple(f2.shape) != (H, W, 16):
        raise ValueError("features must be float32 [H, W, 16]")
    count = entries.shape[0]
    cost = torch.empty(count, dtype=torch.float32, device=f1.device)
    check(lib().ff_cost_f32_fwd(_ptr(f1, torch.float32, "f1"), _ptr(f2, torch.float32, "f2"), W, H, n, radius,
                                _ptr(entries, torch.int32, "entries"), count, _ptr(cost), _stream()),
          "ff_cost_f32_fwd")
    return cost


def acc_scratch(W: int, H: int, device):
    """Scratch of ff_cost_f32_bwd: two int64 [H, W, 16] accumulators and one
    overflow word."""
    return torch.empty(2 * H * W * 16 + 1, dtype=torch.int64, device=device)


def cost_f32_grad(f1, f2, entries, grad_cost, n: int = 1, radius: int = 3, out=None, acc=None):
    """Gradients (d/df1, d/df2) of sum_e grad_cost[e] * cost[e]; `out` may
    name the two output tensors, `acc` the int64 [2 * H * W * 16 + 1] scratch
    (the accumulators and their overflow count; the gradients are NaN when it
    is nonzero)."""
    H, W, _ = f1.shape
    if acc is None:
        acc = acc_scratch(W, H, f1.device)
    if acc.dtype != torch.int64 or acc.numel() < 2 * H * W * 16 + 1 or not acc.is_contiguous():
        raise ValueError("acc: contiguous int64 scratch of 2 * H * W * 16 + 1 words expected")
    g1, g2 = out if out is not None else (torch.empty_like(f1), torch.empty_like(f2))
    check(lib().ff_cost_f32_bwd(_ptr(f1, torch.float32, "f1"), _ptr(f2, torch.float32, "f2"), W, H, n, radius,
                                _ptr(entries, torch.int32, "entries"), entries.shape[0],
                                _ptr(grad_cost, torch.float32, "grad_cost"), _ptr(acc), _ptr(g1), _ptr(g2),
                                _stream()), "ff_cost_f32_bwd")
    return g1, g2


class PatchCost(torch.autograd.Function):
    """cost[e] = sum over the (2r+1)^2 subsampled patch of |f1 - f2(+flow)|^2."""

    @staticmethod
    def forward(ctx, f1, f2, entries, n: int = 1, radius: int = 3):
        f1 = f1.contiguous()
        f2 = f2.contiguous()
        entries = entries.contiguous()
        ctx.save_for_backward(f1, f2, entries)
        ctx.n, ctx.radius = n, radius
        return cost_f32(f1, f2, entries, n, radius)

    @staticmethod
    def backward(ctx, grad_cost):
        f1, f2, entries = ctx.saved_tensors
        g1, g2 = cost_f32_grad(f1, f2, entries, grad_cost.contiguous().float(), ctx.n, ctx.radius)
        return g1, g2, None, None, None


def patch_cost(f1, f2, entries, n: int = 1, radius: int = 3):
    return PatchCost.apply(f1, f2, entries, n, radius)


# ---------------------------------------------------------------------------
# DescNet: three 3x3 convolutions 1 -> 32 -> 32 -> 16 (ReLU after the first
# two), bf16 weights and activations, float32 accumulation, all passes in the
# library's kernels.  Float32 master weights, Adam in a kernel.
# ---------------------------------------------------------------------------

import ctypes as _C
import math as _math

LAYERS = ((1, 32, True), (32, 32, True), (32, 16, False))


def _bf16_bits(t: torch.Tensor) -> torch.Tensor:
    """float32 tensor -> uint16 bit patterns of its bf16 rounding (kernel)."""
    t = t.contiguous().float()
    out = torch.empty(t.shape, dtype=torch.int16, device=t.device)
    check(lib().ff_f32_to_bf16(_ptr(t, torch.float32), t.numel(), _ptr(out), _stream()), "ff_f32_to_bf16")
    return out


def bf16_bits_to_f32(bits: torch.Tensor) -> torch.Tensor:
    """uint16 bf16 bit patterns (int16 tensor) -> float32 (exact)."""
    return (bits.to(torch.int32) << 16).view(torch.float32)


class DescNet:
    """Weights, Adam state and the forward/backward passes of the network."""

    def __init__(self, seed: int = 0, device="cuda", normalize: bool = True, delta: float = 1e-4):
        g = torch.Generator().manual_seed(seed)
        self.device = torch.device(device)
        # unit-length output features: the triplet margin then has a fixed
        # scale (squared distances per pixel in [0, 4])
        self.normalize, self.delta = normalize, float(delta)
        self.w, self.b = [], []
        for cin, cout, _ in LAYERS:
            std = _math.sqrt(2.0 / (9 * cin))
            self.w.append((torch.randn((cout, 9, cin), generator=g) * std).float().to(self.device))
            self.b.append(torch.zeros(cout, dtype=torch.float32, device=self.device))
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step = 0
        self._sync_bf16()

    def _sync_bf16(self):
        self.wb = [_bf16_bits(w) for w in self.w]

    def state_dict(self):
        return {"w": [w.cpu() for w in self.w], "b": [b.cpu() for b in self.b], "step": self.step}

    def load_state_dict(self, sd):
        self.w = [w.to(self.device).float() for w in sd["w"]]
        self.b = [b.to(self.device).float() for b in sd["b"]]
        self.step = int(sd.get("step", 0))
        self._sync_bf16()

    def input_from_images(self, imgs: torch.Tensor) -> torch.Tensor:
        """uint8 [B, H, W] -> bf16 bits [B, H, W, 1] (v / 255 - 0.5)."""
        imgs = imgs.contiguous()
        out = torch.empty(imgs.shape + (1,), dtype=torch.int16, device=imgs.device)
        check(lib().ff_image_to_bf16(_ptr(imgs, torch.uint8), imgs.numel(), _ptr(out), _stream()), "ff_image_to_bf16")
        return out

    def forward(self, x_bits: torch.Tensor, keep: bool = False):
        """x_bits: bf16 bits [B, H, W, 1]; returns float32 features [B, H, W, 16]
        (and the bf16 activations of every layer input when keep=True)."""
        B, H, W, _ = x_bits.shape
        acts = [x_bits]
        out = None
        for k, (cin, cout, relu) in enumerate(LAYERS):
            last = k == len(LAYERS) - 1
            o32 = torch.empty((B, H, W, cout), dtype=torch.float32, device=x_bits.device) if last else None
            o16 = None if last else torch.empty((B, H, W, cout), dtype=torch.int16, device=x_bits.device)
            check(lib().ff_conv3x3_fwd(_ptr(acts[-1]), B, H, W, cin, cout, _ptr(self.wb[k]), _ptr(self.b[k]),
                                       int(relu), _ptr(o32), _ptr(o16), _stream()), "ff_conv3x3_fwd")
            if last:
                out = o32
            else:
                acts.append(o16)
        if self.normalize:
            inv = torch.empty((B, H, W), dtype=torch.float32, device=x_bits.device)
            check(lib().ff_l2norm16_fwd(_ptr(out), out.numel() // 16, self.delta, _ptr(out), _ptr(inv), _stream()),
                  "ff_l2norm16_fwd")
            acts.append((out, inv))
        return (out, acts) if keep else out

    def backward(self, acts, grad_out: torch.Tensor):
        """Gradients (w, b) of all layers for upstream float32 grad_out
        [B, H, W, 16] of the features."""
        B, H, W, _ = grad_out.shape
        gws, gbs = [None] * 3, [None] * 3
        g32 = grad_out.contiguous().float()
        if self.normalize:
            y, inv = acts[len(LAYERS)]
            gn = torch.empty_like(g32)
            check(lib().ff_l2norm16_bwd(_ptr(y), _ptr(inv), _ptr(g32, torch.float32), g32.numel() // 16, _ptr(gn),
                                        _stream()), "ff_l2norm16_bwd")
            g32 = gn
        for k in range(len(LAYERS) - 1, -1, -1):
            cin, cout, relu = LAYERS[k]
            nbytes = int(lib().ff_conv3x3_wgrad_scratch_bytes(B, H, cin, cout))
            scratch = torch.empty(nbytes // 4, dtype=torch.float32, device=grad_out.device)
            gw = torch.empty((cout, 9, cin), dtype=torch.float32, device=grad_out.device)
            gb = torch.empty(cout, dtype=torch.float32, device=grad_out.device)
            check(lib().ff_conv3x3_bwd_weight(_ptr(acts[k]), _ptr(g32, torch.float32), B, H, W, cin, cout,
                                              _ptr(scratch), nbytes, _ptr(gw), _ptr(gb), _stream()),
                  "ff_conv3x3_bwd_weight")
            gws[k], gbs[k] = gw, gb
            if k == 0:
                break
            # gradient of the layer input, then through the previous ReLU
            g16 = _bf16_bits(g32)
            flip = torch.empty((cin, 9, cout), dtype=torch.int16, device=grad_out.device)
            gin = torch.empty((B, H, W, cin), dtype=torch.float32, device=grad_out.device)
            check(lib().ff_conv3x3_bwd_data(_ptr(g16), B, H, W, cin, cout, _ptr(self.wb[k]), _ptr(flip), _ptr(gin),
                                            None, _stream()), "ff_conv3x3_bwd_data")
            g32 = torch.empty_like(gin)
            check(lib().ff_relu_bwd(_ptr(acts[k]), _ptr(gin, torch.float32), gin.numel(), _ptr(g32), None,
                                    _stream()), "ff_relu_bwd")
        return gws, gbs

    def adam(self, gws, gbs, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        params = self.w + self.b
        grads = gws + gbs
        for k, (p, g) in enumerate(zip(params, grads)):
            wbits = self.wb[k] if k < len(self.w) else None
            g = g.contiguous()  # named, so the buffer outlives the launch
            check(lib().ff_adam_step(_ptr(p, torch.float32), _ptr(g, torch.float32), _ptr(self.m[k]),
                                     _ptr(self.v[k]), p.numel(), lr, b1, b2, eps, self.step, _ptr(wbits), _stream()),
                  "ff_adam_step")

    def infer(self, x_bits: torch.Tensor) -> torch.Tensor:
        """Inference of the whole network in one launch (ff_descnet_fwd):
        the same float32 features [B, H, W, 16] as forward(), bit for bit."""
        B, H, W, _ = x_bits.shape
        out = torch.empty((B, H, W, 16), dtype=torch.float32, device=x_bits.device)
        check(lib().ff_descnet_fwd(_ptr(x_bits), B, H, W, _ptr(self.wb[0]), _ptr(self.b[0]), _ptr(self.wb[1]),
                                   _ptr(self.b[1]), _ptr(self.wb[2]), _ptr(self.b[2]), int(self.normalize), self.delta,
                                   _ptr(out), _stream()), "ff_descnet_fwd")
        return out

    def features(self, img: torch.Tensor) -> torch.Tensor:
        """uint8 [H, W] -> float32 [H, W, 16]."""
        return self.forward(self.input_from_images(img[None]))[0]


class TripletSampler:
    """Anchors for the triplet loss of one image pair: the pixels kept by the
    plain method's consistency check, with their plain flows (host copy made
    once).  sample() draws anchors p, the positive p + F(p) and a negative =
    positive + an offset of Chebyshev radius 2..8 px that stays in the image."""

    def __init__(self, flow: torch.Tensor, keep: torch.Tensor):
        import numpy as np
        self.H, self.W = keep.shape
        k = keep.cpu().numpy().astype(bool)
        f = flow.cpu().numpy().astype(np.int64)
        self.ys, self.xs = np.nonzero(k)
        self.fx, self.fy = f[self.ys, self.xs, 0], f[self.ys, self.xs, 1]

    def __len__(self):
        return len(self.xs)

    def sample(self, count: int, rng, negatives: int = 1):
        """int32 entries (x, y, fx, fy): positives [m, 4] and negatives
        [m, 4] (negatives == 1) or [m, negatives, 4] candidates, m <= count.
        A candidate offset that fails (radius < 2 or out of the image) is
        replaced by the anchor's first valid one."""
        import numpy as np
        if len(self.xs) == 0:
            raise ValueError("no consistent matches")
        K = max(1, int(negatives))
        sel = rng.integers(0, len(self.xs), size=count * 2)
        xs, ys, fx, fy = self.xs[sel], self.ys[sel], self.fx[sel], self.fy[sel]
        ox = rng.integers(-8, 9, size=(len(xs), K))
        oy = rng.integers(-8, 9, size=(len(xs), K))
        tx, ty = (xs + fx)[:, None] + ox, (ys + fy)[:, None] + oy
        ok = (np.maximum(np.abs(ox), np.abs(oy)) >= 2) & (tx >= 0) & (tx < self.W) & (ty >= 0) & (ty < self.H)
        idx = np.nonzero(ok.any(1))[0][:count]
        ok, ox, oy = ok[idx], ox[idx], oy[idx]
        first = ok.argmax(1)
        r = np.arange(len(idx))
        ox = np.where(ok, ox, ox[r, first][:, None])
        oy = np.where(ok, oy, oy[r, first][:, None])
        pos = np.stack([xs[idx], ys[idx], fx[idx], fy[idx]], 1).astype(np.int32)
        neg = np.stack([np.broadcast_to(xs[idx, None], ox.shape), np.broadcast_to(ys[idx, None], ox.shape),
                        fx[idx, None] + ox, fy[idx, None] + oy], 2).astype(np.int32)
        return pos, (neg[:, 0] if negatives == 1 else neg)


def triplets(flow: torch.Tensor, keep: torch.Tensor, count: int, rng):
    """One-off TripletSampler(flow, keep).sample(count, rng)."""
    return TripletSampler(flow, keep).sample(count, rng)


def triplet_hinge(cost: torch.Tensor, m: int, margin: float, scale: float, weight: float):
    """ff_triplet_hinge: (loss [1], grad_cost [2m]) of costs [2m] (positives, then negatives)."""
    grad = torch.empty_like(cost)
    loss = torch.empty(1, dtype=torch.float32, device=cost.device)
    check(lib().ff_triplet_hinge(_ptr(cost, torch.float32), m, margin, scale, weight, _ptr(grad), _ptr(loss),
                                 _stream()), "ff_triplet_hinge")
    return loss, grad


def train_step(net: DescNet, batch, rng, samples: int = 4096, margin: float = 1.0, lr: float = 1e-3,
               negatives: int = 1):
    """One Adam step of the triplet hinge max(0, margin + (C(p, pos) - C(p, neg)) / 49)
    averaged over anchors of every pair in `batch` = [(img1, img2, flow, keep)]
    (or [(img1, img2, TripletSampler)]) with the plain method's flows and
    consistency masks.  The costs enter as means over the 49 patch samples
    (per-pixel squared distances of unit features lie in [0, 4], so the
    margin has a fixed scale).  With negatives > 1 each anchor draws that many
    candidate negatives and keeps the one of lowest current cost (hardest).
    Every pass runs in the library's kernels: network forward, patch costs,
    hinge, cost backward into the feature gradient, network backward, Adam.
    Triplet sampling is host-side data preparation."""
    B = len(batch)
    imgs = torch.stack([b[0] for b in batch] + [b[1] for b in batch])   # [2B, H, W]
    feats, acts = net.forward(net.input_from_images(imgs), keep=True)
    dev = feats.device
    H, W = imgs.shape[1:]
    picks = []
    for k, item in enumerate(batch):
        sampler = item[2] if len(item) == 3 else TripletSampler(item[2], item[3])
        pos, neg = sampler.sample(samples, rng, negatives)
        pe = torch.from_numpy(pos).to(dev)
        ne = torch.from_numpy(neg).to(dev)
        if negatives > 1 and len(pos):
            cand = ne.reshape(-1, 4).contiguous()
            c = cost_f32(feats[k], feats[B + k], cand, 1, 3).reshape(len(pos), negatives)
            ne = ne[torch.arange(len(pos), device=dev), c.argmin(1)]
        picks.append(torch.cat([pe, ne]).contiguous())
    total = sum(len(e) // 2 for e in picks)
    grad = torch.empty_like(feats)
    acc = acc_scratch(W, H, dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    for k, entries in enumerate(picks):
        m = len(entries) // 2
        gcost = torch.empty(0, dtype=torch.float32, device=dev)
        if m:
            cost = cost_f32(feats[k], feats[B + k], entries, 1, 3)
            lk, gcost = triplet_hinge(cost, m, margin, 1.0 / 49.0, 1.0 / max(total, 1))
            loss += lk
        # with no entries the backward writes zero gradients
        cost_f32_grad(feats[k], feats[B + k], entries, gcost, 1, 3, out=(grad[k], grad[B + k]), acc=acc)
    gws, gbs = net.backward(acts, grad)
    net.adam(gws, gbs, lr=lr)
    return float(loss)


def scale_images(img1: torch.Tensor, img2: torch.Tensor, levels: int) -> torch.Tensor:
    """Scale-space images B_n (n = 2^l) of both images, uint8 [2L, H, W]:
    rows 0..L-1 are img1's scales, rows L..2L-1 img2's."""
    from .flowfields import descriptors
    return torch.stack([descriptors(img, 1 << lv)[0] for img in (img1, img2) for lv in range(levels)])


def learned_features(net: DescNet, scales: torch.Tensor) -> torch.Tensor:
    """DescNet features of every scale image in one launch: float32 [2L, H, W, 16]."""
    return net.infer(net.input_from_images(scales))


def learned_flow_fields(net: DescNet, img1: torch.Tensor, img2: torch.Tensor, params, scales=None) -> dict:
    """Flow Fields on DescNet features of the scale-space images B_n
    (ff_flow_fields_f32).  Returns the same keys as flow_fields; costs are
    float32 bit patterns."""
    L = params.levels
    if scales is None:
        scales = scale_images(img1, img2, L)
    feats = learned_features(net, scales)
    return flow_fields_f32([feats[lv] for lv in range(L)], [feats[L + lv] for lv in range(L)], params)


def flow_fields_f32(f1, f2, params) -> dict:
    """ff_flow_fields_f32 on per-scale float32 feature maps [H, W, 16]."""
    H, W, _ = f1[0].shape
    L = params.levels
    cp = params.to_c()
    dev = f1[0].device
    nbytes = int(lib().ff_workspace_bytes_f32(W, H, cp))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = {
        "flow_fwd": torch.empty((H, W, 2), dtype=torch.int16, device=dev),
        "flow_bwd": torch.empty((H, W, 2), dtype=torch.int16, device=dev),
        "cost_fwd": torch.empty((H, W), dtype=torch.int32, device=dev),
        "cost_bwd": torch.empty((H, W), dtype=torch.int32, device=dev),
        "keep_fwd": torch.empty((H, W), dtype=torch.uint8, device=dev),
        "keep_bwd": torch.empty((H, W), dtype=torch.uint8, device=dev),
        "n_evals": torch.zeros(2, dtype=torch.int64, device=dev),
    }
    a1 = (_C.c_void_p * L)(*[t.data_ptr() for t in f1])
    a2 = (_C.c_void_p * L)(*[t.data_ptr() for t in f2])
    for t in list(f1) + list(f2):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (H, W, 16):
            raise ValueError("features must be contiguous float32 CUDA tensors [H, W, 16]")
    check(lib().ff_flow_fields_f32(_C.cast(a1, _C.c_void_p), _C.cast(a2, _C.c_void_p), W, H, cp, _ptr(ws),
                                   ws.numel(), _ptr(out["flow_fwd"]), _ptr(out["flow_bwd"]), _ptr(out["cost_fwd"]),
                                   _ptr(out["cost_bwd"]), _ptr(out["keep_fwd"]), _ptr(out["keep_bwd"]),
                                   _ptr(out["n_evals"]), _stream()), "ff_flow_fields_f32")
    return out


def quantize_u8(f: torch.Tensor) -> torch.Tensor:
    f = f.contiguous()
    q = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
    scratch = torch.empty(int(lib().ff_quantize_scratch_bytes()) // 4, dtype=torch.float32, device=f.device)
    check(lib().ff_quantize_u8(_ptr(f, torch.float32), f.numel(), _ptr(scratch), _ptr(q), _stream()),
          "ff_quantize_u8")
    return q


def quantize_pair_u8(f1: torch.Tensor, f2: torch.Tensor):
    """Both maps to bytes with the range of their union (ff_quantize_pair_u8)."""
    f1, f2 = f1.contiguous(), f2.contiguous()
    if f1.shape != f2.shape:
        raise ValueError("quantize_pair_u8: maps of the same shape")
    q1 = torch.empty(f1.shape, dtype=torch.uint8, device=f1.device)
    q2 = torch.empty(f2.shape, dtype=torch.uint8, device=f2.device)
    scratch = torch.empty(int(lib().ff_quantize_scratch_bytes()) // 4, dtype=torch.float32, device=f1.device)
    check(lib().ff_quantize_pair_u8(_ptr(f1, torch.float32), _ptr(f2, torch.float32), f1.numel(), _ptr(scratch),
                                    _ptr(q1), _ptr(q2), _stream()), "ff_quantize_pair_u8")
    return q1, q2
