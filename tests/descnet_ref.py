"""Float64 reference of the descriptor network (torch.nn.functional.conv2d),
optionally rounding to bfloat16 where the GPU kernels round."""
import torch
import torch.nn.functional as F

LAYERS = ((1, 32, True), (32, 32, True), (32, 16, False))


def torch_weight(w):
    """[cout][9][cin] (tap = 3*ky + kx) -> conv2d layout [cout][cin][3][3]."""
    cout, _, cin = w.shape
    return w.reshape(cout, 3, 3, cin).permute(0, 3, 1, 2)


def bf16(t):
    return t.to(torch.bfloat16).to(t.dtype)


def l2norm(h, delta):
    """Per-pixel unit length over the channel axis (dim 1): h / sqrt(|h|^2 + delta)."""
    return h / torch.sqrt((h * h).sum(1, keepdim=True) + delta)


def forward(x, ws, bs, round_bf16=False, delta=None):
    """x: [B, H, W, 1] -> features [B, H, W, 16] (float64); delta not None
    appends the per-pixel normalisation of the output."""
    h = x.permute(0, 3, 1, 2)
    for k, (cin, cout, relu) in enumerate(LAYERS):
        w = torch_weight(bf16(ws[k]) if round_bf16 else ws[k])
        h = F.conv2d(h, w, bs[k], padding=1)
        if relu:
            h = torch.relu(h)
        if round_bf16 and k < len(LAYERS) - 1:
            h = bf16(h)
    if delta is not None:
        h = l2norm(h, delta)
    return h.permute(0, 2, 3, 1)


def reference_chain(x, ws, bs, probe):
    """The network's forward in float64 with the kernels' rounding points
    (bf16 activations after the first two layers) and its exact float64
    backward (no gradient rounding): per layer the activations a_k, outputs
    y_k, and the weight, bias and upstream gradients."""
    a, ys = [x], []
    for k, (cin, cout, relu) in enumerate(LAYERS):
        y = F.conv2d(a[-1], torch_weight(ws[k]), bs[k], padding=1)
        ys.append(y)
        if relu:
            a.append(bf16(torch.relu(y)))
    g = probe
    gw, gb, gy = [None] * 3, [None] * 3, [None] * 3
    for k in (2, 1, 0):
        gy[k] = g
        gw[k] = torch.nn.grad.conv2d_weight(a[k], torch_weight(ws[k]).shape, g, padding=1)
        gb[k] = g.sum((0, 2, 3))
        if k:
            g = torch.nn.grad.conv2d_input(a[k].shape, torch_weight(ws[k]), g, padding=1) * (ys[k - 1] > 0)
    return a, ys, gw, gb, gy
