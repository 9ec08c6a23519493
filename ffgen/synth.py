"""Seeded synthetic image pairs with ground-truth flow and occlusion.

These pairs stand in for the optical-flow benchmarks the paper evaluates on
(MPI-Sintel-sized 1024x436 frames, KITTI-sized 1242x375 frames); no item of
those datasets is reproduced.  Nothing here computes any part of the Flow
Fields method: the module only draws textures, moves layers and records the
true displacement of every pixel of the first image.

Construction ("canvas method"):
  * one large texture canvas is drawn per pair;
  * the background and every moving layer show crops of that canvas, so
    translated content exists beyond the frame and no holes appear;
  * a layer drawn later lies above the earlier ones (depth = draw order);
  * the ground-truth flow of an img1 pixel is the translation of the top-most
    layer at that pixel; it is occluded if its target leaves the frame or is
    covered in img2 by a higher layer.

Workload presets (generator seed = 0x5EED0000 + 1000 * config + pair):
  1: 160x120, 3x3-box-blurred uniform noise, 4 rectangles, t in [-20, 20]^2,
     static background, img2 + N(0, 2).
  2: 1024x436, three-octave noise (grid spacing 1, 4, 16 px, bilinear), a
     moving background and 12 star-shaped polygons (3-8 vertices, radii
     20-200 px), t in [-150, 150]^2, img2 + N(0, 2).
  3: 1242x375, radial expansion about a random focus of expansion with
     |flow| <= 120 px (rounded to integers) and 3 translated boxes.
  4: like 2 with W in [256, 1280], H in [192, 512] and t in [-100, 100]^2.
  5: like 2 (training pairs for the learned descriptor).
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 0x5EED0000
FF_SEED = 12345


def pair_seed(config: int, pair: int = 0) -> int:
    return SEED_BASE + 1000 * config + pair


@dataclasses.dataclass
class Pair:
    img1: np.ndarray          # uint8 [H][W]
    img2: np.ndarray          # uint8 [H][W]
    flow_gt: np.ndarray       # int32 [H][W][2]  (dx, dy) of img1 pixels
    occ: np.ndarray           # bool  [H][W]     True = occluded / leaves frame

    @property
    def shape(self):
        return self.img1.shape


def _round_u8(x: np.ndarray) -> np.ndarray:
    # numpy rounds half to even
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def _box3(img: np.ndarray) -> np.ndarray:
    p = np.pad(img.astype(np.float64), 1, mode="edge")
    acc = np.zeros(img.shape, np.float64)
    for dy in range(3):
        for dx in range(3):
            acc += p[dy:dy + img.shape[0], dx:dx + img.shape[1]]
    return acc / 9.0


def _bilinear_up(grid: np.ndarray, spacing: int, H: int, W: int) -> np.ndarray:
    ys = np.arange(H) / spacing
    xs = np.arange(W) / spacing
    y0 = np.floor(ys).astype(np.int64)
    x0 = np.floor(xs).astype(np.int64)
    wy = (ys - y0)[:, None]
    wx = (xs - x0)[None, :]
    g = grid
    a = g[y0][:, x0]
    b = g[y0][:, x0 + 1]
    c = g[y0 + 1][:, x0]
    d = g[y0 + 1][:, x0 + 1]
    return (a * (1 - wx) + b * wx) * (1 - wy) + (c * (1 - wx) + d * wx) * wy


def texture_box_noise(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    return _round_u8(_box3(rng.integers(0, 256, size=(H, W)).astype(np.float64)))


def texture_octaves(rng: np.random.Generator, H: int, W: int, octaves=(1, 4, 16)) -> np.ndarray:
    acc = np.zeros((H, W), np.float64)
    for s in octaves:
        if s == 1:
            acc += rng.random((H, W))
        else:
            acc += _bilinear_up(rng.random((H // s + 2, W // s + 2)), s, H, W)
    lo, hi = acc.min(), acc.max()
    return _round_u8((acc - lo) * (255.0 / max(hi - lo, 1e-12)))


def _polygon_mask(cx, cy, verts, H, W):
    """Even-odd point-in-polygon test of every pixel centre."""
    ys, xs = np.mgrid[0:H, 0:W]
    inside = np.zeros((H, W), bool)
    n = len(verts)
    for k in range(n):
        x1, y1 = verts[k]
        x2, y2 = verts[(k + 1) % n]
        cond = (y1 > ys) != (y2 > ys)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = (x2 - x1) * (ys - y1) / (y2 - y1) + x1
        inside ^= cond & (xs < xint)
    return inside


def _random_polygon(rng, H, W, rmin=20, rmax=200):
    cx = rng.uniform(0, W)
    cy = rng.uniform(0, H)
    k = int(rng.integers(3, 9))
    ang = np.sort(rng.uniform(0, 2 * np.pi, size=k))
    rad = rng.uniform(rmin, rmax, size=k)
    verts = [(cx + r * np.cos(a), cy + r * np.sin(a)) for a, r in zip(ang, rad)]
    return _polygon_mask(cx, cy, verts, H, W)


def _compose_layers(canvas, pad, H, W, masks, trans, offs, noise_rng, noise_sigma=2.0):
    """Paint layers (index 0 = background covering everything) into both frames.

    masks[k]: bool [H][W] footprint of layer k in img1 coordinates.
    trans[k]: integer (tx, ty) displacement of layer k from img1 to img2.
    offs[k]:  integer (ox, oy) offset of layer k's texture inside the canvas.
    """
    ys, xs = np.mgrid[0:H, 0:W]
    L = len(masks)
    top1 = np.zeros((H, W), np.int32)
    for k in range(1, L):
        top1[masks[k]] = k
    top2 = np.zeros((H, W), np.int32)
    for k in range(1, L):
        tx, ty = trans[k]
        # pixel y of img2 shows layer k iff y - t lies in the layer's footprint
        sx = xs - tx
        sy = ys - ty
        ok = (sx >= 0) & (sx < W) & (sy >= 0) & (sy < H)
        hit = np.zeros((H, W), bool)
        hit[ok] = masks[k][sy[ok], sx[ok]]
        top2[hit] = k
    img1 = np.empty((H, W), np.float64)
    img2 = np.empty((H, W), np.float64)
    for k in range(L):
        ox, oy = offs[k]
        tx, ty = trans[k]
        sel1 = top1 == k
        img1[sel1] = canvas[pad + ys[sel1] + oy, pad + xs[sel1] + ox]
        sel2 = top2 == k
        img2[sel2] = canvas[pad + ys[sel2] - ty + oy, pad + xs[sel2] - tx + ox]
    img2 += noise_rng.normal(0.0, noise_sigma, size=img2.shape)
    flow = np.zeros((H, W, 2), np.int32)
    tr = np.asarray(trans, np.int32)
    flow[..., 0] = tr[top1, 0]
    flow[..., 1] = tr[top1, 1]
    tx_, ty_ = xs + flow[..., 0], ys + flow[..., 1]
    inside = (tx_ >= 0) & (tx_ < W) & (ty_ >= 0) & (ty_ < H)
    occ = ~inside
    cover = np.zeros((H, W), np.int32)
    cover[inside] = top2[ty_[inside], tx_[inside]]
    occ |= inside & (cover != top1)
    return img1.astype(np.uint8), _round_u8(img2), flow, occ


def make_layers_pair(seed: int, H: int, W: int, n_layers: int, tmax: int, kind: str,
                     bg_tmax: int = 0, texture: str = "octaves") -> Pair:
    rng = np.random.default_rng(seed)
    omax = 64
    pad = tmax + omax + 2
    ch, cw = H + 2 * pad, W + 2 * pad
    canvas = (texture_octaves(rng, ch, cw) if texture == "octaves"
              else texture_box_noise(rng, ch, cw)).astype(np.float64)
    masks = [np.ones((H, W), bool)]
    trans = [(int(rng.integers(-bg_tmax, bg_tmax + 1)), int(rng.integers(-bg_tmax, bg_tmax + 1)))
             if bg_tmax > 0 else (0, 0)]
    offs = [(0, 0)]
    for _ in range(n_layers):
        if kind == "rect":
            w = int(rng.integers(16, 61))
            h = int(rng.integers(16, 61))
            x0 = int(rng.integers(0, max(1, W - w)))
            y0 = int(rng.integers(0, max(1, H - h)))
            m = np.zeros((H, W), bool)
            m[y0:y0 + h, x0:x0 + w] = True
        else:
            m = _random_polygon(rng, H, W)
        masks.append(m)
        trans.append((int(rng.integers(-tmax, tmax + 1)), int(rng.integers(-tmax, tmax + 1))))
        offs.append((int(rng.integers(-omax, omax + 1)), int(rng.integers(-omax, omax + 1))))
    img1, img2, flow, occ = _compose_layers(canvas, pad, H, W, masks, trans, offs, rng)
    return Pair(img1, img2, flow, occ)


def make_radial_pair(seed: int, H: int, W: int, fmax: int = 120, n_boxes: int = 3,
                     box_tmax: int = 40) -> Pair:
    rng = np.random.default_rng(seed)
    pad = fmax + box_tmax + 70
    canvas = texture_octaves(rng, H + 2 * pad, W + 2 * pad).astype(np.float64)
    cx = rng.uniform(0.25 * W, 0.75 * W)
    cy = rng.uniform(0.25 * H, 0.75 * H)
    corners = np.array([[0, 0], [W - 1, 0], [0, H - 1], [W - 1, H - 1]], np.float64)
    dmax = np.max(np.hypot(corners[:, 0] - cx, corners[:, 1] - cy))
    alpha = fmax / dmax
    ys, xs = np.mgrid[0:H, 0:W]
    fx = np.rint(alpha * (xs - cx)).astype(np.int32)
    fy = np.rint(alpha * (ys - cy)).astype(np.int32)
    img1 = canvas[pad + ys, pad + xs].copy()
    # img2: forward splat of the expanding background (injective per axis for
    # alpha >= 0); unhit pixels take the canvas at the inverse-mapped position
    inv_x = np.rint(cx + (xs - cx) / (1 + alpha)).astype(np.int64)
    inv_y = np.rint(cy + (ys - cy) / (1 + alpha)).astype(np.int64)
    img2 = canvas[pad + inv_y, pad + inv_x].copy()
    tx_, ty_ = xs + fx, ys + fy
    inside = (tx_ >= 0) & (tx_ < W) & (ty_ >= 0) & (ty_ < H)
    img2[ty_[inside], tx_[inside]] = img1[inside]
    flow = np.stack([fx, fy], axis=-1)
    occ = ~inside
    # translated foreground boxes on top (depth = draw order)
    cover2 = np.full((H, W), -1, np.int32)
    top1 = np.full((H, W), -1, np.int32)
    for b in range(n_boxes):
        w = int(rng.integers(40, 161))
        h = int(rng.integers(30, 121))
        x0 = int(rng.integers(0, W - w))
        y0 = int(rng.integers(0, H - h))
        tx = int(rng.integers(-box_tmax, box_tmax + 1))
        ty = int(rng.integers(-box_tmax, box_tmax + 1))
        ox = int(rng.integers(-60, 61))
        oy = int(rng.integers(-60, 61))
        m1 = np.zeros((H, W), bool)
        m1[y0:y0 + h, x0:x0 + w] = True
        img1[m1] = canvas[pad + ys[m1] + oy, pad + xs[m1] + ox]
        top1[m1] = b
        flow[m1] = (tx, ty)
        m2 = np.zeros((H, W), bool)
        m2[max(0, y0 + ty):max(0, min(H, y0 + h + ty)), max(0, x0 + tx):max(0, min(W, x0 + w + tx))] = True
        img2[m2] = canvas[pad + ys[m2] - ty + oy, pad + xs[m2] - tx + ox]
        cover2[m2] = b
    img2 += rng.normal(0.0, 2.0, size=img2.shape)
    tx_, ty_ = xs + flow[..., 0], ys + flow[..., 1]
    inside = (tx_ >= 0) & (tx_ < W) & (ty_ >= 0) & (ty_ < H)
    occ = ~inside
    tgt_cover = np.full((H, W), -2, np.int32)
    tgt_cover[inside] = cover2[ty_[inside], tx_[inside]]
    occ |= inside & (tgt_cover != top1)
    return Pair(img1.astype(np.uint8), _round_u8(img2), flow.astype(np.int32), occ)


@dataclasses.dataclass(frozen=True)
class FFConfig:
    """Flow Fields schedule of one workload preset."""
    levels: int
    iters: int
    R_num: int = 1
    R_den: int = 1
    radius: int = 3
    eps: float = 1.0
    seed: int = FF_SEED


CONFIG_PARAMS = {
    1: FFConfig(levels=3, iters=4),
    2: FFConfig(levels=5, iters=6),
    3: FFConfig(levels=5, iters=6, R_num=3, R_den=2),
    4: FFConfig(levels=5, iters=6),
    5: FFConfig(levels=5, iters=6),
}


def batch_shapes(n_pairs: int = 64, config: int = 4):
    rng = np.random.default_rng(pair_seed(config, 999))
    Ws = rng.integers(256, 1281, size=n_pairs)
    Hs = rng.integers(192, 513, size=n_pairs)
    return [(int(h), int(w)) for h, w in zip(Hs, Ws)]


def make_pair(config: int, pair: int = 0, shape=None) -> Pair:
    """Deterministic synthetic pair of a workload preset (see module doc)."""
    seed = pair_seed(config, pair)
    if config == 1:
        H, W = shape or (120, 160)
        return make_layers_pair(seed, H, W, 4, 20, "rect", texture="box")
    if config in (2, 5):
        H, W = shape or (436, 1024)
        return make_layers_pair(seed, H, W, 12, 150, "poly", bg_tmax=30)
    if config == 3:
        H, W = shape or (375, 1242)
        return make_radial_pair(seed, H, W)
    if config == 4:
        H, W = shape or batch_shapes()[pair]
        return make_layers_pair(seed, H, W, 12, 100, "poly", bg_tmax=30)
    raise ValueError(f"unknown config {config}")


def random_images(seed: int, H: int, W: int, kind: str = "box"):
    """Small unstructured image pairs for edge-case tests (no ground truth)."""
    rng = np.random.default_rng(seed)
    if kind == "box":
        a = texture_box_noise(rng, H, W)
        b = texture_box_noise(rng, H, W)
    else:
        a = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        b = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    return a, b


def translated_crops(seed: int, H: int, W: int, tx: int, ty: int, noise: float = 0.0):
    """Two windows of one canvas offset by an integer translation (tx, ty):
    img2(x + t) == img1(x) wherever both lie inside the frame, with no
    border artefacts since the canvas extends beyond both windows."""
    rng = np.random.default_rng(seed)
    pad = abs(tx) + abs(ty) + 8
    canvas = texture_box_noise(rng, H + 2 * pad, W + 2 * pad)
    img1 = canvas[pad:pad + H, pad:pad + W].copy()
    img2 = canvas[pad - ty:pad - ty + H, pad - tx:pad - tx + W].astype(np.float64)
    if noise > 0:
        img2 += rng.normal(0, noise, size=img2.shape)
    return img1, _round_u8(img2)
