"""ctypes wrappers of the plain-C oracle (``ff_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every wrapper takes
and returns NumPy arrays in the layouts documented at the top of
``ff_oracle.c``; no GPU code is involved.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

UNSET = 0xFFFFFFFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ff_oracle.c")
_LIB = os.path.join(_HERE, "libff_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (plain -O2, OpenMP threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i, u64, dbl = C.c_int, C.c_uint64, C.c_double
        L.or_blur.argtypes = [P, i, i, i, P]
        L.or_descriptor.argtypes = [P, i, i, i, P]
        L.or_cost.argtypes = [P, P, i, i, i, i, i, i, i, i]
        L.or_cost.restype = C.c_uint32
        L.or_nn.argtypes = [P, P, i, i, i, P, P, i]
        L.or_init_coarse.argtypes = [P, P, P, i, i, i, i, P, P, P]
        L.or_nn_topl.argtypes = [P, P, i, i, i, i, P, P, i]
        L.or_init_coarse_l.argtypes = [P, i, P, P, i, i, i, i, P, P, P]
        L.or_propagate_raster.argtypes = [P, P, i, i, i, i, i, P, P, P]
        L.or_flow_fields_x.argtypes = [P, P, i, i, i, i, i, i, i, i, i, i, i, i, i, i, i, dbl, u64, i, P, P, P, P,
                                       P, P, P]
        L.or_make_stages.argtypes = [i, i, i, P, P]
        L.or_make_stages.restype = i
        L.or_rescore.argtypes = [P, P, i, i, i, i, i, P, P, P]
        L.or_seed_level_m.argtypes = [P, P, P, P, i, i, i, i, i, P, P, P]
        L.or_propagate_m.argtypes = [P, P, i, i, i, i, i, i, P, P, P, i]
        L.or_random_search_m.argtypes = [P, P, i, i, i, i, i, i, u64, i, i, i, P, P, P, i]
        L.or_nn_topl_step.argtypes = [P, P, i, i, i, i, i, P, P, i]
        L.or_consistency_grid.argtypes = [P, P, P, P, i, i, i, dbl, P]
        L.or_flow_fields_x.restype = i
        L.or_seed_level.argtypes = [P, P, P, P, i, i, i, i, P, P, P]
        L.or_propagate.argtypes = [P, P, i, i, i, i, i, P, P, P, i]
        L.or_random_search.argtypes = [P, P, i, i, i, i, i, u64, i, i, i, P, P, P, i]
        L.or_mix64.argtypes = [u64]
        L.or_mix64.restype = u64
        L.or_rs_offset.argtypes = [u64, i, i, i, i, i, i, P, P]
        L.or_rs_radius.argtypes = [i, i, i]
        L.or_rs_radius.restype = i
        L.or_consistency.argtypes = [P, P, P, P, i, i, dbl, P]
        L.or_consistency2.argtypes = [P, P, P, P, P, P, i, i, dbl, P]
        L.or_sparsify.argtypes = [P, P, P, P, i, i, i, i, P]
        L.or_region_filter.argtypes = [P, P, P, i, i, i, P]
        L.or_flow_fields.argtypes = [P, P, i, i, i, i, i, i, i, i, i, i, dbl, u64, i, P, P, P, P, P, P, P]
        L.or_flow_fields.restype = i
        L.or_flow_fields_sub.argtypes = [P, P, i, i, i, i, i, i, i, i, i, i, i, dbl, u64, i, P, P, P, P, P, P, P]
        L.or_flow_fields_sub.restype = i
        L.or_cost_sub.argtypes = [P, P, i, i, i, i, i, i, i, i, i]
        L.or_cost_sub.restype = C.c_uint32
        L.or_propagate_sub.argtypes = [P, P, i, i, i, i, i, i, P, P, P, i]
        L.or_random_search_sub.argtypes = [P, P, i, i, i, i, i, i, u64, i, i, i, P, P, P, i]
        L.or_consistency_sub.argtypes = [P, P, P, P, i, i, i, dbl, P]
        L.or_cost_f32.argtypes = [P, P, i, i, i, i, i, i, i, i]
        L.or_cost_f32.restype = C.c_uint32
        L.or_quantize_u8.argtypes = [P, C.c_int64, P]
        L.or_quantize_pair_u8.argtypes = [P, P, C.c_int64, P, P]
        L.or_flow_fields_f32.argtypes = [P, P, i, i, i, i, i, i, i, i, i, i, dbl, u64, i, P, P, P, P, P, P, P]
        L.or_flow_fields_f32.restype = i
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def cells(W: int, H: int, n: int):
    return -(-W // n), -(-H // n)


def blur(img: np.ndarray, n: int) -> np.ndarray:
    img = _u8(img)
    H, W = img.shape
    out = np.empty_like(img)
    lib().or_blur(_p(img), W, H, n, _p(out))
    return out


def descriptor(blurred: np.ndarray, n: int) -> np.ndarray:
    b = _u8(blurred)
    H, W = b.shape
    out = np.empty((H, W, 16), np.uint8)
    lib().or_descriptor(_p(b), W, H, n, _p(out))
    return out


def descriptors_all(img: np.ndarray, levels: int):
    return [descriptor(blur(img, 1 << l), 1 << l) for l in range(levels)]


def cost(Da, Db, n: int, r: int, x: int, y: int, fx: int, fy: int) -> int:
    H, W = Da.shape[:2]
    return int(lib().or_cost(_p(Da), _p(Db), W, H, n, r, x, y, fx, fy))


def nn(Da1, Db1, nc: int, nthreads: int = 1):
    H, W = Da1.shape[:2]
    Wc, Hc = cells(W, H, nc)
    idx = np.empty((Hc, Wc), np.int32)
    dist = np.empty((Hc, Wc), np.int64)
    lib().or_nn(_p(Da1), _p(Db1), W, H, nc, _p(idx), _p(dist), nthreads)
    return idx, dist


def nn_topl(Da1, Db1, nc: int, l: int, nthreads: int = 1, rstep: int = 1):
    """The l nearest pixels of every coarsest-grid cell, ranked by (distance,
    index): idx [Hc][Wc][l] (-1 past the image's pixel count), dist alike;
    rstep = 2: among the pixels with even x and y only."""
    H, W = Da1.shape[:2]
    Wc, Hc = cells(W, H, nc)
    idx = np.empty((Hc, Wc, l), np.int32)
    dist = np.empty((Hc, Wc, l), np.int64)
    lib().or_nn_topl_step(_p(Da1), _p(Db1), W, H, nc, l, rstep, _p(idx), _p(dist), nthreads)
    return idx, dist


def init_coarse_l(cand, Da, Db, nc: int, r: int = 3):
    """Seeds from l ranked candidates per cell (cand [Hc][Wc][l]): the lowest
    E_nc, the earlier rank on equal cost; returns (flow, cost, n_evals)."""
    H, W = Da.shape[:2]
    Wc, Hc = cells(W, H, nc)
    cand = np.ascontiguousarray(cand, np.int32)
    l = cand.shape[-1]
    flow = np.empty((Hc, Wc, 2), np.int16)
    cost_ = np.empty((Hc, Wc), np.uint32)
    ne = np.zeros(1, np.uint64)
    lib().or_init_coarse_l(_p(cand), l, _p(Da), _p(Db), W, H, nc, r, _p(flow), _p(cost_), _p(ne))
    return flow, cost_, int(ne[0])


def init_coarse(idx, Da, Db, nc: int, r: int = 3):
    H, W = Da.shape[:2]
    Wc, Hc = cells(W, H, nc)
    flow = np.empty((Hc, Wc, 2), np.int16)
    cost_ = np.empty((Hc, Wc), np.uint32)
    ne = np.zeros(1, np.uint64)
    idx = np.ascontiguousarray(idx, np.int32)
    lib().or_init_coarse(_p(idx), _p(Da), _p(Db), W, H, nc, r, _p(flow), _p(cost_), _p(ne))
    return flow, cost_, int(ne[0])


def seed_level(cflow, ccost, Da, Db, n: int, r: int = 3):
    H, W = Da.shape[:2]
    Wn, Hn = cells(W, H, n)
    flow = np.empty((Hn, Wn, 2), np.int16)
    cost_ = np.empty((Hn, Wn), np.uint32)
    ne = np.zeros(1, np.uint64)
    cflow = np.ascontiguousarray(cflow, np.int16)
    ccost = np.ascontiguousarray(ccost, np.uint32)
    lib().or_seed_level(_p(cflow), _p(ccost), _p(Da), _p(Db), W, H, n, r, _p(flow), _p(cost_), _p(ne))
    return flow, cost_, int(ne[0])


def propagate(Da, Db, n: int, pass_: int, flow, cost_, r: int = 3, nthreads: int = 1):
    """In-place propagation step on copies; returns (flow, cost, n_evals)."""
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_propagate(_p(Da), _p(Db), W, H, n, r, pass_, _p(flow), _p(cost_), _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def propagate_raster(Da, Db, n: int, pass_: int, flow, cost_, r: int = 3):
    """Serial-order propagation step on copies; returns (flow, cost, n_evals)."""
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_propagate_raster(_p(Da), _p(Db), W, H, n, r, pass_, _p(flow), _p(cost_), _p(ne))
    return flow, cost_, int(ne[0])


def stages(levels: int, fast_x2: bool = False, subscales: bool = False):
    """(grid scale n, patch scale m) of every stage of the schedule, coarse
    to fine."""
    n = np.zeros(16, np.int32)
    m = np.zeros(16, np.int32)
    k = lib().or_make_stages(levels, int(bool(fast_x2)), int(bool(subscales)), _p(n), _p(m))
    return [(int(a), int(b)) for a, b in zip(n[:k], m[:k])]


def rescore(Da, Db, n: int, m: int, flow, cost_, r: int = 3):
    """Same grid, new patch scale: every set cell's cost at patch scale m;
    returns (cost, n_evals)."""
    H, W = Da.shape[:2]
    flow = np.ascontiguousarray(flow, np.int16)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_rescore(_p(Da), _p(Db), W, H, n, m, r, _p(flow), _p(cost_), _p(ne))
    return cost_, int(ne[0])


def seed_level_m(cflow, ccost, Da, Db, n: int, m: int, r: int = 3):
    """Hand-over to the grid of scale n with costs at patch scale m."""
    H, W = Da.shape[:2]
    Wn, Hn = cells(W, H, n)
    flow = np.empty((Hn, Wn, 2), np.int16)
    cost_ = np.empty((Hn, Wn), np.uint32)
    ne = np.zeros(1, np.uint64)
    cflow = np.ascontiguousarray(cflow, np.int16)
    ccost = np.ascontiguousarray(ccost, np.uint32)
    lib().or_seed_level_m(_p(cflow), _p(ccost), _p(Da), _p(Db), W, H, n, m, r, _p(flow), _p(cost_), _p(ne))
    return flow, cost_, int(ne[0])


def propagate_m(Da, Db, n: int, m: int, pass_: int, flow, cost_, r: int = 3, nthreads: int = 1):
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_propagate_m(_p(Da), _p(Db), W, H, n, m, r, pass_, _p(flow), _p(cost_), _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def random_search_m(Da, Db, n: int, m: int, Rn: int, seed: int, stream: int, gen: int, pass_: int, flow, cost_,
                    r: int = 3, nthreads: int = 1):
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_random_search_m(_p(Da), _p(Db), W, H, n, m, r, Rn, seed, stream, gen, pass_, _p(flow), _p(cost_),
                             _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def rs_radius(n: int, R_num: int, R_den: int) -> int:
    return int(lib().or_rs_radius(n, R_num, R_den))


def random_search(Da, Db, n: int, Rn: int, seed: int, stream: int, level: int, pass_: int, flow, cost_,
                  r: int = 3, nthreads: int = 1):
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_random_search(_p(Da), _p(Db), W, H, n, r, Rn, seed, stream, level, pass_, _p(flow), _p(cost_),
                           _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def mix64(z: int) -> int:
    return int(lib().or_mix64(z))


def rs_offset(seed: int, stream: int, level: int, pass_: int, j: int, i: int, Rn: int):
    ox, oy = C.c_int(), C.c_int()
    lib().or_rs_offset(seed, stream, level, pass_, j, i, Rn, C.byref(ox), C.byref(oy))
    return ox.value, oy.value


def consistency(fa, ca, fb, cb, eps: float = 1.0):
    H, W = ca.shape
    keep = np.empty((H, W), np.uint8)
    args = [np.ascontiguousarray(a) for a in (fa, ca, fb, cb)]
    lib().or_consistency(*[_p(a) for a in args], W, H, float(eps), _p(keep))
    return keep


def consistency_grid(fa, ca, fb, cb, W: int, H: int, n: int, eps: float = 1.0):
    """Keep mask of a field on the grid of scale n (one match per n x n
    region) against the backward field on the same grid."""
    Wn, Hn = cells(W, H, n)
    keep = np.empty((Hn, Wn), np.uint8)
    args = [np.ascontiguousarray(a) for a in (fa, ca, fb, cb)]
    lib().or_consistency_grid(*[_p(a) for a in args], W, H, n, float(eps), _p(keep))
    return keep


def consistency2(fa, ca, fb1, cb1, fb2, cb2, eps: float = 1.0):
    """Keep mask of field a against two backward fields (Sec. 3.7)."""
    H, W = ca.shape
    keep = np.empty((H, W), np.uint8)
    args = [np.ascontiguousarray(a) for a in (fa, ca, fb1, cb1, fb2, cb2)]
    lib().or_consistency2(*[_p(a) for a in args], W, H, float(eps), _p(keep))
    return keep


def region_filter(flow, cost, keep, s: int) -> np.ndarray:
    """Keep mask without the small regions next to removed outliers (Sec. 3.7)."""
    H, W = keep.shape
    out = np.empty((H, W), np.uint8)
    flow = np.ascontiguousarray(flow, np.int16)
    cost = np.ascontiguousarray(cost, np.uint32)
    keep = np.ascontiguousarray(keep, np.uint8)
    lib().or_region_filter(_p(flow), _p(cost), _p(keep), W, H, s, _p(out))
    return out


def sparsify(fa, keep, fb1, fb2=None, q: int = 3, e: int = 1) -> np.ndarray:
    """Selected pixel index (y * W + x, or -1) of every q x q region (Sec. 3.8)."""
    H, W = keep.shape
    sel = np.empty((-(-H // q), -(-W // q)), np.int32)
    fa = np.ascontiguousarray(fa, np.int16)
    keep = np.ascontiguousarray(keep, np.uint8)
    fb1 = np.ascontiguousarray(fb1, np.int16)
    fb2 = None if fb2 is None else np.ascontiguousarray(fb2, np.int16)
    lib().or_sparsify(_p(fa), _p(keep), _p(fb1), None if fb2 is None else _p(fb2), W, H, q, e, _p(sel))
    return sel


def flow_fields(img1, img2, levels: int, iters: int, radius: int = 3, R_num: int = 1, R_den: int = 1,
                eps: float = 1.0, seed: int = 12345, nthreads: int = 1, plus_iters: int = 0, Rp_num: int = 0,
                fine_iters: int = 0, subpixel: int = 0, nn_l: int = 1, raster: bool = False,
                fast_x2: bool = False, subscales: bool = False) -> dict:
    """The whole schedule on one pair.  plus_iters > 0: Flow Fields+ (P steps
    at R^+ = Rp_num / R_den before the `iters` steps at R); fine_iters > 0:
    the finest scale runs only that many steps at R (Flow Fields+ Fast);
    subpixel = s > 0: flows in units of 1/2^s pixel, bilinear targets, costs
    of cost_sub (scaled by 4^s); nn_l > 1: seeds reranked among the nn_l
    nearest pixels (Eq. 4); raster: serial-order propagation steps; fast_x2:
    Flow Fields+ Fast x2 (finest scale skipped, seeds among the even pixels,
    fields and masks on the grid of scale 2, fine_iters steps there);
    subscales: the sub-scale stages of Sec. 3.3 (see stages())."""
    img1, img2 = _u8(img1), _u8(img2)
    H, W = img1.shape
    Ho, Wo = (-(-H // 2), -(-W // 2)) if fast_x2 else (H, W)
    out = {
        "flow_fwd": np.empty((Ho, Wo, 2), np.int16), "flow_bwd": np.empty((Ho, Wo, 2), np.int16),
        "cost_fwd": np.empty((Ho, Wo), np.uint32), "cost_bwd": np.empty((Ho, Wo), np.uint32),
        "keep_fwd": np.empty((Ho, Wo), np.uint8), "keep_bwd": np.empty((Ho, Wo), np.uint8),
    }
    ne = np.zeros(2, np.uint64)
    if nn_l != 1 or raster or fast_x2 or subscales:
        rc = lib().or_flow_fields_x(_p(img1), _p(img2), W, H, levels, iters, radius, R_num, R_den, plus_iters,
                                    Rp_num, fine_iters, subpixel, nn_l, int(bool(raster)), int(bool(fast_x2)),
                                    int(bool(subscales)), float(eps), seed, nthreads,
                                    _p(out["flow_fwd"]), _p(out["flow_bwd"]), _p(out["cost_fwd"]),
                                    _p(out["cost_bwd"]), _p(out["keep_fwd"]), _p(out["keep_bwd"]), _p(ne))
    elif subpixel:
        rc = lib().or_flow_fields_sub(_p(img1), _p(img2), W, H, levels, iters, radius, R_num, R_den, plus_iters,
                                      Rp_num, fine_iters, subpixel, float(eps), seed, nthreads, _p(out["flow_fwd"]),
                                      _p(out["flow_bwd"]), _p(out["cost_fwd"]), _p(out["cost_bwd"]),
                                      _p(out["keep_fwd"]), _p(out["keep_bwd"]), _p(ne))
    else:
        rc = lib().or_flow_fields(_p(img1), _p(img2), W, H, levels, iters, radius, R_num, R_den, plus_iters, Rp_num,
                                  fine_iters, float(eps), seed, nthreads, _p(out["flow_fwd"]), _p(out["flow_bwd"]),
                                  _p(out["cost_fwd"]), _p(out["cost_bwd"]), _p(out["keep_fwd"]), _p(out["keep_bwd"]),
                                  _p(ne))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out["n_evals"] = (int(ne[0]), int(ne[1]))
    return out


def cost_sub(Da, Db, n: int, r: int, x: int, y: int, fx: int, fy: int, s: int) -> int:
    """Subpixel matching error (flow in units of 1/2^s pixel), scaled by 4^s."""
    H, W = Da.shape[:2]
    return int(lib().or_cost_sub(_p(Da), _p(Db), W, H, n, r, x, y, fx, fy, s))


def propagate_sub(Da, Db, n: int, s: int, pass_: int, flow, cost_, r: int = 3, nthreads: int = 1):
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_propagate_sub(_p(Da), _p(Db), W, H, n, r, s, pass_, _p(flow), _p(cost_), _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def random_search_sub(Da, Db, n: int, s: int, Rn: int, seed: int, stream: int, level: int, pass_: int, flow, cost_,
                      r: int = 3, nthreads: int = 1):
    H, W = Da.shape[:2]
    flow = np.array(flow, np.int16, order="C", copy=True)
    cost_ = np.array(cost_, np.uint32, order="C", copy=True)
    ne = np.zeros(1, np.uint64)
    lib().or_random_search_sub(_p(Da), _p(Db), W, H, n, r, s, Rn, seed, stream, level, pass_, _p(flow), _p(cost_),
                               _p(ne), nthreads)
    return flow, cost_, int(ne[0])


def consistency_sub(fa, ca, fb, cb, s: int, eps: float = 1.0):
    H, W = ca.shape
    keep = np.empty((H, W), np.uint8)
    args = [np.ascontiguousarray(a) for a in (fa, ca, fb, cb)]
    lib().or_consistency_sub(*[_p(a) for a in args], W, H, s, float(eps), _p(keep))
    return keep


def cost_f32(Fa, Fb, n: int, r: int, x: int, y: int, fx: int, fy: int) -> float:
    """Single-precision learned-feature cost: four channel-group partial sums
    (fused multiply-adds, order v, u, c), added as (s0 + s1) + (s2 + s3)."""
    Fa = np.ascontiguousarray(Fa, np.float32)
    Fb = np.ascontiguousarray(Fb, np.float32)
    H, W = Fa.shape[:2]
    bits = lib().or_cost_f32(_p(Fa), _p(Fb), W, H, n, r, x, y, fx, fy)
    return float(np.array([bits], np.uint32).view(np.float32)[0])


def quantize_u8(f) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float32)
    q = np.empty(f.shape, np.uint8)
    lib().or_quantize_u8(_p(f), f.size, _p(q))
    return q


def quantize_pair_u8(f1, f2):
    """Both maps quantised to bytes with the range of their union."""
    f1 = np.ascontiguousarray(f1, np.float32)
    f2 = np.ascontiguousarray(f2, np.float32)
    assert f1.shape == f2.shape
    q1, q2 = np.empty(f1.shape, np.uint8), np.empty(f2.shape, np.uint8)
    lib().or_quantize_pair_u8(_p(f1), _p(f2), f1.size, _p(q1), _p(q2))
    return q1, q2


def flow_fields_f32(F1, F2, levels: int, iters: int, radius: int = 3, R_num: int = 1, R_den: int = 1,
                    eps: float = 1.0, seed: int = 12345, nthreads: int = 1, plus_iters: int = 0, Rp_num: int = 0,
                    fine_iters: int = 0) -> dict:
    """The multi-scale schedule on learned float features F1[l], F2[l]
    (float32 [H][W][16] per scale 2^l); costs come back as float32."""
    F1 = [np.ascontiguousarray(f, np.float32) for f in F1]
    F2 = [np.ascontiguousarray(f, np.float32) for f in F2]
    H, W = F1[0].shape[:2]
    arr1 = (C.c_void_p * levels)(*[f.ctypes.data for f in F1])
    arr2 = (C.c_void_p * levels)(*[f.ctypes.data for f in F2])
    out = {
        "flow_fwd": np.empty((H, W, 2), np.int16), "flow_bwd": np.empty((H, W, 2), np.int16),
        "cost_fwd": np.empty((H, W), np.uint32), "cost_bwd": np.empty((H, W), np.uint32),
        "keep_fwd": np.empty((H, W), np.uint8), "keep_bwd": np.empty((H, W), np.uint8),
    }
    ne = np.zeros(2, np.uint64)
    rc = lib().or_flow_fields_f32(C.cast(arr1, C.c_void_p), C.cast(arr2, C.c_void_p), W, H, levels, iters, radius,
                                  R_num, R_den, plus_iters, Rp_num, fine_iters, float(eps), seed, nthreads, _p(out["flow_fwd"]), _p(out["flow_bwd"]),
                                  _p(out["cost_fwd"]), _p(out["cost_bwd"]), _p(out["keep_fwd"]), _p(out["keep_bwd"]),
                                  _p(ne))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out["n_evals"] = (int(ne[0]), int(ne[1]))
    return out
