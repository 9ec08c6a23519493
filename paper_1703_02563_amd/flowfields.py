"""Python entry points of the Flow Fields hot path (same names as the C ABI).

Tensors are CUDA tensors (device memory); PyTorch provides allocation and the
current stream, the library does the work.  Layouts follow
include/flowfields.h: images uint8 [H, W]; descriptors uint8 [H, W, 16];
level grids of scale n have ceil(H/n) x ceil(W/n) cells with flows int16
[Hn, Wn, 2] = (dx, dy) and costs stored as int32 [Hn, Wn] holding the
uint32 bit pattern (0xFFFFFFFF, i.e. -1, marks an UNSET cell).
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import ffi
from .ffi import FFParams, FFTuning, check, lib

UNSET_I32 = -1  # 0xFFFFFFFF viewed as int32


@dataclasses.dataclass
class Tuning:
    """Launch tables of the level kernels per scale log2 n = 0..6 (see
    ff_tuning): speed only, results never depend on them."""
    variant: list
    passes: list
    variant_f32: list
    passes_f32: list

    def to_c(self) -> FFTuning:
        t = FFTuning()
        for name in ("variant", "passes", "variant_f32", "passes_f32"):
            vals = [int(v) for v in getattr(self, name)]
            if len(vals) != 7:
                raise ValueError(f"Tuning.{name}: 7 entries (log2 n = 0..6)")
            getattr(t, name)[:] = vals
        return t

    def replace(self, **kw) -> "Tuning":
        return dataclasses.replace(self, **{k: list(v) for k, v in kw.items()})


def default_tuning() -> Tuning:
    """The library's built-in launch tables (ff_default_tuning)."""
    t = FFTuning()
    lib().ff_default_tuning(ctypes.byref(t))
    return Tuning(list(t.variant), list(t.passes), list(t.variant_f32), list(t.passes_f32))


@dataclasses.dataclass
class Params:
    """Schedule of one Flow Field computation (see ff_params)."""
    levels: int = 5
    iters: int = 6
    radius: int = 3
    R_num: int = 1
    R_den: int = 1
    eps: float = 1.0
    seed: int = 12345
    plus_iters: int = 0  # Flow Fields+: steps at R+ = Rp_num / R_den before the `iters` steps at R
    Rp_num: int = 0
    fine_iters: int = 0  # Flow Fields+ Fast: steps at R on the finest scale (0: as the other scales)
    subpixel: int = 0  # 3: flows, random-search offsets and the threshold in 1/8 px, bilinear targets
    tuning: Tuning | None = None  # launch tables of the calls (None: the built-in tables)
    nn_l: int = 1  # seed candidates: the nn_l nearest pixels, reranked by patch cost (Eq. 1 / Eq. 4)
    raster: bool = False  # propagation steps in serial order (anti-diagonal wavefronts)
    fast_x2: bool = False  # Flow Fields+ Fast x2: no finest scale, outputs on the grid of scale 2
    subscales: bool = False  # Flow Fields+ sub-scales: a stage of patch scale 3n/2 before scale n

    def to_c(self) -> FFParams:
        p = FFParams(self.levels, self.iters, self.radius, self.R_num, self.R_den, self.eps, self.seed,
                     self.plus_iters, self.Rp_num, self.fine_iters, self.subpixel, None, self.nn_l,
                     int(bool(self.raster)), int(bool(self.fast_x2)), int(bool(self.subscales)))
        if self.tuning is not None:
            p._tuning = self.tuning.to_c()  # kept alive with the struct that points at it
            p.tuning = ctypes.pointer(p._tuning)
        return p


def _stream():
    return C_void(torch.cuda.current_stream().cuda_stream)


def C_void(v):
    import ctypes
    return ctypes.c_void_p(v)


def _ptr(t: torch.Tensor | None, dtype=None, what: str = "tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return C_void(t.data_ptr())


def cells(W: int, H: int, n: int):
    return -(-W // n), -(-H // n)


def descriptors(img: torch.Tensor, n: int, rowmajor: bool = False, wform: bool = False):
    """Scale-space image and the descriptor map of scale n: uint8
    [H + 8n, W + 8n, 16], a replicated border of 4n pixels, the pixels of a
    row in phase order (x mod n, then x // n); the layout every entry point
    taking a descriptor map expects (see ff_descriptors).  rowmajor=True also
    returns the plain [H, W, 16] descriptors (the NN seed's input);
    wform=True also returns the weight-class row map uint8 [H + 6n, W, 16]
    (ff_wform_map_bytes).  Returns (blurred, desc[, plain][, wform])."""
    H, W = img.shape
    P = 4 * n
    hsum = torch.empty((H, W), dtype=torch.int16, device=img.device)
    blurred = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    desc = torch.empty((H + 2 * P, W + 2 * P, 16), dtype=torch.uint8, device=img.device)
    plain = torch.empty((H, W, 16), dtype=torch.uint8, device=img.device) if rowmajor else None
    wf = torch.empty((H + 6 * n, W, 16), dtype=torch.uint8, device=img.device) if wform else None  # 3n border rows
    assert desc.numel() == int(lib().ff_descriptor_map_bytes(W, H, n))
    assert wf is None or wf.numel() == int(lib().ff_wform_map_bytes(W, H, n))
    check(lib().ff_descriptors(_ptr(img, torch.uint8, "img"), W, H, n, _ptr(hsum), _ptr(blurred), _ptr(desc),
                               _ptr(plain), _ptr(wf), _stream()), "ff_descriptors")
    out = (blurred, desc)
    if rowmajor:
        out += (plain,)
    if wform:
        out += (wf,)
    return out


def _map_dims(desc_a, desc_b, n: int):
    """(W, H) of the image behind two descriptor maps of scale n."""
    Hp, Wp = desc_a.shape[:2]
    W, H = Wp - 8 * n, Hp - 8 * n
    if W < 1 or H < 1 or tuple(desc_b.shape) != tuple(desc_a.shape) or desc_a.shape[2:] != (16,):
        raise ValueError("descriptor maps must both be uint8 [H + 8n, W + 8n, 16]")
    return W, H


def init_nn(desc_a1, desc_b1, desc_ac, desc_bc, nc: int, radius: int = 3, n_evals: torch.Tensor | None = None):
    """Exact NN seed of the coarsest grid; returns (flow, cost, nn_key)."""
    H, W = desc_a1.shape[:2]
    Wc, Hc = cells(W, H, nc)
    dev = desc_a1.device
    nb = torch.empty(((W * H + 31) // 32) * 32, dtype=torch.int32, device=dev)
    key = torch.empty((Hc, Wc), dtype=torch.int64, device=dev)
    flow = torch.empty((Hc, Wc, 2), dtype=torch.int16, device=dev)
    cost = torch.empty((Hc, Wc), dtype=torch.int32, device=dev)
    if _map_dims(desc_ac, desc_bc, nc) != (W, H) or tuple(desc_b1.shape) != (H, W, 16):
        raise ValueError("init_nn: level-1 descriptors [H, W, 16] and scale-nc maps of the same image size")
    check(lib().ff_init_nn(_ptr(desc_a1, torch.uint8), _ptr(desc_b1, torch.uint8), _ptr(desc_ac, torch.uint8),
                           _ptr(desc_bc, torch.uint8), W, H, nc, radius, _ptr(nb), _ptr(key), _ptr(flow),
                           _ptr(cost), _ptr(n_evals, torch.int64), _stream()), "ff_init_nn")
    return flow, cost, key


def nn_topl(desc_a1, desc_b1, nc: int, l: int):
    """The l nearest pixels of every coarsest-grid cell (ff_nn_topl): int64
    [Hc, Wc, l] entries (squared distance << 32) | q, ranked; -1 past the
    image's pixel count."""
    H, W = desc_a1.shape[:2]
    Wc, Hc = cells(W, H, nc)
    dev = desc_a1.device
    if tuple(desc_b1.shape) != (H, W, 16):
        raise ValueError("nn_topl: level-1 descriptors [H, W, 16] of two images of one size")
    nb = torch.empty(((W * H + 31) // 32) * 32, dtype=torch.int32, device=dev)
    nbytes = int(lib().ff_nn_topl_scratch_bytes(W, H, nc))
    scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    cand = torch.empty((Hc, Wc, l), dtype=torch.int64, device=dev)
    check(lib().ff_nn_topl(_ptr(desc_a1, torch.uint8), _ptr(desc_b1, torch.uint8), W, H, nc, l, _ptr(nb),
                           _ptr(scratch), nbytes, _ptr(cand), _stream()), "ff_nn_topl")
    return cand


def init_nn_l(desc_a1, desc_b1, desc_ac, desc_bc, nc: int, nn_l: int, radius: int = 3,
              n_evals: torch.Tensor | None = None):
    """Seed of the coarsest grid from the nn_l nearest pixels (ff_init_nn_l);
    returns (flow, cost, nn_key)."""
    H, W = desc_a1.shape[:2]
    Wc, Hc = cells(W, H, nc)
    dev = desc_a1.device
    if _map_dims(desc_ac, desc_bc, nc) != (W, H) or tuple(desc_b1.shape) != (H, W, 16):
        raise ValueError("init_nn_l: level-1 descriptors [H, W, 16] and scale-nc maps of the same image size")
    nb = torch.empty(((W * H + 31) // 32) * 32, dtype=torch.int32, device=dev)
    nbytes = int(lib().ff_nn_topl_scratch_bytes(W, H, nc))
    scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    key = torch.empty((Hc, Wc), dtype=torch.int64, device=dev)
    flow = torch.empty((Hc, Wc, 2), dtype=torch.int16, device=dev)
    cost = torch.empty((Hc, Wc), dtype=torch.int32, device=dev)
    check(lib().ff_init_nn_l(_ptr(desc_a1, torch.uint8), _ptr(desc_b1, torch.uint8), _ptr(desc_ac, torch.uint8),
                             _ptr(desc_bc, torch.uint8), W, H, nc, radius, nn_l, _ptr(nb), _ptr(scratch), nbytes,
                             _ptr(key), _ptr(flow), _ptr(cost), _ptr(n_evals, torch.int64), _stream()),
          "ff_init_nn_l")
    return flow, cost, key


def seed_level(cflow, ccost, desc_a, desc_b, n: int, radius: int = 3, n_evals=None):
    W, H = _map_dims(desc_a, desc_b, n)
    Wn, Hn = cells(W, H, n)
    flow = torch.empty((Hn, Wn, 2), dtype=torch.int16, device=desc_a.device)
    cost = torch.empty((Hn, Wn), dtype=torch.int32, device=desc_a.device)
    check(lib().ff_seed_level(_ptr(cflow, torch.int16), _ptr(ccost, torch.int32), _ptr(desc_a, torch.uint8),
                              _ptr(desc_b, torch.uint8), W, H, n, radius, _ptr(flow), _ptr(cost),
                              _ptr(n_evals, torch.int64), _stream()), "ff_seed_level")
    return flow, cost


def propagate_level(desc_a, desc_b, n: int, pass_: int, flow, cost, radius: int = 3, n_evals=None):
    """One propagation step, in place on (flow, cost)."""
    W, H = _map_dims(desc_a, desc_b, n)
    check(lib().ff_propagate_level(_ptr(desc_a, torch.uint8), _ptr(desc_b, torch.uint8), W, H, n, radius, pass_,
                                   _ptr(flow, torch.int16), _ptr(cost, torch.int32), _ptr(n_evals, torch.int64),
                                   _stream()), "ff_propagate_level")


def rescore_level(desc_m_a, desc_m_b, W: int, H: int, n: int, m: int, flow, cost, radius: int = 3, n_evals=None):
    """Costs of the grid of scale n moved to patch scale m (in place on cost);
    desc_m_a/desc_m_b: descriptor maps of scale m."""
    check(lib().ff_rescore_level(_ptr(desc_m_a, torch.uint8), _ptr(desc_m_b, torch.uint8), W, H, n, m, radius,
                                 _ptr(flow, torch.int16), _ptr(cost, torch.int32), _ptr(n_evals, torch.int64),
                                 _stream()), "ff_rescore_level")


def propagate_raster(desc_a, desc_b, n: int, pass_: int, flow, cost, radius: int = 3, n_evals=None):
    """One propagation step in serial order, in place on (flow, cost)."""
    W, H = _map_dims(desc_a, desc_b, n)
    check(lib().ff_propagate_raster(_ptr(desc_a, torch.uint8), _ptr(desc_b, torch.uint8), W, H, n, radius, pass_,
                                    _ptr(flow, torch.int16), _ptr(cost, torch.int32), _ptr(n_evals, torch.int64),
                                    _stream()), "ff_propagate_raster")


def random_search(desc_a, desc_b, n: int, Rn: int, seed: int, stream_id: int, level: int, pass_: int, flow, cost,
                  radius: int = 3, n_evals=None):
    """One random-search step, in place on (flow, cost)."""
    W, H = _map_dims(desc_a, desc_b, n)
    check(lib().ff_random_search(_ptr(desc_a, torch.uint8), _ptr(desc_b, torch.uint8), W, H, n, radius, Rn, seed,
                                 stream_id, level, pass_, _ptr(flow, torch.int16), _ptr(cost, torch.int32),
                                 _ptr(n_evals, torch.int64), _stream()), "ff_random_search")


def run_level(desc_a, desc_b, level: int, params: Params, stream_id: int, mode: int, flow, cost, nn_key=None,
              coarse_flow=None, coarse_cost=None, n_evals=None, n_work=None, scratch=None, wform_a=None, wform_b=None):
    """All steps of one scale, in place on (flow, cost); see ff_run_level.
    n_work: optional int64 [2] device counters of the evaluations computed
    (owned cells, all cells); scratch: optional reusable second grid;
    wform_a/wform_b: the weight-class row maps of scale 2^level (both or
    neither)."""
    W, H = _map_dims(desc_a, desc_b, 1 << level)
    if (wform_a is None) != (wform_b is None):
        raise ValueError("run_level: both weight-class maps or neither")
    nbytes = int(lib().ff_run_level_scratch_bytes(W, H, level))
    if scratch is None:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=desc_a.device)
    elif scratch.numel() * scratch.element_size() < nbytes:
        raise ValueError("run_level: scratch too small")
    check(lib().ff_run_level(_ptr(desc_a, torch.uint8), _ptr(desc_b, torch.uint8), _ptr(wform_a, torch.uint8),
                             _ptr(wform_b, torch.uint8), W, H, level, params.to_c(),
                             stream_id, mode, _ptr(nn_key, torch.int64), _ptr(coarse_flow, torch.int16),
                             _ptr(coarse_cost, torch.int32), _ptr(flow, torch.int16), _ptr(cost, torch.int32),
                             _ptr(scratch), nbytes, _ptr(n_evals, torch.int64), _ptr(n_work, torch.int64),
                             _stream()), "ff_run_level")


def run_level_pair(desc_a, desc_b, level: int, params: Params, mode: int, flows, costs, nn_keys=None,
                   coarse_flows=None, coarse_costs=None, n_evals=None, n_work=None, scratch=None, wform_a=None,
                   wform_b=None):
    """One scale of both directions in one set of launches (see
    ff_run_level_pair): flows/costs (and nn_keys, coarse_flows,
    coarse_costs where the mode reads them) are pairs of tensors, direction
    0 then 1; n_evals: optional int64 [2] per direction; n_work: optional
    int64 [2] summed over both directions."""
    W, H = _map_dims(desc_a, desc_b, 1 << level)
    if (wform_a is None) != (wform_b is None):
        raise ValueError("run_level_pair: both weight-class maps or neither")
    nbytes = 2 * int(lib().ff_run_level_scratch_bytes(W, H, level))
    if scratch is None:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=desc_a.device)
    elif scratch.numel() * scratch.element_size() < nbytes:
        raise ValueError("run_level_pair: scratch too small")

    def pair(ts, dtype):
        if ts is None:
            return None
        if len(ts) != 2:
            raise ValueError("run_level_pair: two tensors per argument, one per direction")
        return (ctypes.c_void_p * 2)(_ptr(ts[0], dtype).value, _ptr(ts[1], dtype).value)

    check(lib().ff_run_level_pair(_ptr(desc_a, torch.uint8), _ptr(desc_b, torch.uint8), _ptr(wform_a, torch.uint8),
                                  _ptr(wform_b, torch.uint8), W, H, level, params.to_c(), mode,
                                  pair(nn_keys, torch.int64), pair(coarse_flows, torch.int16),
                                  pair(coarse_costs, torch.int32), pair(flows, torch.int16), pair(costs, torch.int32),
                                  _ptr(scratch), nbytes, _ptr(n_evals, torch.int64), _ptr(n_work, torch.int64),
                                  _stream()), "ff_run_level_pair")


def level_launches(params: Params, level: int, cost_kind: int = 0) -> int:
    """Blocked launches the call's tables give one scale (ff_level_launches)."""
    t = params.tuning.to_c() if params.tuning is not None else None
    return int(lib().ff_level_launches(ctypes.byref(t) if t is not None else None, params.iters, level, cost_kind))


def consistency_filter(flow_a, cost_a, flow_b, cost_b, eps: float = 1.0, both: bool = True):
    H, W = cost_a.shape
    keep_a = torch.empty((H, W), dtype=torch.uint8, device=cost_a.device)
    keep_b = torch.empty((H, W), dtype=torch.uint8, device=cost_a.device) if both else None
    check(lib().ff_consistency_filter(_ptr(flow_a, torch.int16), _ptr(cost_a, torch.int32), _ptr(flow_b, torch.int16),
                                      _ptr(cost_b, torch.int32), W, H, eps, _ptr(keep_a), _ptr(keep_b), _stream()),
          "ff_consistency_filter")
    return keep_a, keep_b


def consistency_filter_grid(flow_a, cost_a, flow_b, cost_b, W: int, H: int, n: int, eps: float = 1.0,
                            both: bool = True):
    """Consistency of fields on the grid of scale n (one match per n x n
    region) of a W x H image."""
    Hn, Wn = cost_a.shape
    keep_a = torch.empty((Hn, Wn), dtype=torch.uint8, device=cost_a.device)
    keep_b = torch.empty((Hn, Wn), dtype=torch.uint8, device=cost_a.device) if both else None
    check(lib().ff_consistency_filter_grid(_ptr(flow_a, torch.int16), _ptr(cost_a, torch.int32),
                                           _ptr(flow_b, torch.int16), _ptr(cost_b, torch.int32), W, H, n, eps,
                                           _ptr(keep_a), _ptr(keep_b), _stream()), "ff_consistency_filter_grid")
    return keep_a, keep_b


def consistency_filter_sub(flow_a, cost_a, flow_b, cost_b, subpixel: int, eps: float = 1.0, both: bool = True):
    """Consistency of fields with flows in units of 1/2^subpixel pixel."""
    H, W = cost_a.shape
    keep_a = torch.empty((H, W), dtype=torch.uint8, device=cost_a.device)
    keep_b = torch.empty((H, W), dtype=torch.uint8, device=cost_a.device) if both else None
    check(lib().ff_consistency_filter_sub(_ptr(flow_a, torch.int16), _ptr(cost_a, torch.int32),
                                          _ptr(flow_b, torch.int16), _ptr(cost_b, torch.int32), W, H, subpixel, eps,
                                          _ptr(keep_a), _ptr(keep_b), _stream()), "ff_consistency_filter_sub")
    return keep_a, keep_b


def consistency_filter2(flow_a, cost_a, flow_b1, cost_b1, flow_b2, cost_b2, eps: float = 1.0):
    """Keep mask of field a against two backward fields (Sec. 3.7)."""
    H, W = cost_a.shape
    for t in (cost_b1, cost_b2):
        if tuple(t.shape) != (H, W):
            raise ValueError("consistency_filter2: the three fields must have the same size")
    keep = torch.empty((H, W), dtype=torch.uint8, device=cost_a.device)
    check(lib().ff_consistency_filter2(_ptr(flow_a, torch.int16), _ptr(cost_a, torch.int32),
                                       _ptr(flow_b1, torch.int16), _ptr(cost_b1, torch.int32),
                                       _ptr(flow_b2, torch.int16), _ptr(cost_b2, torch.int32), W, H, eps, _ptr(keep),
                                       _stream()), "ff_consistency_filter2")
    return keep


def region_filter(flow, cost, keep, s: int) -> torch.Tensor:
    """Keep mask without the regions of fewer than s pixels that border a
    removed outlier of similar flow (Sec. 3.7)."""
    H, W = keep.shape
    out = torch.empty((H, W), dtype=torch.uint8, device=keep.device)
    nbytes = int(lib().ff_region_filter_scratch_bytes(W, H))
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=keep.device)
    check(lib().ff_region_filter(_ptr(flow, torch.int16), _ptr(cost, torch.int32), _ptr(keep, torch.uint8), W, H, s,
                                 _ptr(scratch), nbytes, _ptr(out), _stream()), "ff_region_filter")
    return out


def sparsify(flow_a, keep_a, flow_b1, flow_b2=None, q: int = 3, e: int = 1) -> torch.Tensor:
    """One sample per q x q region (Sec. 3.8): int32 [ceil(H/q)][ceil(W/q)]
    pixel indices y * W + x of the selections, -1 where none."""
    H, W = keep_a.shape
    sel = torch.empty((-(-H // q), -(-W // q)), dtype=torch.int32, device=keep_a.device)
    check(lib().ff_sparsify(_ptr(flow_a, torch.int16), _ptr(keep_a, torch.uint8), _ptr(flow_b1, torch.int16),
                            _ptr(flow_b2, torch.int16), W, H, q, e, _ptr(sel), _stream()), "ff_sparsify")
    return sel


def flow_fields_two_backward(img1, img2, params: Params, seed2: int | None = None, radius2: int | None = None):
    """Flow Fields with the check against two backward fields (Sec. 3.7).
    The second backward field is the forward field of a second run on the
    swapped images with generator seed `seed2` (default seed + 1) and patch
    radius `radius2` (default the same radius); keep_fwd becomes the mask
    against both backward fields (keep_bwd stays the single check of the
    first backward field).  Adds flow_bwd2 and cost_bwd2 to the result."""
    out = flow_fields(img1, img2, params)
    p2 = dataclasses.replace(params, seed=params.seed + 1 if seed2 is None else seed2,
                             radius=params.radius if radius2 is None else radius2)
    o2 = flow_fields(img2, img1, p2, backward=False)
    out["keep_fwd"] = consistency_filter2(out["flow_fwd"], out["cost_fwd"], out["flow_bwd"], out["cost_bwd"],
                                          o2["flow_fwd"], o2["cost_fwd"], params.eps)
    out["flow_bwd2"], out["cost_bwd2"] = o2["flow_fwd"], o2["cost_fwd"]
    return out


def workspace_bytes(W: int, H: int, params: Params) -> int:
    p = params.to_c()
    return int(lib().ff_workspace_bytes(W, H, p))


class FlowFields:
    """Reusable buffers for repeated ff_flow_fields calls on one frame size."""

    def __init__(self, W: int, H: int, params: Params, device="cuda", backward: bool = True):
        """backward=False: the forward field only (flow_fwd, cost_fwd,
        n_evals[0]); no backward field and no consistency masks."""
        self.W, self.H, self.params, self.backward = W, H, params, backward
        self._cp = params.to_c()
        nbytes = int(lib().ff_workspace_bytes(W, H, self._cp))
        if nbytes == 0:
            raise ffi.FlowFieldsError(ffi.FF_ERR_ARG, "ff_workspace_bytes")
        dev = torch.device(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        Ho, Wo = ((H + 1) // 2, (W + 1) // 2) if params.fast_x2 else (H, W)  # Fast x2: grid of scale 2
        self.out = {
            "flow_fwd": torch.empty((Ho, Wo, 2), dtype=torch.int16, device=dev),
            "flow_bwd": torch.empty((Ho, Wo, 2), dtype=torch.int16, device=dev),
            "cost_fwd": torch.empty((Ho, Wo), dtype=torch.int32, device=dev),
            "cost_bwd": torch.empty((Ho, Wo), dtype=torch.int32, device=dev),
            "keep_fwd": torch.empty((Ho, Wo), dtype=torch.uint8, device=dev),
            "keep_bwd": torch.empty((Ho, Wo), dtype=torch.uint8, device=dev),
            "n_evals": torch.zeros(2, dtype=torch.int64, device=dev),
        }
        if not backward:
            for k in ("flow_bwd", "cost_bwd", "keep_fwd", "keep_bwd"):
                del self.out[k]

    def capture(self, img1: torch.Tensor, img2: torch.Tensor):
        """Records one call on these input buffers into a HIP graph
        (torch.cuda.CUDAGraph; a warm-up call runs first).  replay() then
        re-runs the whole call with one graph launch; the inputs are read
        from the same buffers at every replay."""
        s = torch.cuda.Stream(device=self.ws.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self(img1, img2)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self(img1, img2)
        self.graph = g
        return g

    def replay(self) -> dict:
        if getattr(self, "graph", None) is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.out

    def __call__(self, img1: torch.Tensor, img2: torch.Tensor) -> dict:
        if tuple(img1.shape) != (self.H, self.W) or tuple(img2.shape) != (self.H, self.W):
            raise ValueError("image shape does not match")
        o = self.out
        check(lib().ff_flow_fields(_ptr(img1, torch.uint8, "img1"), _ptr(img2, torch.uint8, "img2"), self.W, self.H,
                                   self._cp, _ptr(self.ws), self.ws.numel(), _ptr(o["flow_fwd"]),
                                   _ptr(o.get("flow_bwd")), _ptr(o["cost_fwd"]), _ptr(o.get("cost_bwd")),
                                   _ptr(o.get("keep_fwd")), _ptr(o.get("keep_bwd")), _ptr(o["n_evals"]), _stream()),
              "ff_flow_fields")
        return o


def flow_fields(img1: torch.Tensor, img2: torch.Tensor, params: Params | None = None, backward: bool = True) -> dict:
    """Forward and backward Flow Fields of one pair plus consistency masks
    (backward=False: the forward field only)."""
    params = params or Params()
    H, W = img1.shape
    ff = FlowFields(W, H, params, device=img1.device, backward=backward)
    return {k: v for k, v in ff(img1, img2).items()}
