"""Batched Flow Fields: many pairs of different sizes per launch, hipGraph replay.

BatchFlowFields owns the device buffers of a batch (images, outputs, the
workspace and the device copy of the pair table) and runs
ff_flow_fields_batched: every stage of the schedule is one persistent launch
over the work items of all pairs.  capture() records one call into a HIP
graph (torch.cuda.CUDAGraph); replay() re-runs it with no host work beyond
the graph launch.
"""
from __future__ import annotations

import ctypes as C

import torch

from .ffi import FF_ERR_ARG, FFParams, FlowFieldsError, check, lib
from .flowfields import Params, _stream


class FFPair(C.Structure):
    """Mirror of ff_pair."""
    _fields_ = [
        ("img1", C.c_void_p), ("img2", C.c_void_p),
        ("W", C.c_int32), ("H", C.c_int32),
        ("flow_fwd", C.c_void_p), ("flow_bwd", C.c_void_p),
        ("cost_fwd", C.c_void_p), ("cost_bwd", C.c_void_p),
        ("keep_fwd", C.c_void_p), ("keep_bwd", C.c_void_p),
        ("n_evals", C.c_void_p),
    ]


_SIGS = {
    "ff_batch_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32, C.POINTER(FFParams)]),
    "ff_batch_table_bytes": (C.c_size_t, [C.c_int32]),
    "ff_batch_table": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(FFParams), C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.c_size_t]),
    "ff_flow_fields_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(FFParams), C.c_void_p, C.c_void_p,
                                         C.c_size_t, C.c_void_p]),
}


def _lib():
    L = lib()
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


class BatchFlowFields:
    """Buffers and launches for a fixed list of frame shapes [(H, W), ...]."""

    def __init__(self, shapes, params: Params, device="cuda"):
        """params.tuning: the level-kernel launch tables of this batch's
        calls (None: the built-in tables)."""
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        self.params = params
        self._cp = params.to_c()
        dev = torch.device(device)
        self.device = dev
        n = len(self.shapes)
        self.img1, self.img2, self.out = [], [], []
        for H, W in self.shapes:
            self.img1.append(torch.zeros((H, W), dtype=torch.uint8, device=dev))
            self.img2.append(torch.zeros((H, W), dtype=torch.uint8, device=dev))
            self.out.append({
                "flow_fwd": torch.empty((H, W, 2), dtype=torch.int16, device=dev),
                "flow_bwd": torch.empty((H, W, 2), dtype=torch.int16, device=dev),
                "cost_fwd": torch.empty((H, W), dtype=torch.int32, device=dev),
                "cost_bwd": torch.empty((H, W), dtype=torch.int32, device=dev),
                "keep_fwd": torch.empty((H, W), dtype=torch.uint8, device=dev),
                "keep_bwd": torch.empty((H, W), dtype=torch.uint8, device=dev),
                "n_evals": torch.zeros(2, dtype=torch.int64, device=dev),
            })
        self.pairs = (FFPair * n)()
        for k, (H, W) in enumerate(self.shapes):
            o = self.out[k]
            self.pairs[k] = FFPair(self.img1[k].data_ptr(), self.img2[k].data_ptr(), W, H,
                                   o["flow_fwd"].data_ptr(), o["flow_bwd"].data_ptr(), o["cost_fwd"].data_ptr(),
                                   o["cost_bwd"].data_ptr(), o["keep_fwd"].data_ptr(), o["keep_bwd"].data_ptr(),
                                   o["n_evals"].data_ptr())
        L = _lib()
        nbytes = int(L.ff_batch_workspace_bytes(self.pairs, n, self._cp))
        tbytes = int(L.ff_batch_table_bytes(n))
        if nbytes == 0 or tbytes == 0:
            raise FlowFieldsError(FF_ERR_ARG, "batch shapes or parameters")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        host = (C.c_uint8 * tbytes)()
        check(L.ff_batch_table(self.pairs, n, self._cp, C.c_void_p(self.ws.data_ptr()), nbytes, host, tbytes),
              "ff_batch_table")
        self.table = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(dev)
        self.graph = None

    def __len__(self):
        return len(self.shapes)

    def set_pair(self, k: int, img1: torch.Tensor, img2: torch.Tensor):
        self.img1[k].copy_(img1)
        self.img2[k].copy_(img2)

    def run(self):
        check(_lib().ff_flow_fields_batched(self.pairs, len(self.shapes), self._cp,
                                            C.c_void_p(self.table.data_ptr()), C.c_void_p(self.ws.data_ptr()),
                                            self.ws.numel(), _stream()), "ff_flow_fields_batched")
        return self.out

    def capture(self):
        """Records one batched call into a HIP graph (warm-up run first)."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.out
