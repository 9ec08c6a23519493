"""ctypes binding of ``libflowfields.so`` (the C ABI in include/flowfields.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  If the library is missing this module raises; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflowfields.so")

FF_OK, FF_ERR_ARG, FF_ERR_LAUNCH, FF_ERR_WORKSPACE, FF_ERR_UNSUPPORTED = range(5)
UNSET = 0xFFFFFFFF


class FlowFieldsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})" if what else status_str(status))


class FFTuning(C.Structure):
    """Mirror of ff_tuning (launch tables per scale log2 n = 0..6)."""
    _fields_ = [
        ("variant", C.c_int32 * 7),
        ("passes", C.c_int32 * 7),
        ("variant_f32", C.c_int32 * 7),
        ("passes_f32", C.c_int32 * 7),
    ]


class FFParams(C.Structure):
    """Mirror of ff_params."""
    _fields_ = [
        ("levels", C.c_int32),
        ("iters", C.c_int32),
        ("radius", C.c_int32),
        ("R_num", C.c_int32),
        ("R_den", C.c_int32),
        ("eps", C.c_float),
        ("seed", C.c_uint64),
        ("plus_iters", C.c_int32),
        ("Rp_num", C.c_int32),
        ("fine_iters", C.c_int32),
        ("subpixel", C.c_int32),
        ("tuning", C.POINTER(FFTuning)),
        ("nn_l", C.c_int32),
        ("raster", C.c_int32),
        ("fast_x2", C.c_int32),
        ("subscales", C.c_int32),
    ]


_lib = None

# name -> (restype, argtypes); P = pointer-sized integer (device address)
_P = C.c_void_p
_I32 = C.c_int32
_SIGS = {
    "ff_version": (C.c_int, []),
    "ff_status_str": (C.c_char_p, [C.c_int]),
    "ff_descriptors": (C.c_int, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "ff_descriptor_map_bytes": (C.c_size_t, [_I32, _I32, _I32]),
    "ff_wform_map_bytes": (C.c_size_t, [_I32, _I32, _I32]),
    "ff_init_nn": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "ff_nn_topl_scratch_bytes": (C.c_size_t, [_I32, _I32, _I32]),
    "ff_nn_topl": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _P, C.c_size_t, _P, _P]),
    "ff_init_nn_l": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, C.c_size_t, _P, _P, _P, _P,
                               _P]),
    "ff_propagate_raster": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    "ff_rescore_level": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    "ff_seed_level": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    "ff_propagate_level": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    "ff_random_search": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, C.c_uint64, _I32, _I32, _I32, _P, _P,
                                   _P, _P]),
    "ff_consistency_filter": (C.c_int, [_P, _P, _P, _P, _I32, _I32, C.c_float, _P, _P, _P]),
    "ff_consistency_filter2": (C.c_int, [_P, _P, _P, _P, _P, _P, _I32, _I32, C.c_float, _P, _P]),
    "ff_consistency_filter_grid": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, C.c_float, _P, _P, _P]),
    "ff_consistency_filter_sub": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, C.c_float, _P, _P, _P]),
    "ff_sparsify": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P]),
    "ff_region_filter_scratch_bytes": (C.c_size_t, [_I32, _I32]),
    "ff_region_filter": (C.c_int, [_P, _P, _P, _I32, _I32, _I32, _P, C.c_size_t, _P, _P]),
    "ff_region_filter_noalloc_max_pixels": (C.c_size_t, []),
    "ff_region_filter_noalloc": (C.c_int, [_P, _P, _P, _I32, _I32, _I32, _P, _P]),
    "ff_workspace_bytes": (C.c_size_t, [_I32, _I32, C.POINTER(FFParams)]),
    "ff_run_level": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, C.POINTER(FFParams), _I32, _I32, _P, _P, _P, _P,
                               _P, _P, C.c_size_t, _P, _P, _P]),
    "ff_run_level_scratch_bytes": (C.c_size_t, [_I32, _I32, _I32]),
    "ff_run_level_pair": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, C.POINTER(FFParams), _I32, _P, _P, _P, _P, _P,
                                    _P, C.c_size_t, _P, _P, _P]),
    "ff_cost_f32_fwd": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _I32, _P, _P]),
    "ff_cost_f32_bwd": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P]),
    "ff_conv3x3_fwd": (C.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _P, _P, _I32, _P, _P, _P]),
    "ff_conv3x3_bwd_data": (C.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P]),
    "ff_conv3x3_wgrad_scratch_bytes": (C.c_size_t, [_I32, _I32, _I32, _I32]),
    "ff_conv3x3_bwd_weight": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _P, C.c_size_t, _P, _P, _P]),
    "ff_relu_bwd": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "ff_f32_to_bf16": (C.c_int, [_P, C.c_int64, _P, _P]),
    "ff_image_to_bf16": (C.c_int, [_P, C.c_int64, _P, _P]),
    "ff_adam_step": (C.c_int, [_P, _P, _P, _P, _I32, C.c_float, C.c_float, C.c_float, C.c_float, _I32, _P, _P]),
    "ff_triplet_hinge": (C.c_int, [_P, _I32, C.c_float, C.c_float, C.c_float, _P, _P, _P]),
    "ff_l2norm16_fwd": (C.c_int, [_P, C.c_int64, C.c_float, _P, _P, _P]),
    "ff_descnet_fwd": (C.c_int, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _I32, C.c_float, _P, _P]),
    "ff_l2norm16_bwd": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P]),
    "ff_quantize_scratch_bytes": (C.c_size_t, []),
    "ff_quantize_u8": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "ff_quantize_pair_u8": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P]),
    "ff_workspace_bytes_f32": (C.c_size_t, [_I32, _I32, C.POINTER(FFParams)]),
    "ff_flow_fields_f32": (C.c_int, [_P, _P, _I32, _I32, C.POINTER(FFParams), _P, C.c_size_t, _P, _P, _P, _P, _P,
                                     _P, _P, _P]),
    "ff_level_variant_count": (C.c_int32, []),
    "ff_level_variant_count_f32": (C.c_int32, []),
    "ff_default_tuning": (None, [C.POINTER(FFTuning)]),
    "ff_level_launches": (C.c_int32, [C.POINTER(FFTuning), _I32, _I32, _I32]),
    "ff_flow_fields": (C.c_int, [_P, _P, _I32, _I32, C.POINTER(FFParams), _P, C.c_size_t, _P, _P, _P, _P, _P, _P,
                                 _P, _P]),
}


def lib():
    """Loads the library (once); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FlowFieldsError(FF_ERR_UNSUPPORTED,
                                  f"{LIB_PATH} is not built (python -m paper_1703_02563_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    try:
        return lib().ff_status_str(s).decode()
    except FlowFieldsError:
        return f"status {s}"


def check(status: int, what: str):
    if status != FF_OK:
        raise FlowFieldsError(status, what)
