"""MI355X-native Flow Fields hot path (Bailer, Taetz, Stricker, "Flow Fields").

The work runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/flowfields.h (``libflowfields.so``); this package is its thin
Python binding.
"""
from .ffi import FlowFieldsError, lib  # noqa: F401
from .flowfields import (FlowFields, Params, Tuning, consistency_filter, consistency_filter2,  # noqa: F401
                         consistency_filter_sub, consistency_filter_grid,
                         default_tuning, descriptors, flow_fields, flow_fields_two_backward, init_nn,
                         level_launches, propagate_level, random_search, run_level, run_level_pair, seed_level,
                         region_filter, sparsify, workspace_bytes, nn_topl, init_nn_l, propagate_raster, rescore_level)

__all__ = ["FlowFieldsError", "lib", "FlowFields", "Params", "Tuning", "consistency_filter", "consistency_filter2",
           "consistency_filter_sub", "consistency_filter_grid",
           "default_tuning", "descriptors", "flow_fields", "flow_fields_two_backward", "init_nn", "level_launches",
           "propagate_level", "random_search", "run_level", "run_level_pair", "seed_level", "region_filter", "sparsify",
           "workspace_bytes", "nn_topl", "init_nn_l", "propagate_raster", "rescore_level"]
