"""MI355X-native Flow Fields hot path (Bailer, Taetz, Stricker, "Flow Fields").

The work runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/flowfields.h (``libflowfields.so``); this package is its thin
Python binding.
"""
from .ffi import FlowFieldsError, lib  # noqa: F401
from .flowfields import (FlowFields, Params, consistency_filter, consistency_filter2, descriptors,  # noqa: F401
                         flow_fields, flow_fields_two_backward,
                         init_nn, level_passes, level_variants, level_variants_f32, propagate_level, random_search,
                         rs_radius, run_level, seed_level, set_level_passes, set_level_variants,
                         set_level_variants_f32, region_filter, sparsify, workspace_bytes)

__all__ = ["FlowFieldsError", "lib", "FlowFields", "Params", "consistency_filter", "consistency_filter2",
           "descriptors", "flow_fields", "flow_fields_two_backward",
           "init_nn", "level_passes", "level_variants", "level_variants_f32", "set_level_passes", "set_level_variants",
           "set_level_variants_f32", "propagate_level", "random_search", "rs_radius", "run_level", "seed_level",
           "region_filter", "sparsify", "workspace_bytes"]
