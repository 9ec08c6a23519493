"""CPU oracle of the Flow Fields hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
The plain-integer path lives in ``ff_oracle.c`` (plain C, scalar loops) and
is reached through the ctypes wrappers in ``oracle.core``; the float cost of
the learned-descriptor form and its gradient live in ``oracle.float_cost``
(NumPy, float64).
"""
from .core import (UNSET, build, lib, blur, descriptor, descriptors_all, cost, nn, init_coarse, seed_level,
                   propagate, random_search, rs_offset, rs_radius, consistency, consistency2, region_filter,
                   sparsify, flow_fields, mix64, cost_f32, quantize_u8, quantize_pair_u8, flow_fields_f32,
                   cost_sub, propagate_sub, random_search_sub, consistency_sub, nn_topl, init_coarse_l,
                   propagate_raster, consistency_grid, stages, rescore, seed_level_m, propagate_m,
                   random_search_m)

__all__ = ["UNSET", "build", "lib", "blur", "descriptor", "descriptors_all", "cost", "nn", "init_coarse",
           "seed_level", "propagate", "random_search", "rs_offset", "rs_radius", "consistency", "consistency2",
           "region_filter", "sparsify", "flow_fields", "mix64", "cost_f32", "quantize_u8", "quantize_pair_u8",
           "flow_fields_f32", "cost_sub", "propagate_sub", "random_search_sub", "consistency_sub", "nn_topl",
           "init_coarse_l", "propagate_raster", "consistency_grid", "stages", "rescore", "seed_level_m",
           "propagate_m", "random_search_m"]
