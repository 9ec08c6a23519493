"""The C ABI library loads, exports every symbol its header declares and
rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

import paper_1703_02563_amd as ff
from paper_1703_02563_amd import ffi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ff_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = ffi.lib()
    names = _declared()
    assert {"ff_init_nn", "ff_propagate_level", "ff_random_search", "ff_consistency_filter",
            "ff_flow_fields"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert lib.ff_version() >= 1


def test_status_strings():
    assert ffi.status_str(0) == "ok"
    assert "invalid" in ffi.status_str(1)
    assert "workspace" in ffi.status_str(3)


def test_workspace_bytes_and_validation():
    lib = ffi.lib()
    p = ff.Params(levels=5, iters=6).to_c()
    n = lib.ff_workspace_bytes(1024, 436, C.byref(p))
    assert n > 1024 * 436 * 16 * 10  # at least the ten descriptor maps
    for bad in (dict(levels=0), dict(levels=8), dict(iters=0), dict(radius=8), dict(R_den=0)):
        q = ff.Params(**{**dict(levels=5, iters=6), **bad}).to_c()
        assert lib.ff_workspace_bytes(64, 64, C.byref(q)) == 0
    assert lib.ff_workspace_bytes(0, 10, C.byref(p)) == 0
    assert lib.ff_workspace_bytes(40000, 10, C.byref(p)) == 0
    # the NN seed's 32-bit descriptor offsets: fewer than 2^27 pixels
    assert lib.ff_workspace_bytes(16384, 8191, C.byref(p)) > 0
    assert lib.ff_workspace_bytes(16384, 8192, C.byref(p)) == 0
    assert lib.ff_workspace_bytes_f32(16384, 8192, C.byref(p)) == 0


def test_bad_arguments_return_before_any_launch():
    lib = ffi.lib()
    p = ff.Params().to_c()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    # NULL image
    assert lib.ff_flow_fields(None, fake, 64, 64, C.byref(p), fake, 1 << 30, fake, fake, fake, fake, fake, None,
                              None, None) == ffi.FF_ERR_ARG
    # backward outputs only partly NULL (all NULL is the forward-only mode)
    assert lib.ff_flow_fields(fake, fake, 64, 64, C.byref(p), fake, 1 << 30, fake, None, fake, fake, fake, None,
                              None, None) == ffi.FF_ERR_ARG
    assert lib.ff_flow_fields(fake, fake, 64, 64, C.byref(p), fake, 1 << 30, fake, None, fake, None, fake, None,
                              None, None) == ffi.FF_ERR_ARG
    # too small a workspace
    assert lib.ff_flow_fields(fake, fake, 64, 64, C.byref(p), fake, 16, fake, fake, fake, fake, fake, None, None,
                              None) == ffi.FF_ERR_WORKSPACE
    # bad sizes / scales / passes
    assert lib.ff_descriptors(fake, 0, 5, 1, fake, fake, fake, None, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_descriptors(fake, 5, 5, 65, fake, fake, fake, None, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_descriptors(fake, 5, 5, 0, fake, fake, fake, None, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_descriptors(fake, 5, 5, 128, fake, fake, fake, None, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_propagate_level(fake, fake, 5, 5, 1, 3, -1, fake, fake, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_random_search(fake, fake, 5, 5, 1, 3, -2, 1, 0, 0, 0, fake, fake, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_consistency_filter(fake, fake, fake, None, 5, 5, 1.0, fake, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_init_nn(fake, fake, fake, fake, 5, 5, 6, 3, fake, fake, fake, fake, None, None) == ffi.FF_ERR_ARG
    assert lib.ff_consistency_filter2(fake, fake, fake, fake, None, fake, 5, 5, 1.0, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_consistency_filter2(fake, fake, fake, fake, fake, fake, 5, 5, -1.0, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_sparsify(fake, fake, fake, None, 5, 5, 0, 1, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_sparsify(fake, fake, fake, None, 5, 5, 65, 1, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_sparsify(fake, fake, fake, None, 5, 5, 3, -1, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_sparsify(fake, fake, None, None, 5, 5, 3, 1, fake, None) == ffi.FF_ERR_ARG
    assert lib.ff_region_filter_scratch_bytes(0, 5) == 0
    assert lib.ff_region_filter_scratch_bytes(10, 5) == 10 * 5 * 12
    assert lib.ff_region_filter(fake, fake, fake, 10, 5, -1, fake, 600, C.c_void_p(0x2000), None) == ffi.FF_ERR_ARG
    assert lib.ff_region_filter(fake, fake, fake, 10, 5, 3, fake, 600, fake, None) == ffi.FF_ERR_ARG  # in place
    assert lib.ff_region_filter(fake, fake, fake, 10, 5, 3, fake, 599, C.c_void_p(0x2000), None) == \
        ffi.FF_ERR_WORKSPACE
    assert lib.ff_region_filter(fake, fake, fake, 10, 5, 3, C.c_void_p(0x3002), 600, C.c_void_p(0x2000), None) == \
        ffi.FF_ERR_ARG  # misaligned scratch
    # bad Flow Fields+ schedules
    for kw in ({"plus_iters": -1}, {"plus_iters": 60, "iters": 6}, {"Rp_num": -2}, {"fine_iters": 65},
               {"fine_iters": -1}, {"Rp_num": (1 << 20) + 1}):
        q = ff.Params(**kw).to_c()
        assert lib.ff_workspace_bytes(64, 64, C.byref(q)) == 0, kw
        assert lib.ff_flow_fields(fake, fake, 64, 64, C.byref(q), fake, 1 << 30, fake, fake, fake, fake, fake, None,
                                  None, None) == ffi.FF_ERR_ARG, kw
    # misaligned convolution input (16-byte loads of channel chunks)
    assert lib.ff_conv3x3_fwd(C.c_void_p(0x1008), 1, 4, 4, 32, 32, fake, None, 0, None, fake, None) == ffi.FF_ERR_ARG


def test_python_binding_rejects_host_tensors():
    import torch
    with pytest.raises(ValueError):
        ff.descriptors(torch.zeros((4, 4), dtype=torch.uint8), 1)


def test_descriptor_map_bytes():
    """Padded descriptor maps: (W + 8n) x (H + 8n) entries of 16 bytes."""
    lib = ff.lib()
    for W, H, n in [(1024, 436, 1), (1024, 436, 16), (1, 1, 64), (37, 53, 4)]:
        assert lib.ff_descriptor_map_bytes(W, H, n) == (W + 8 * n) * (H + 8 * n) * 16
    assert lib.ff_descriptor_map_bytes(0, 5, 1) == 0
    # a sub-scale (not a power of two) has the same padding: 4 n per side
    assert lib.ff_descriptor_map_bytes(5, 5, 3) == (5 + 24) * (5 + 24) * 16
    assert lib.ff_descriptor_map_bytes(5, 5, 65) == 0 and lib.ff_descriptor_map_bytes(5, 5, 0) == 0
    assert lib.ff_descriptor_map_bytes(5, 5, 128) == 0


def test_default_tuning_and_validation():
    """The built-in launch tables, and tables out of range rejected before
    anything is enqueued."""
    lib = ff.lib()
    assert lib.ff_level_variant_count_f32() == 5
    t = ff.default_tuning()
    assert t.variant_f32 == [0, 0, 1, 1, 1, 1, 1] and t.passes_f32 == [1] * 7
    assert all(0 <= v < lib.ff_level_variant_count() for v in t.variant)
    assert t.variant == [31, 11, 30, 26, 32, 3, 3] and t.passes == [3, 3, 3, 3, 3, 0, 0]
    fake = C.c_void_p(0x1000)
    for bad in (dict(variant=[lib.ff_level_variant_count()] * 7), dict(variant=[-1] * 7), dict(passes=[65] * 7),
                dict(passes_f32=[-1] * 7), dict(variant_f32=[5] * 7)):
        q = ff.Params(tuning=t.replace(**bad)).to_c()
        assert lib.ff_workspace_bytes(64, 64, C.byref(q)) == 0, bad
        assert lib.ff_flow_fields(fake, fake, 64, 64, C.byref(q), fake, 1 << 30, fake, fake, fake, fake, fake, None,
                                  None, None) == ffi.FF_ERR_ARG, bad
    ok = ff.Params(tuning=t.replace(variant=[3] * 7, passes=[2] * 7)).to_c()
    assert lib.ff_workspace_bytes(64, 64, C.byref(ok)) > 0


def test_level_launches_follow_the_run_length_table():
    """Launches per scale: the halo of the blocked kernel holds 6 steps
    (3 per side pair), the run-length table caps a run; tables per call."""
    lib = ff.lib()
    t = ff.default_tuning().replace(variant=[3] * 7)  # 16x16 tiles, the widest halo
    for passes, T, expect in [(0, 6, 1), (0, 9, 2), (1, 6, 6), (2, 6, 3), (3, 6, 2), (4, 7, 2), (0, 1, 1)]:
        tc = t.replace(passes=[passes] * 7).to_c()
        assert lib.ff_level_launches(C.byref(tc), T, 1, 0) == expect, (passes, T)
        assert ff.level_launches(ff.Params(iters=T, tuning=t.replace(passes=[passes] * 7)), 1) == expect
    assert lib.ff_level_launches(None, 6, 1, 0) == 3  # the built-in table at n = 2: a halo of 2, 2 steps per launch
    assert lib.ff_level_launches(None, 6, 2, 0) == 2  # at n = 4: a halo of 6 capped at 3 steps per launch
    assert lib.ff_level_launches(None, 0, 1, 0) == -1 and lib.ff_level_launches(None, 6, 9, 0) == -1
    assert lib.ff_level_launches(None, 6, 1, 2) == -1


def test_run_level_pair_validation():
    """ff_run_level_pair rejects bad arguments, a short scratch and the
    forms the blocked kernels do not run, before anything is enqueued."""
    lib = ff.lib()
    fake = C.c_void_p(0x1000)
    two = (C.c_void_p * 2)(0x1000, 0x2000)
    one_null = (C.c_void_p * 2)(0x1000, None)
    W, H, lv = 64, 48, 0
    need = 2 * lib.ff_run_level_scratch_bytes(W, H, lv)

    def call(prm=None, mode=0, flows=two, costs=two, keys=None, scratch_bytes=need):
        q = (prm or ff.Params(levels=1, iters=2)).to_c()
        return lib.ff_run_level_pair(fake, fake, None, None, W, H, lv, C.byref(q), mode, keys, None, None, flows,
                                     costs, fake, scratch_bytes, None, None, None)

    assert call(flows=None) == ffi.FF_ERR_ARG
    assert call(costs=one_null) == ffi.FF_ERR_ARG
    assert call(mode=1) == ffi.FF_ERR_ARG  # no NN keys
    assert call(mode=3) == ffi.FF_ERR_ARG
    assert call(scratch_bytes=need - 1) == ffi.FF_ERR_WORKSPACE
    assert call(prm=ff.Params(levels=1, iters=2, subpixel=3)) == ffi.FF_ERR_UNSUPPORTED
    assert call(prm=ff.Params(levels=1, iters=2, raster=True)) == ffi.FF_ERR_UNSUPPORTED


def test_noalloc_region_filter_validation():
    """Sizes beyond the static scratch array and bad arguments return before
    anything is enqueued."""
    lib = ffi.lib()
    fake = C.c_void_p(0x1000)
    out = C.c_void_p(0x2000)
    maxpx = int(lib.ff_region_filter_noalloc_max_pixels())
    assert maxpx == 1 << 21
    assert lib.ff_region_filter_noalloc(fake, fake, fake, 2049, 1024, 3, out, None) == ffi.FF_ERR_WORKSPACE
    assert lib.ff_region_filter_noalloc(fake, fake, fake, 10, 5, -1, out, None) == ffi.FF_ERR_ARG
    assert lib.ff_region_filter_noalloc(fake, fake, fake, 10, 5, 3, fake, None) == ffi.FF_ERR_ARG  # in place
    assert lib.ff_region_filter_noalloc(None, fake, fake, 10, 5, 3, out, None) == ffi.FF_ERR_ARG
    assert lib.ff_region_filter_noalloc(fake, fake, fake, 0, 5, 3, out, None) == ffi.FF_ERR_ARG


def test_subpixel_arguments():
    """The subpixel form accepts 0 or 3 bits and frames up to 4095 px; the
    batch and learned-feature calls do not support it."""
    lib = ffi.lib()
    fake = C.c_void_p(0x1000)
    for bad in (1, 2, 4, -1):
        q = ff.Params(subpixel=bad).to_c()
        assert lib.ff_workspace_bytes(64, 64, C.byref(q)) == 0, bad
    q = ff.Params(subpixel=3).to_c()
    assert lib.ff_workspace_bytes(64, 64, C.byref(q)) > 0
    assert lib.ff_flow_fields(fake, fake, 4096, 8, C.byref(q), fake, 1 << 40, fake, fake, fake, fake, fake, None,
                              None, None) == ffi.FF_ERR_ARG
    assert lib.ff_consistency_filter_sub(fake, fake, fake, fake, 8, 8, 4, C.c_float(1.0), fake, None, None) == \
        ffi.FF_ERR_ARG
