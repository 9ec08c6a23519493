"""Autotuner of the level-kernel launch configuration.

The temporally blocked level kernel comes in several variants (tile size,
workgroup size, load unrolling; see ff_level_variant_count).  Results never
depend on the variant; speed does, and differently at every scale.  The tuner
times complete ff_flow_fields calls with HIP events on the current stream and
picks, scale by scale (coordinate descent from the current table), the
fastest variant.  Tables are cached in a JSON file keyed by GPU
architecture, frame size and schedule.
"""
from __future__ import annotations

import json
import os

import torch

from . import flowfields as ffm

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _key(W, H, params: ffm.Params) -> str:
    # the architecture (not the marketing name, which depends on how the
    # runtime was started) identifies the kernels' target
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"{arch}|{W}x{H}|L{params.levels}|T{params.iters}|r{params.radius}"


def time_call(fn, reps: int = 10, warmup: int = 2) -> float:
    """Median milliseconds of fn() over reps, HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(img1: torch.Tensor, img2: torch.Tensor, params: ffm.Params, reps: int = 10, verbose: bool = False,
         rounds: int = 2):
    """Returns (table, log): table = {"variants": [...], "passes": [...]},
    the fastest level-kernel variant and then the fastest run length (most
    propagation steps per launch, 0 = no limit) of every scale, by
    coordinate descent repeated `rounds` times (the two interact)."""
    H, W = img1.shape
    runner = ffm.FlowFields(W, H, params, device=img1.device)
    return tune_call(lambda: runner(img1, img2), params.levels, reps, verbose, rounds)


def tune_call(fn, levels: int, reps: int = 10, verbose: bool = False, rounds: int = 2, variants=None):
    """tune() for any timed call `fn` (a batch, for instance); `variants`
    restricts the variant indices tried."""
    nvar = int(ffm.lib().ff_level_variant_count())
    choices = list(range(nvar)) if variants is None else list(variants)
    table = ffm.level_variants()
    passes = ffm.level_passes(0)
    log = []

    def best_of(choices, apply):
        best = None
        for c in choices:
            apply(c)
            ms = time_call(fn, reps=reps)
            log.append({"log2n": lv, "choice": c, "ms": ms})
            if verbose:
                print(f"autotune: log2n={lv} {c} {ms:.4f} ms", flush=True)
            if best is None or ms < best[1]:
                best = (c, ms)
        return best[0]

    for _ in range(rounds):
        for lv in range(levels):
            def set_variant(v):
                trial = list(table)
                trial[lv] = v
                ffm.set_level_variants(trial)
            table[lv] = best_of([("variant", v) for v in choices], lambda c: set_variant(c[1]))[1]
            ffm.set_level_variants(table)
        for lv in range(levels):
            def set_passes(p):
                trial = list(passes)
                trial[lv] = p
                ffm.set_level_passes(trial, 0)
            passes[lv] = best_of([("passes", p) for p in (0, 3, 2, 1)], lambda c: set_passes(c[1]))[1]
            ffm.set_level_passes(passes, 0)
    return {"variants": table, "passes": passes}, log


def batch_key(npairs: int, params: ffm.Params) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"{arch}|batch{npairs}|L{params.levels}|T{params.iters}|r{params.radius}"


def load_batch(npairs: int, params: ffm.Params, path: str = DEFAULT_CACHE):
    """The cached table of batches of `npairs` pairs, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(batch_key(npairs, params))


def save_entry(key: str, table, path: str = DEFAULT_CACHE) -> None:
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[key] = table
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def load(W: int, H: int, params: ffm.Params, path: str = DEFAULT_CACHE) -> bool:
    """Applies a cached table if one exists for this device and shape."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        cache = json.load(f)
    entry = cache.get(_key(W, H, params))
    if entry is None:
        return False
    if isinstance(entry, list):  # variants only
        entry = {"variants": entry}
    ffm.set_level_variants(entry["variants"])
    if "passes" in entry:
        ffm.set_level_passes(entry["passes"], 0)
    return True


def save(W: int, H: int, params: ffm.Params, table, path: str = DEFAULT_CACHE) -> None:
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[_key(W, H, params)] = table if isinstance(table, dict) else list(table)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
