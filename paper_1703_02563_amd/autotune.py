"""Autotuner of the level-kernel launch tables.

The temporally blocked level kernel comes in several variants (tile size,
workgroup size, load unrolling; see ff_level_variant_count) and runs a scale
in runs of a few steps per launch.  Results never depend on the tables;
speed does, and differently at every scale.  The tuner times complete calls
with HIP events on the current stream and picks, scale by scale (coordinate
descent from a start table), the fastest variant and then the fastest run
length.  Tables travel with each call (Params.tuning, the C ABI's
ff_tuning) and are cached in a JSON file keyed by GPU architecture, frame
size and schedule.
"""
from __future__ import annotations

import dataclasses
import json
import os

import torch

from . import flowfields as ffm

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _arch() -> str:
    # the architecture (not the marketing name, which depends on how the
    # runtime was started) identifies the kernels' target
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"


def _key(W, H, params: ffm.Params) -> str:
    return f"{_arch()}|{W}x{H}|L{params.levels}|T{params.iters}|r{params.radius}"


def batch_key(npairs: int, params: ffm.Params) -> str:
    return f"{_arch()}|batch{npairs}|L{params.levels}|T{params.iters}|r{params.radius}"


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
    """Returns (tuning, log) for ff_flow_fields on this pair's shape."""
    H, W = img1.shape

    def make(prm):
        runner = ffm.FlowFields(W, H, prm, device=img1.device)
        return lambda: runner(img1, img2)
    return tune_call(make, params, reps, verbose, rounds)


def tune_call(make, params: ffm.Params, reps: int = 10, verbose: bool = False, rounds: int = 2, variants=None):
    """Coordinate descent over the byte-descriptor tables: make(params) must
    return the call to time with those params; `variants` restricts the
    variant indices tried.  Starts from params.tuning (or the built-in
    table); returns (tuning, log)."""
    nvar = int(ffm.lib().ff_level_variant_count())
    choices = list(range(nvar)) if variants is None else list(variants)
    tun = params.tuning or ffm.default_tuning()
    log = []

    def timed(t):
        return time_call(make(dataclasses.replace(params, tuning=t)), reps=reps)

    for _ in range(rounds):
        for what, opts in (("variant", choices), ("passes", (0, 3, 2, 1))):
            for lv in range(params.levels):
                best = None
                for c in opts:
                    vals = list(getattr(tun, what))
                    vals[lv] = c
                    trial = tun.replace(**{what: vals})
                    ms = timed(trial)
                    log.append({"log2n": lv, what: c, "ms": ms})
                    if verbose:
                        print(f"autotune: log2n={lv} {what} {c} {ms:.4f} ms", flush=True)
                    if best is None or ms < best[1]:
                        best = (trial, ms)
                tun = best[0]
    return tun, log


def _entry_to_tuning(entry) -> ffm.Tuning:
    t = ffm.default_tuning()
    if isinstance(entry, list):  # variants only
        entry = {"variants": entry}
    t = t.replace(variant=entry["variants"])
    if "passes" in entry:
        t = t.replace(passes=entry["passes"])
    return t


def _load_entry(key: str, path: str):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        entry = json.load(f).get(key)
    return None if entry is None else _entry_to_tuning(entry)


def load(W: int, H: int, params: ffm.Params, path: str = DEFAULT_CACHE):
    """The cached tables for this device and shape, or None."""
    return _load_entry(_key(W, H, params), path)


def load_batch(npairs: int, params: ffm.Params, path: str = DEFAULT_CACHE):
    """The cached tables of batches of `npairs` pairs, or None."""
    return _load_entry(batch_key(npairs, params), path)


def save_entry(key: str, tuning: ffm.Tuning, path: str = DEFAULT_CACHE) -> None:
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[key] = {"variants": list(tuning.variant), "passes": list(tuning.passes)}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def save(W: int, H: int, params: ffm.Params, tuning: ffm.Tuning, path: str = DEFAULT_CACHE) -> None:
    save_entry(_key(W, H, params), tuning, path)
