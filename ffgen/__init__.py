"""Seeded synthetic inputs (image pairs, ground truth) and quality metrics.

Holds none of the Flow Fields arithmetic; shared by the tests, the oracle
checks and the benchmark.
"""
from .synth import (FF_SEED, CONFIG_PARAMS, FFConfig, Pair, batch_shapes, make_pair, pair_seed,
                    random_images, translated_crops)
from .metrics import epe_stats

__all__ = ["FF_SEED", "CONFIG_PARAMS", "FFConfig", "Pair", "batch_shapes", "make_pair", "pair_seed",
           "random_images", "translated_crops", "epe_stats"]
