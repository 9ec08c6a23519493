"""Per-call launch tables for the tests."""
import dataclasses

import paper_1703_02563_amd as ff


def with_tuning(prm, **tables):
    """prm with launch tables = the built-in ones with the given entries
    (variant, passes, variant_f32, passes_f32: lists per scale log2 n)
    replaced; 7 entries each, shorter lists are padded from the defaults."""
    base = prm.tuning or ff.default_tuning()
    full = {}
    for k, v in tables.items():
        v = [int(x) for x in v]
        full[k] = v + list(getattr(base, k))[len(v):]
    return dataclasses.replace(prm, tuning=base.replace(**full))
