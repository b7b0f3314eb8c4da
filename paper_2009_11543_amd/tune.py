"""Autotuning of per-index sort options, with a JSON cache.

For an index (keys + bitmap) the candidates are the radix sort at several
digit widths and, when a CDF model is given, the splitter and learned
bucketing sorts; each is timed on the device by ckey_tune_index (one warm-up
and one timed rebuild).  Results are cached by (rows, key bytes, |D|, device
name) so a table's later rebuilds reuse the choice.
"""
import json
import os

import numpy as np
import torch

from . import ckey


def _cache_key(keys, nbits):
    dev = torch.cuda.get_device_name(keys.data.device)
    return f"n={keys.n};L={keys.key_bytes};nbits={nbits};dev={dev}"


def candidates(model=None, digit_bits=(5, 6, 7, 8)):
    c = [dict(method=ckey.CKEY_SORT_RADIX, digit_bits=d) for d in digit_bits]
    if model is not None:
        c.append(dict(method=ckey.CKEY_SORT_SPLITTER, model=model))
        c.append(dict(method=ckey.CKEY_SORT_LEARNED, model=model))
    return c


def _describe(opt):
    return {k: (v if k != "model" else "model") for k, v in opt.items()}


def autotune(keys, bitmap, model=None, cache_path=None, digit_bits=(5, 6, 7, 8)):
    """Fastest option dict for rebuilding ``keys`` with ``bitmap`` (host array or
    None for a first build); with a cache file, reuse a previous decision."""
    bitmap = None if bitmap is None else np.asarray(bitmap, np.uint8)
    nbits = 8 * keys.key_bytes if bitmap is None else ckey.ckey_plan_query(bitmap)["nbits"]
    key = _cache_key(keys, nbits)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    cands = candidates(model, digit_bits)
    if key in cache:
        want = cache[key]["choice"]
        for c in cands:
            if _describe(c) == want:
                return c, cache[key]
    best, times = ckey.ckey_tune_index({"keys": keys, "bitmap": bitmap}, cands)
    rec = {"choice": _describe(cands[best]), "times_ms": [float(t) for t in times],
           "candidates": [_describe(c) for c in cands]}
    if cache_path:
        cache[key] = rec
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return cands[best], rec
