"""Autotuning of per-index sort options, with a JSON cache.

For an index (keys + bitmap) the candidates are the radix sort at several
digit widths and both pass tiles, and, when CDF models are given (one per
bucket count), the splitter and learned bucketing sorts at every given bucket
count and every in-LDS bucket capacity that holds its mean bucket with room
to spare.  Each is timed on the device by ckey_tune_index (one warm-up and one
timed rebuild).  Results are cached by (rows, key bytes, |D|, device name) so
a table's later rebuilds reuse the choice.
"""
import json
import os

import numpy as np
import torch

from . import ckey

# In-LDS capacity (rows) of each bucketing tile choice (ckey_sort_opts.tile).
BUCKET_TILE_ROWS = {1: 2560, 2: 5120, 3: 10240}


def _cache_key(keys, nbits):
    dev = torch.cuda.get_device_name(keys.data.device)
    return f"n={keys.n};L={keys.key_bytes};nbits={nbits};dev={dev}"


def fit_models(sorted_first_words, bucket_log2s, steps=300, batch=1 << 16, seed=3):
    """One CDF model per bucket count, fitted to the sorted first compressed
    words of a previous rebuild (device int64 tensor)."""
    out = {}
    for b in bucket_log2s:
        m = ckey.CdfModel(bucket_log2=b, seed=seed, device=sorted_first_words.device)
        ckey.ckey_cdf_fit(m, sorted_first_words, steps=steps, batch=batch)
        out[b] = m
    return out


def candidates(n, words, models=None, digit_bits=(5, 6, 7, 8), headroom=1.25):
    """Option dicts to time.  models: {bucket_log2: CdfModel} (or None)."""
    tiles = (1, 2) if 1 <= words <= 8 else (0,)
    c = [dict(method=ckey.CKEY_SORT_RADIX, digit_bits=d, tile=t) for d in digit_bits for t in tiles]
    for b, model in sorted((models or {}).items()):
        mean = n / (1 << b)
        caps = [t for t, rows in BUCKET_TILE_ROWS.items() if rows >= headroom * mean]
        for t in caps[:2]:  # the two smallest capacities that fit
            for meth in (ckey.CKEY_SORT_SPLITTER, ckey.CKEY_SORT_LEARNED):
                c.append(dict(method=meth, model=model, tile=t))
    return c


def _describe(opt):
    d = {k: v for k, v in opt.items() if k != "model"}
    if "model" in opt:
        d["bucket_log2"] = opt["model"].bucket_log2
    return d


def autotune(keys, bitmap, model=None, cache_path=None, digit_bits=(5, 6, 7, 8), models=None):
    """Fastest option dict for rebuilding ``keys`` with ``bitmap`` (host array or
    None for a first build); with a cache file, reuse a previous decision.
    model / models: a CdfModel, or {bucket_log2: CdfModel}, for the bucketing
    candidates."""
    bitmap = None if bitmap is None else np.asarray(bitmap, np.uint8)
    nbits = 8 * keys.key_bytes if bitmap is None else ckey.ckey_plan_query(bitmap)["nbits"]
    words = max(1, -(-nbits // 64))
    if model is not None:
        models = dict(models or {})
        models[model.bucket_log2] = model
    key = _cache_key(keys, nbits)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    cands = candidates(keys.n, words, models, digit_bits)
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
