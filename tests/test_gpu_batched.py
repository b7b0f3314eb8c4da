"""GPU tests of the batched table rebuild: all indexes of one table (uneven key
widths, duplicates, var-length-like titles) rebuilt by one call on forked
streams, the same rebuild captured in a HIP graph and replayed (radix and
bucketing methods, with the bucketing sorts' overflow handled on the device),
and the autotuner -- every result compared bit-exactly with the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11543_amd import ckey
    return ckey


@pytest.fixture(scope="module")
def table():
    tab = datagen.table_indexes(1 << 15, seed=3)
    refs = {}
    for name, rows in tab.items():
        k = O.Keys(rows)
        perm = O.full_sort(k)
        d, _ = O.dbits(k, perm)
        refs[name] = (perm, d)
    return tab, refs


def specs_for(ck, tab, refs, first_build_every=2):
    specs = []
    for x, (name, rows) in enumerate(tab.items()):
        bm = None if x % first_build_every == 0 else refs[name][1]
        specs.append({"keys": ck.DeviceKeys.from_numpy(rows), "bitmap": bm, "want_pair_pos": True})
    return specs


def check(ck, tab, refs, outs):
    for (name, rows), o in zip(tab.items(), outs):
        perm, d = refs[name]
        np.testing.assert_array_equal(o["perm"].cpu().numpy().view(np.uint32), perm, err_msg=name)
        np.testing.assert_array_equal(o["bitmap"].cpu().numpy(), d, err_msg=name)


def test_table_rebuild_concurrent(ck, table):
    tab, refs = table
    outs = ck.ckey_rebuild_index(specs_for(ck, tab, refs))
    check(ck, tab, refs, outs)
    # pair positions of one refreshed index against the oracle's refine
    name = list(tab)[1]
    k = O.Keys(tab[name])
    perm, d = refs[name]
    _, pos = O.refine(O.compress(k, d), perm, d)
    np.testing.assert_array_equal(outs[1]["pair_pos"].cpu().numpy().view(np.uint32), pos)


def test_table_rebuild_per_index_options(ck, table):
    tab, refs = table
    specs = specs_for(ck, tab, refs)
    for x, s in enumerate(specs):
        s["opts"] = dict(method=ck.CKEY_SORT_RADIX, digit_bits=4 + x % 5)
    check(ck, tab, refs, ck.ckey_rebuild_index(specs))


def test_table_rebuild_mixed_methods(ck, table):
    """Radix and bucketing indexes in one call (the bucketing ones enqueue
    after the radix ones and wait on their overflow counts): every index still
    gets the oracle's permutation and D-bitmap."""
    import torch
    tab, refs = table
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    specs, models = bucketing_specs(ck, tab, refs, flags)
    check(ck, tab, refs, ck.ckey_rebuild_index(specs))
    torch.cuda.synchronize()
    assert int(flags.item()) & ck.CKEY_FLAG_SPIN_LIMIT == 0


def test_graph_replays(ck, table):
    import torch
    tab, refs = table
    g = ck.RebuildGraph(specs_for(ck, tab, refs))
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for o in g.outs:  # make stale results detectable
            o["perm"].fill_(-1)
            o["bitmap"].fill_(0xAA)
        g.launch()
        torch.cuda.synchronize()
        check(ck, tab, refs, g.outs)
        # eager work between replays: torch ops and an ordinary library call
        junk.mul_(1.5).add_(1.0)
        rows = tab["int64"]
        ck.ckey_rebuild_index([{"keys": ck.DeviceKeys.from_numpy(rows), "bitmap": None}])
        torch.cuda.synchronize()


def bucketing_specs(ck, tab, refs, flags):
    """Refreshes of every index but the first, two of every three with a
    bucketing method whose model is fitted to the index's previous rebuild."""
    specs = specs_for(ck, tab, refs, first_build_every=1 << 30)
    models = []
    for x, (name, rows) in enumerate(tab.items()):
        if x % 3 == 2:
            continue  # stays radix
        prev = ck.ckey_rebuild_index([dict(specs[x], want_ckeys=True)])[0]
        model = ck.CdfModel(bucket_log2=8, seed=3)
        ck.ckey_cdf_fit(model, prev["ckeys"][0].contiguous(), steps=50, batch=1 << 12)
        models.append(model)
        specs[x]["opts"] = dict(method=ck.CKEY_SORT_SPLITTER if x % 3 == 0 else ck.CKEY_SORT_LEARNED,
                                model=model, flags=flags)
    return specs, models


def test_graph_mixed_methods_replays(ck, table):
    """Radix, splitter and learned indexes of one table captured in one graph:
    the bucketing sorts decide on the device whether a bucket overflowed, so
    nothing waits on the host.  Every replay (eager work between them) gives
    the oracle's permutations and D-bitmaps, and raises the overflow flag
    exactly when the same call does uncaptured (the Zipf column's long runs of
    equal keys overflow its buckets)."""
    import torch
    tab, refs = table
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    specs, models = bucketing_specs(ck, tab, refs, flags)
    ck.ckey_rebuild_index(specs)
    torch.cuda.synchronize()
    eager_flags = int(flags.item())
    g = ck.RebuildGraph(specs)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for o in g.outs:
            o["perm"].fill_(-1)
            o["bitmap"].fill_(0xAA)
        flags.zero_()
        print(f"mixed-method graph replay {rep}", flush=True)
        g.launch()
        torch.cuda.synchronize()
        check(ck, tab, refs, g.outs)
        assert int(flags.item()) == eager_flags
        junk.mul_(1.5).add_(1.0)
        ck.ckey_rebuild_index([{"keys": ck.DeviceKeys.from_numpy(tab["int64"]), "bitmap": None}])
        torch.cuda.synchronize()


def concentrated_keys(T, n_uniform, heavy, seed):
    """8-byte keys: n_uniform uniform values plus, for each (bucket, rows,
    distinct) in heavy, `rows` values inside [T[b], T[b+1]) drawn from
    `distinct` different values (distinct < rows makes runs of equal keys)."""
    rng = np.random.default_rng(seed)
    parts = [rng.integers(0, 2 ** 63, n_uniform, dtype=np.uint64) * np.uint64(2)]
    B = len(T)
    for b, rows, distinct in heavy:
        lo = int(T[b])
        hi = int(T[b + 1]) if b + 1 < B else (1 << 64)
        vals = lo + (rng.random(distinct) * (hi - lo - 1)).astype(np.uint64)
        parts.append(vals[rng.integers(0, distinct, rows)])
    v = rng.permutation(np.concatenate(parts))
    return np.ascontiguousarray(v.astype(">u8").view(np.uint8).reshape(-1, 8))


@pytest.mark.parametrize("case", ["second_chance", "residual", "widespread"])
def test_graph_bucketing_overflow_paths(ck, case):
    """The device-side overflow handling of a captured bucketing sort.  The
    thresholds come from uniform training words; the keys pile up in chosen
    buckets.  second_chance: three buckets beyond the in-LDS capacity but
    within the second chance's -- sorted there, no fallback, no flag.
    residual: one bucket beyond even that -- the gated radix sort runs and
    the flag is raised.  widespread: 80 overflowing buckets (more than the
    second chance takes) -- the gate opens at once.  Every replay gives the
    oracle's order."""
    import torch
    B = 1 << 8
    rng = np.random.default_rng(21)
    train = np.sort(rng.integers(0, 2 ** 63, 1 << 14, dtype=np.uint64) * np.uint64(2))
    T = O.thresholds(train, B)
    heavy = {"second_chance": [(10, 4000, 4000), (100, 3500, 3000), (200, 5000, 4900)],
             "residual": [(50, 12000, 11000), (60, 3000, 3000)],
             "widespread": [(b, 3000, 2900) for b in range(20, 20 + 80 * 2, 2)]}[case]
    rows = concentrated_keys(T, 1 << 15, heavy, 5)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    model = ck.CdfModel(bucket_log2=8, seed=3)
    model.thresholds().copy_(torch.from_numpy(T.view(np.int64)).cuda())
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    # a first build (every bit position): the first compressed word is the key
    spec = {"keys": ck.DeviceKeys.from_numpy(rows), "bitmap": None,
            "opts": dict(method=ck.CKEY_SORT_SPLITTER, model=model, flags=flags)}
    g = ck.RebuildGraph([spec])
    for rep in range(3):
        g.outs[0]["perm"].fill_(-1)
        flags.zero_()
        print(f"overflow graph {case} replay {rep}: n={len(rows)}", flush=True)
        g.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.outs[0]["perm"].cpu().numpy().view(np.uint32), perm)
        np.testing.assert_array_equal(g.outs[0]["bitmap"].cpu().numpy(), d)
        f = int(flags.item())
        assert bool(f & ck.CKEY_FLAG_BUCKET_OVERFLOW) == (case != "second_chance"), f
        assert f & ck.CKEY_FLAG_SPIN_LIMIT == 0
    # the same call without capture takes the host path: same order
    out = ck.ckey_rebuild_index([spec])[0]
    np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm)


def test_autotune(ck, table, tmp_path):
    from paper_2009_11543_amd import tune
    tab, refs = table
    rows = tab["day_id"]
    perm, d = refs["day_id"]
    keys = ck.DeviceKeys.from_numpy(rows)
    cache = str(tmp_path / "tune.json")
    choice, rec = tune.autotune(keys, d, cache_path=cache)
    assert len(rec["times_ms"]) == len(rec["candidates"]) and min(rec["times_ms"]) > 0
    choice2, rec2 = tune.autotune(keys, d, cache_path=cache)  # from the cache
    assert choice2 == choice
    out = ck.ckey_rebuild_index([{"keys": keys, "bitmap": d, "opts": choice}])[0]
    np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm)


@pytest.mark.parametrize("tile", [1, 2])
def test_radix_pass_tiles_exact(ck, table, tile):
    """Both radix pass tiles (1024 and 512 threads) give the oracle's order for
    keys of 1, 2 and 6 words and several digit widths."""
    tab, refs = table
    for name in ("int32_a", "day_id", "title"):
        perm, d = refs[name]
        for db in (5, 8):
            out = ck.ckey_rebuild_index([{"keys": ck.DeviceKeys.from_numpy(tab[name]), "bitmap": None,
                                          "opts": dict(method=ck.CKEY_SORT_RADIX, digit_bits=db, tile=tile)}])[0]
            np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm, err_msg=name)
            np.testing.assert_array_equal(out["bitmap"].cpu().numpy(), d, err_msg=name)


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_bucket_capacity_tiles_exact(ck, table, tile):
    """Every in-LDS bucket capacity (2560, 5120, 10240 rows) gives the oracle's
    order, with both bucketing methods and two bucket counts."""
    from paper_2009_11543_amd import tune
    tab, refs = table
    for name in ("int64", "day_id"):
        perm, d = refs[name]
        spec = {"keys": ck.DeviceKeys.from_numpy(tab[name]), "bitmap": d}
        prev = ck.ckey_rebuild_index([dict(spec, want_ckeys=True)])[0]
        models = tune.fit_models(prev["ckeys"][0].contiguous(), (8, 10), steps=50, batch=1 << 12)
        for b, model in models.items():
            for meth in (ck.CKEY_SORT_SPLITTER, ck.CKEY_SORT_LEARNED):
                out = ck.ckey_rebuild_index([dict(spec, opts=dict(method=meth, model=model, tile=tile))])[0]
                np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm,
                                              err_msg=f"{name} b={b} method={meth}")


def test_autotune_bucket_counts_and_tiles(ck, table):
    """The autotuner over digit widths, pass tiles, bucket counts and bucket
    capacities: its choice rebuilds the index exactly."""
    from paper_2009_11543_amd import tune
    tab, refs = table
    perm, d = refs["int64"]
    keys = ck.DeviceKeys.from_numpy(tab["int64"])
    prev = ck.ckey_rebuild_index([{"keys": keys, "bitmap": d, "want_ckeys": True}])[0]
    models = tune.fit_models(prev["ckeys"][0].contiguous(), (8, 10), steps=50, batch=1 << 12)
    choice, rec = tune.autotune(keys, d, models=models)
    kinds = {(c["method"], c.get("tile"), c.get("bucket_log2")) for c in rec["candidates"]}
    assert (ck.CKEY_SORT_RADIX, 2, None) in kinds and (ck.CKEY_SORT_SPLITTER, 1, 10) in kinds
    assert len(rec["times_ms"]) == len(rec["candidates"]) and min(rec["times_ms"]) > 0
    out = ck.ckey_rebuild_index([{"keys": keys, "bitmap": d, "opts": choice}])[0]
    np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm)

