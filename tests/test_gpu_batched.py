"""GPU tests of the batched table rebuild: all indexes of one table (uneven key
widths, duplicates, var-length-like titles) rebuilt by one call on forked
streams, the same rebuild captured in a HIP graph and replayed, and the
autotuner -- every result compared bit-exactly with the oracle."""
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
    specs = specs_for(ck, tab, refs, first_build_every=1 << 30)  # refreshes but index 0
    models = []
    for x, (name, rows) in enumerate(tab.items()):
        if x % 3 == 2:
            continue  # stays radix
        prev = ck.ckey_rebuild_index([dict(specs[x], want_ckeys=True)])[0]
        model = ck.CdfModel(bucket_log2=8, seed=3)
        ck.ckey_cdf_fit(model, prev["ckeys"][0].contiguous(), steps=50, batch=1 << 12)
        models.append(model)
        specs[x]["opts"] = dict(method=ck.CKEY_SORT_SPLITTER if x % 3 == 0 else ck.CKEY_SORT_LEARNED,
                                model=model)
    check(ck, tab, refs, ck.ckey_rebuild_index(specs))
    torch.cuda.synchronize()


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


def test_graph_rejects_bucketing(ck, table):
    tab, refs = table
    model = ck.CdfModel(bucket_log2=8)
    with pytest.raises(ck.CkeyError):
        ck.RebuildGraph(specs_for(ck, tab, refs)[:1], method=ck.CKEY_SORT_SPLITTER, model=model)


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
