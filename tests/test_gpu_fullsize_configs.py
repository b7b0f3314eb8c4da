"""Full-size checks of the other configurations: URL-like varchar keys at
2^24 rows (flat bytes + offsets), 32-byte keys at 2^28 rows (uniform, and
2^16 clusters that share a 31-byte stem) and the eight-index table at 2^24
rows rebuilt in one call.  As for the 2^26 DNA keys, the
oracle cannot sort these sizes in test time, so the checks are what holds at
any size plus rows the oracle computes one by one:
  * the first build's permutation is a permutation whose adjacent rows are in
    non-decreasing full-key order, ties by ascending row id (which determines
    it uniquely);
  * its D-bitmap is the union of the adjacent pairs' D positions (Theorem 1's
    definition), computed on the host from the permuted keys;
  * compressed words of sampled rows equal the oracle's;
  * compress + sort with the chosen methods gives the same permutation."""
import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen

pytestmark = pytest.mark.gpu

CHUNK = 1 << 23


@pytest.fixture(scope="module")
def ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11543_amd import ckey
    return ckey


def check_order_and_d(words, perm, d):
    """words: (n, W) big-endian uint64 view of the zero-padded keys."""
    n, W = words.shape
    seen = np.zeros(n, np.bool_)
    seen[perm] = True
    assert seen.all()
    union = np.zeros(64 * W, np.bool_)
    for a in range(0, n - 1, CHUNK):
        b = min(n, a + CHUNK + 1)
        w = words[perm[a:b]]
        lt = np.zeros(b - a - 1, np.bool_)
        eq = np.ones(b - a - 1, np.bool_)
        for j in range(W):
            x, y = w[:-1, j], w[1:, j]
            lt |= eq & (x < y)
            eq &= x == y
        assert np.all(lt | (eq & (perm[a:b - 1] < perm[a + 1:b])))
        x = w[:-1] ^ w[1:]
        nz = x != 0
        first = np.argmax(nz, axis=1)
        has = nz.any(axis=1)
        xv = x[np.arange(len(x)), first][has]
        lead = 63 - np.floor(np.log2(xv.astype(np.float64))).astype(np.int64)
        lead = np.where((xv >> (63 - lead).astype(np.uint64)) == 0, lead + 1, lead)
        union[64 * first[has] + lead] = True
    np.testing.assert_array_equal(d, np.packbits(union)[: len(d)])


def model_for(ck, train_rows, d, bucket_log2):
    import torch
    kt = ck.DeviceKeys(torch.from_numpy(train_rows).cuda())
    ckt, ridt = ck.ckey_compress(kt, d)
    ck.ckey_sort(ckt, ck.ckey_plan_query(d)["nbits"], ridt)
    model = ck.CdfModel(bucket_log2=bucket_log2, seed=3)
    ck.ckey_cdf_fit(model, ckt[0].contiguous(), steps=200, batch=1 << 16)
    return model


def run_config(ck, keys, rows, train_rows, bucket_log2, methods, overflow=None):
    """overflow: method -> whether the bucketing sort must raise
    CKEY_FLAG_BUCKET_OVERFLOW on these keys (its radix fallback ran)."""
    import torch
    first = ck.ckey_rebuild_index([{"keys": keys, "bitmap": None}])[0]
    d = first["bitmap"].cpu().numpy()
    perm = first["perm"].cpu().numpy().view(np.uint32)
    del first
    n, L = rows.shape
    check_order_and_d(rows.view(">u8"), perm, d)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, 4096, replace=False))
    ckd, _ = ck.ckey_compress(keys, d)
    ref = O.compress(O.Keys(np.ascontiguousarray(rows[sample])), d)
    np.testing.assert_array_equal(ck.as_u64(ckd[:, torch.from_numpy(sample).cuda()]), ref)
    del ckd
    model = model_for(ck, train_rows, d, bucket_log2) if methods != ["radix"] else None
    for m in methods:
        opts = {} if m == "radix" else dict(
            method=ck.CKEY_SORT_SPLITTER if m == "splitter" else ck.CKEY_SORT_LEARNED, model=model)
        flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        _, rid = ck.ckey_compress_sort(keys, d, flags=flags, **opts)
        print(f"  {m}: compress_sort n={n}", flush=True)
        np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
        f = int(flags.item())
        assert f & ck.CKEY_FLAG_SPIN_LIMIT == 0
        if overflow and m in overflow:
            assert bool(f & ck.CKEY_FLAG_BUCKET_OVERFLOW) == overflow[m], (m, f)
        del rid
    torch.cuda.empty_cache()


def test_url_varchar_2p24(ck):
    rows, lens = datagen.url_keys(1 << 24, seed=1)
    flat, offs = datagen.pack_varlen(rows, lens)
    keys = ck.DeviceKeys.from_numpy(flat, key_bytes=128, offsets=offs)
    del flat, offs
    train = datagen.url_keys(1 << 20, seed=2)[0]
    run_config(ck, keys, rows, train, 12, ["radix", "splitter", "learned"])


def test_uniform32_2p28(ck):
    import torch
    rows = datagen.uniform_keys(1 << 28, seed=1)
    keys = ck.DeviceKeys(torch.from_numpy(rows).cuda())
    run_config(ck, keys, rows, datagen.uniform_keys(1 << 22, seed=2), 16, ["splitter", "learned"])


def test_cluster32_2p28(ck):
    import torch
    rows = datagen.cluster_keys(1 << 28, seed=1)
    keys = ck.DeviceKeys(torch.from_numpy(rows).cuda())
    # the training rebuild's stems are not the test's: buckets hold a Poisson
    # number of 4096-row clusters, far beyond the in-LDS capacity, so both
    # bucketing methods must finish through the radix fallback and say so
    run_config(ck, keys, rows, datagen.cluster_keys(1 << 22, seed=2), 16, ["radix", "splitter", "learned"],
               overflow={"splitter": True, "learned": True})


def test_table8_2p24_batched(ck):
    """All eight indexes of the 2^24-row table rebuilt in one call (forked
    streams): each index's permutation and D-bitmap by the same checks."""
    import torch
    tab = datagen.table_indexes(1 << 24, seed=1)
    keys = {name: ck.DeviceKeys(torch.from_numpy(rows).cuda()) for name, rows in tab.items()}
    outs = ck.ckey_rebuild_index([{"keys": k, "bitmap": None} for k in keys.values()])
    for (name, rows), out in zip(tab.items(), outs):
        n, L = rows.shape
        W = (L + 7) // 8
        padded = np.zeros((n, 8 * W), np.uint8)
        padded[:, :L] = rows
        perm = out["perm"].cpu().numpy().view(np.uint32)
        d = out["bitmap"].cpu().numpy()
        check_order_and_d(padded.view(">u8"), perm, np.concatenate([d, np.zeros(8 * W - L, np.uint8)]))
