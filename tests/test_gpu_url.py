"""GPU parity on the URL-like varchar workload (keys of 20-120 bytes over
[a-z0-9./], zero-padded to 128, passed as flat bytes + offsets): D, the
compressed words, the permutation of every sort method and the rebuild's
refreshed bitmap against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen

pytestmark = pytest.mark.gpu

L = 128


@pytest.fixture(scope="module")
def ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11543_amd import ckey
    return ckey


@pytest.fixture(scope="module")
def url16(ck):
    rows, lens = datagen.url_keys(1 << 16, seed=1)
    flat, offs = datagen.pack_varlen(rows, lens)
    k = O.Keys(flat, L=L, offsets=offs)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    dk = ck.DeviceKeys.from_numpy(flat, key_bytes=L, offsets=offs)
    return rows, lens, k, perm, d, dk


def test_url_dbits_and_compress(ck, url16):
    import torch
    rows, lens, k, perm, d, dk = url16
    order = torch.from_numpy(perm.view(np.int32)).cuda()
    got = ck.ckey_distinction_bits(dk, order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), d)
    ckd, rid = ck.ckey_compress(dk, d)
    np.testing.assert_array_equal(ck.as_u64(ckd), O.compress(k, d))
    np.testing.assert_array_equal(rid.cpu().numpy(), np.arange(k.n, dtype=np.int32))


@pytest.mark.parametrize("method", ["radix", "splitter", "learned"])
def test_url_compress_sort(ck, url16, method):
    import torch
    rows, lens, k, perm, d, dk = url16
    opts = {}
    if method != "radix":
        # model fitted to a training rebuild of another seed, compressed with d
        rt, lt = datagen.url_keys(1 << 15, seed=2)
        ft, ot = datagen.pack_varlen(rt, lt)
        kt = ck.DeviceKeys.from_numpy(ft, key_bytes=L, offsets=ot)
        ckt, ridt = ck.ckey_compress(kt, d)
        ck.ckey_sort(ckt, ck.ckey_plan_query(d)["nbits"], ridt)
        model = ck.CdfModel(bucket_log2=8, seed=1)
        ck.ckey_cdf_fit(model, ckt[0].contiguous(), steps=100, batch=4096)
        opts = dict(method=ck.CKEY_SORT_SPLITTER if method == "splitter" else ck.CKEY_SORT_LEARNED,
                    model=model)
    ckd, rid = ck.ckey_compress_sort(dk, d, **opts)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), O.compress(k, d)[:, perm])


def test_url_rebuild(ck, url16):
    rows, lens, k, perm, d, dk = url16
    first = ck.ckey_rebuild_index([{"keys": dk, "bitmap": None}])[0]
    np.testing.assert_array_equal(first["perm"].cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(first["bitmap"].cpu().numpy(), d)
    again = ck.ckey_rebuild_index([{"keys": dk, "bitmap": d}])[0]
    np.testing.assert_array_equal(again["perm"].cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(again["bitmap"].cpu().numpy(), d)
