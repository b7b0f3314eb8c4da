"""GPU parity of the DS-metadata maintenance calls (Sec. 4.3) against the
oracle: the variant bitmap (OR of key xor reference) and batched inserts into
the D-bitmap and variant bitmap, bit-exact, over fixed and variable-length
keys, aligned and unaligned strides, empty and single-key sets; plus
full-size properties."""
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


def host(t):
    return t.cpu().numpy()


def fixed_case(seed, n, L, stride, alphabet=None):
    rows = datagen.random_small_keys(n, stride, seed, alphabet)
    return rows, O.Keys(rows, L=L)


def dev_keys(ck, rows, L):
    import torch
    if rows.shape[0] == 0:
        return ck.DeviceKeys(torch.zeros((0, rows.shape[1]), dtype=torch.uint8, device="cuda"), L)
    return ck.DeviceKeys.from_numpy(rows, key_bytes=L)


VARIANT_CASES = [  # (n, L, stride)
    (1, 5, 5), (2, 1, 1), (300, 3, 3), (1000, 16, 16), (4097, 16, 32), (3000, 13, 16),
    (2500, 20, 20), (2049, 7, 9), (5000, 64, 64), (700, 100, 112), (64, 300, 300),
]


@pytest.mark.parametrize("case", VARIANT_CASES)
def test_variant_fixed(ck, case):
    n, L, stride = case
    rows, k = fixed_case(n * 7 + L, n, L, stride, None if n % 2 else [0x41, 0x43, 0x47, 0x54])
    var, ref = ck.ckey_variant_bitmap(dev_keys(ck, rows, L))
    np.testing.assert_array_equal(host(var), O.variant(k, 0))
    np.testing.assert_array_equal(host(ref), rows[0, :L])


def test_variant_given_reference_and_empty(ck):
    import torch
    rows, k = fixed_case(5, 800, 24, 24)
    ref = torch.from_numpy(rows[417, :24].copy()).cuda()
    var, ref_out = ck.ckey_variant_bitmap(dev_keys(ck, rows, 24), ref=ref)
    np.testing.assert_array_equal(host(var), O.variant(k, 417))
    np.testing.assert_array_equal(host(ref_out), rows[417, :24])
    var, ref_out = ck.ckey_variant_bitmap(dev_keys(ck, rows[:0], 24))
    assert not host(var).any() and not host(ref_out).any()


def test_variant_varlen(ck):
    rows = datagen.title_keys(5000, seed=4)
    lens = (rows != 0).sum(axis=1)
    flat, offs = datagen.pack_varlen(rows, lens)
    k = O.Keys(flat, L=48, offsets=offs)
    dk = ck.DeviceKeys.from_numpy(flat, key_bytes=48, offsets=offs)
    var, ref = ck.ckey_variant_bitmap(dk)
    np.testing.assert_array_equal(host(var), O.variant(k, 0))
    np.testing.assert_array_equal(host(ref), rows[0])


def sorted_order(rows, L):
    return np.array(sorted(range(len(rows)), key=lambda i: (bytes(rows[i, :L]), i)), np.uint32)


INSERT_CASES = [  # (n_index, n_batch, L, stride, alphabet)
    (0, 1, 4, 4, None), (0, 300, 3, 3, [0, 1, 0x80]), (1, 1, 2, 2, None), (1, 50, 5, 8, None),
    (2000, 1, 8, 8, None), (3000, 700, 4, 4, [0, 1, 2, 0xF0]), (5000, 3000, 16, 16, None),
    (4000, 2500, 13, 16, [0x41, 0x43, 0x47, 0x54]), (2500, 2500, 7, 7, [0, 0xFF]),
    (6000, 1200, 64, 64, [0x41, 0x43, 0x47, 0x54]),
]


@pytest.mark.parametrize("case", INSERT_CASES)
@pytest.mark.parametrize("sort_inside", [True, False])
def test_insert_matches_oracle(ck, case, sort_inside):
    import torch
    ni, nb, L, stride, alphabet = case
    seed = ni * 3 + nb + L
    allrows = datagen.random_small_keys(ni + nb, stride, seed, alphabet)
    if ni > 10:  # batch keys equal to index keys, and repeats inside the batch
        allrows[ni: ni + nb // 4] = allrows[: nb // 4]
        allrows[ni + nb // 2: ni + nb // 2 + nb // 8] = allrows[ni: ni + nb // 8]
    k = O.Keys(allrows, L=L)
    idx_rows, bat_rows = allrows[:ni], allrows[ni:]
    iorder = sorted_order(idx_rows, L)
    d_index, _ = O.dbits(O.Keys(idx_rows, L=L), iorder) if ni else (np.zeros(L, np.uint8), 0)
    rng = np.random.default_rng(seed)
    extra = rng.integers(0, 256, L, dtype=np.uint8) & rng.integers(0, 256, L, dtype=np.uint8) \
        & rng.integers(0, 256, L, dtype=np.uint8)
    d_old = d_index | extra       # a superset of the index's D, as DS-metadata is
    ref_row = 0
    v_old = O.variant(k, ref_row) & rng.integers(0, 256, L, dtype=np.uint8)
    want_d, want_v = O.insert(k, iorder, np.arange(ni, ni + nb, dtype=np.uint32), d_old, v_old,
                              ref_row=ref_row)
    dbm = torch.from_numpy(d_old.copy()).cuda()
    vbm = torch.from_numpy(v_old.copy()).cuda()
    ref = torch.from_numpy(allrows[ref_row, :L].copy()).cuda()
    border = None
    if not sort_inside:
        border = torch.from_numpy(sorted_order(bat_rows, L).view(np.int32)).cuda()
    ck.ckey_insert_keys(dev_keys(ck, idx_rows, L), torch.from_numpy(iorder.view(np.int32)).cuda(),
                        dev_keys(ck, bat_rows, L), dbm, variant=vbm, ref=ref, batch_order=border)
    np.testing.assert_array_equal(host(dbm), want_d)
    np.testing.assert_array_equal(host(vbm), want_v)


def test_insert_index_stored_in_order_and_varlen(ck):
    import torch
    rows = datagen.title_keys(3000, seed=9)
    srt = rows[sorted_order(rows, 48)]
    idx_rows, bat_rows = srt[::2].copy(), rows[1::2].copy()
    allrows = np.vstack([idx_rows, bat_rows])
    lens = (allrows != 0).sum(axis=1)
    flat, offs = datagen.pack_varlen(allrows, lens)
    k = O.Keys(flat, L=48, offsets=offs)
    ni = len(idx_rows)
    iorder = np.arange(ni, dtype=np.uint32)
    d_old, _ = O.dbits(O.Keys(idx_rows), None)
    want_d, _ = O.insert(k, iorder, np.arange(ni, len(allrows), dtype=np.uint32), d_old)
    fi, oi = datagen.pack_varlen(idx_rows, lens[:ni])
    fb, ob = datagen.pack_varlen(bat_rows, lens[ni:])
    dbm = torch.from_numpy(d_old.copy()).cuda()
    ck.ckey_insert_keys(ck.DeviceKeys.from_numpy(fi, key_bytes=48, offsets=oi), None,
                        ck.DeviceKeys.from_numpy(fb, key_bytes=48, offsets=ob), dbm)
    np.testing.assert_array_equal(host(dbm), want_d)


def test_fullsize_variant_dna(ck):
    """2^26 DNA windows: every byte position takes all four bases, so the
    variant bitmap is the OR of their pairwise xors in every byte: 0x17 (A=0x41,
    C=0x43, G=0x47, T=0x54).  D is 0x16 per byte: the last bit separates A from
    T but never first -- the variant bitmap is a strict superset of D."""
    import torch
    rows = datagen.dna_window_keys(1 << 26, seed=1)
    dk = ck.DeviceKeys(torch.from_numpy(rows).cuda())
    var, ref = ck.ckey_variant_bitmap(dk)
    assert (host(var) == 0x17).all()
    np.testing.assert_array_equal(host(ref), rows[0])


def test_fullsize_insert_property(ck):
    """2^22-row DNA index plus a 2^14-row batch from another seed: the batched
    insert gives D(index) | D(index + batch), with both D's from first builds."""
    import torch
    ni, nb = 1 << 22, 1 << 14
    idx_rows = datagen.dna_window_keys(ni, seed=1)
    bat_rows = datagen.dna_window_keys(nb, seed=5)
    both = np.vstack([idx_rows, bat_rows])
    outs = ck.ckey_rebuild_index([{"keys": ck.DeviceKeys(torch.from_numpy(idx_rows).cuda()), "bitmap": None},
                                  {"keys": ck.DeviceKeys(torch.from_numpy(both).cuda()), "bitmap": None}])
    d_index, d_union = host(outs[0]["bitmap"]), host(outs[1]["bitmap"])
    dbm = torch.from_numpy(d_index.copy()).cuda()
    ck.ckey_insert_keys(ck.DeviceKeys(torch.from_numpy(idx_rows).cuda()), outs[0]["perm"],
                        ck.DeviceKeys(torch.from_numpy(bat_rows).cuda()), dbm)
    np.testing.assert_array_equal(host(dbm), d_index | d_union)
