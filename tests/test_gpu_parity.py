"""GPU parity: libckey.so (through its C ABI) against the CPU oracle.

Every comparison is bit-exact: D-bitmaps, compressed words, permutations and
per-pair D positions.  Sizes span several 4096-key sort tiles plus ragged
tails; edge cases cover empty, single-row, all-equal and unsorted inputs,
supersets of D and variable-length keys.
"""
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


def dev_keys(ck, rows=None, flat=None, offsets=None, L=None, stride_pad=0):
    if rows is not None:
        if stride_pad:
            rows = np.concatenate([rows, np.full((rows.shape[0], stride_pad), 0xEE, np.uint8)], 1)
        return ck.DeviceKeys.from_numpy(rows, key_bytes=L)
    return ck.DeviceKeys.from_numpy(flat, key_bytes=L, offsets=offsets)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


# ----------------------------------------------------------------- D bits --

@pytest.mark.parametrize("n,L,seed", [(2, 1, 0), (1000, 3, 1), (9000, 16, 2), (20000, 37, 3),
                                      (5000, 64, 4), (3, 2048, 5)])
def test_distinction_bits(ck, n, L, seed):
    rows = datagen.random_small_keys(n, L, seed, [0x00, 0x41, 0x43, 0x47, 0x54, 0xFF])
    k = O.Keys(rows)
    perm = O.full_sort(k)
    ref, _ = O.dbits(k, perm)
    import torch
    dk = dev_keys(ck, rows)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    order = torch.from_numpy(perm.view(np.int32)).cuda()
    got = ck.ckey_distinction_bits(dk, order=order, flags=flags)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    assert int(flags.item()) & ck.CKEY_FLAG_DESCENDING == 0
    # physically sorted copy, no order array
    dks = dev_keys(ck, np.ascontiguousarray(rows[perm]))
    got2 = ck.ckey_distinction_bits(dks)
    np.testing.assert_array_equal(got2.cpu().numpy(), ref)


def test_distinction_bits_unsorted_flag(ck):
    import torch
    rows = np.array([[1, 2], [1, 1], [3, 0]], np.uint8)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_distinction_bits(dev_keys(ck, rows), flags=flags)
    assert int(flags.item()) & ck.CKEY_FLAG_DESCENDING


def test_distinction_bits_stride_and_varlen(ck):
    rng = np.random.default_rng(9)
    n, L = 3000, 13
    lens = rng.integers(1, L + 1, n)
    rows = rng.choice(np.frombuffer(b"ab\x01", np.uint8), (n, L))
    rows[np.arange(L)[None, :] >= lens[:, None]] = 0
    flat, offs = datagen.pack_varlen(rows, lens)
    kv = O.Keys(flat, L=L, offsets=offs)
    perm = O.full_sort(kv)
    ref, _ = O.dbits(kv, perm)
    import torch
    order = torch.from_numpy(perm.view(np.int32)).cuda()
    got = ck.ckey_distinction_bits(dev_keys(ck, flat=flat, offsets=offs, L=L), order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    # fixed width with junk bytes past key_bytes in a wider stride (odd stride 16)
    got = ck.ckey_distinction_bits(dev_keys(ck, rows, L=L, stride_pad=3), order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)


@pytest.mark.parametrize("L,pad", [(37, 11), (64, 0), (100, 12)])
def test_distinction_bits_wide_aligned_rows(ck, L, pad):
    """16-byte aligned rows (16 bytes of both keys per step), key lengths that
    end inside a 16-byte chunk, junk bytes past the key in the stride."""
    import torch
    n = 20000
    rows = datagen.random_small_keys(n, L, L + pad, [0x41, 0x43, 0x47, 0x54])
    rows[:, : L // 3] = 0x41  # long shared prefixes: the first difference lies late
    k = O.Keys(rows)
    perm = O.full_sort(k)
    ref, _ = O.dbits(k, perm)
    order = torch.from_numpy(perm.view(np.int32)).cuda()
    got = ck.ckey_distinction_bits(dev_keys(ck, rows, L=L, stride_pad=pad), order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)


@pytest.mark.parametrize("L,maxlen", [(64, 64), (120, 100)])
def test_distinction_bits_long_byte_keys(ck, L, maxlen):
    """Byte-addressed keys (variable length, and fixed width at an odd stride)
    with long shared prefixes, so that the first difference lies several
    16-byte steps in; keys end inside a step, and the last keys sit next to
    the end of the byte buffer, where the comparison goes word by word."""
    import torch
    rng = np.random.default_rng(L)
    n = 6000
    lens = rng.integers(1, maxlen + 1, n)
    rows = rng.choice(np.frombuffer(b"ab", np.uint8), (n, L))
    rows[:, : L // 2] = 0x41
    rows[np.arange(L)[None, :] >= lens[:, None]] = 0
    flat, offs = datagen.pack_varlen(rows, lens)
    kv = O.Keys(flat, L=L, offsets=offs)
    perm = O.full_sort(kv)
    ref, _ = O.dbits(kv, perm)
    order = torch.from_numpy(perm.view(np.int32)).cuda()
    got = ck.ckey_distinction_bits(dev_keys(ck, flat=flat, offsets=offs, L=L), order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    got = ck.ckey_distinction_bits(dev_keys(ck, rows, L=L, stride_pad=3), order=order)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)


# --------------------------------------------------------------- compress --

def bitmaps_for(rows, seed):
    k = O.Keys(rows)
    L = rows.shape[1]
    d, _ = O.dbits(k, O.full_sort(k))
    rng = np.random.default_rng(seed)
    return [d, np.full(L, 0xFF, np.uint8), d | rng.integers(0, 256, L, dtype=np.uint8),
            O.variant(k, 0), np.zeros(L, np.uint8)]


@pytest.mark.parametrize("n,L,seed,pad", [(1, 8, 0, 0), (4097, 16, 1, 0), (10000, 64, 2, 0),
                                          (3000, 35, 3, 0), (2500, 20, 4, 12), (700, 130, 5, 2),
                                          (257, 512, 6, 0)])
def test_compress(ck, n, L, seed, pad):
    rows = datagen.random_small_keys(n, L, seed, [0x41, 0x43, 0x47, 0x54] if seed % 2 else None)
    k = O.Keys(rows)
    dk = dev_keys(ck, rows, L=L, stride_pad=pad)
    for bm in bitmaps_for(rows, seed):
        ref = O.compress(k, bm)
        got, rid = ck.ckey_compress(dk, bm)
        np.testing.assert_array_equal(ck.as_u64(got), ref)
        np.testing.assert_array_equal(u32(rid), np.arange(n, dtype=np.uint32))
        # extra words are zero-filled
        got2, _ = ck.ckey_compress(dk, bm, words=ref.shape[0] + 2)
        g2 = ck.as_u64(got2)
        np.testing.assert_array_equal(g2[: ref.shape[0]], ref)
        assert not g2[ref.shape[0]:].any()


def test_compress_table3_windows_shape(ck, golden_dir):
    import json
    import os
    g = json.load(open(os.path.join(golden_dir, "table3_indbtab_dbitmap.json")))
    bm = np.array([int(b, 2) for b in g["bytes_1_to_35"]], np.uint8)
    rows = datagen.random_small_keys(5000, 35, 11)
    ref = O.compress(O.Keys(rows), bm)
    got, _ = ck.ckey_compress(dev_keys(ck, rows), bm)
    np.testing.assert_array_equal(ck.as_u64(got), ref)
    assert ref.shape[0] == 1


def test_compress_varlen(ck):
    rng = np.random.default_rng(12)
    n, L = 5000, 40
    lens = rng.integers(0, L + 1, n)
    rows = rng.choice(np.frombuffer(b"Ab z", np.uint8), (n, L))
    rows[np.arange(L)[None, :] >= lens[:, None]] = 0
    flat, offs = datagen.pack_varlen(rows, lens)
    kv = O.Keys(flat, L=L, offsets=offs)
    dk = dev_keys(ck, flat=flat, offsets=offs, L=L)
    for bm in bitmaps_for(rows, 12):
        np.testing.assert_array_equal(ck.as_u64(ck.ckey_compress(dk, bm)[0]), O.compress(kv, bm))


def test_compress_key_too_long_flag(ck):
    import torch
    flat = np.frombuffer(b"abcdefgh", np.uint8)
    offs = np.array([0, 2, 8], np.uint64)
    dk = dev_keys(ck, flat=flat, offsets=offs, L=4)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_compress(dk, np.full(4, 0xFF, np.uint8), flags=flags)
    assert int(flags.item()) & ck.CKEY_FLAG_KEY_TOO_LONG


# ------------------------------------------------------------------- sort --

@pytest.mark.parametrize("n,w,nbits,seed", [(0, 1, 8, 0), (1, 1, 8, 0), (2, 1, 3, 1),
                                            (4096, 1, 40, 2), (4097, 1, 41, 3),
                                            (50000, 3, 192, 4), (12345, 2, 70, 5),
                                            (30000, 1, 1, 6), (70001, 1, 64, 7),
                                            (9000, 4, 256, 8), (20000, 5, 300, 9),
                                            (7001, 6, 350, 10), (5000, 7, 420, 11),
                                            (12345, 8, 512, 12), (3000, 9, 560, 13)])
def test_sort_radix(ck, n, w, nbits, seed):
    import torch
    rng = np.random.default_rng(seed)
    # few distinct values per word to force many ties and skewed digits
    vals = rng.integers(0, 2 ** 63, 64, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    ckh = vals[rng.integers(0, 64, (w, n))] if n else np.zeros((w, 0), np.uint64)
    # clear bits past nbits (they are zero in real compressed keys)
    for kk in range(w):
        have = min(64, max(0, nbits - 64 * kk))
        mask = np.uint64(0) if have == 0 else np.uint64(((1 << have) - 1) << (64 - have))
        ckh[kk] &= mask
    ref = O.csort(ckh) if n else np.zeros(0, np.uint32)
    ckd = torch.from_numpy(ckh.view(np.int64)).cuda()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, nbits, rid, flags=flags)
    np.testing.assert_array_equal(u32(rid), ref)
    np.testing.assert_array_equal(ck.as_u64(ckd), ckh[:, ref])
    assert int(flags.item()) == 0


@pytest.mark.parametrize("digit_bits", [1, 5, 7])
def test_sort_digit_widths(ck, digit_bits):
    import torch
    rng = np.random.default_rng(digit_bits)
    n = 20000
    ckh = (rng.integers(0, 1 << 20, (2, n), dtype=np.uint64) << np.uint64(44))
    ref = O.csort(ckh)
    ckd = torch.from_numpy(ckh.view(np.int64)).cuda()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, 84, rid, digit_bits=digit_bits)
    np.testing.assert_array_equal(u32(rid), ref)


@pytest.mark.parametrize("n", [1, 5000, 70001])
def test_sort_skip_trivial_passes(ck, n):
    """skip_trivial drops exactly the passes whose digit is equal for every
    row (here the 6 constant leading bytes of 16-byte keys, sorted over all
    128 bits, and the zero low byte of every word) and keeps the order."""
    import ctypes
    import torch
    rows = datagen.random_small_keys(n, 16, 11, None)
    rows[:, :6] = np.frombuffer(b"\x07\x00\x41\xff\x10\x02", np.uint8)
    rows[:, 15] = 0
    k = O.Keys(rows)
    ref = O.full_sort(k)
    bm = np.full(16, 0xFF, np.uint8)
    lib = ck._lib
    outs, launches = [], []
    for skip in (False, True):
        ckd, rid = ck.ckey_compress(dev_keys(ck, rows), bm)
        lib.ckey_profile_reset()
        lib.ckey_profile_enable(1)
        ck.ckey_sort(ckd, 128, rid, skip_trivial=skip)
        torch.cuda.synchronize()
        ms, c = ctypes.c_double(), ctypes.c_uint64()
        lib.ckey_profile_read(b"onesweep", ctypes.byref(ms), ctypes.byref(c))
        lib.ckey_profile_enable(0)
        launches.append(int(c.value))
        outs.append((u32(rid).copy(), ck.as_u64(ckd).copy()))
    for r, c in outs:
        np.testing.assert_array_equal(r, ref)
        np.testing.assert_array_equal(c, O.compress(k, bm)[:, ref])
    if n > 1:
        assert launches == [16, 9]
    else:
        assert launches == [0, 0]


# ---------------------------------------------------------------- rebuild --

def check_rebuild(ck, k, dk, bm, want_ck=True):
    perm_ref = O.full_sort(k)
    d_true, _ = O.dbits(k, perm_ref)
    out = ck.ckey_rebuild_index([{"keys": dk, "bitmap": bm, "want_pair_pos": True,
                                  "want_ckeys": want_ck}])[0]
    np.testing.assert_array_equal(u32(out["perm"]), perm_ref)
    np.testing.assert_array_equal(out["bitmap"].cpu().numpy(), d_true)
    bm_used = np.full(k.L, 0xFF, np.uint8) if bm is None else bm
    ckr = O.compress(k, bm_used)
    _, pos_ref = O.refine(ckr, perm_ref, bm_used)
    if k.n > 1:
        np.testing.assert_array_equal(u32(out["pair_pos"]), pos_ref)
    if want_ck:
        np.testing.assert_array_equal(ck.as_u64(out["ckeys"]), ckr[:, perm_ref])
    return d_true


@pytest.mark.parametrize("n,L,seed", [(0, 4, 0), (1, 4, 0), (2, 4, 1), (5000, 8, 2),
                                      (20000, 64, 3), (12289, 35, 4)])
def test_rebuild_first_and_refresh(ck, n, L, seed):
    alphabet = [0x41, 0x43, 0x47, 0x54] if seed % 2 else [0, 1, 0x80, 0xFF, 7]
    rows = datagen.random_small_keys(n, L, seed, alphabet)
    k = O.Keys(rows)
    dk = dev_keys(ck, rows)
    d_true = check_rebuild(ck, k, dk, None)
    rng = np.random.default_rng(seed)
    for bm in [d_true, d_true | rng.integers(0, 256, L, dtype=np.uint8), O.variant(k, 0)]:
        check_rebuild(ck, k, dk, bm)


def test_rebuild_all_equal_keys(ck):
    rows = np.full((9000, 12), 0x5A, np.uint8)
    k = O.Keys(rows)
    out = ck.ckey_rebuild_index([{"keys": dev_keys(ck, rows), "bitmap": None,
                                  "want_pair_pos": True}])[0]
    np.testing.assert_array_equal(u32(out["perm"]), np.arange(9000, dtype=np.uint32))
    assert not out["bitmap"].cpu().numpy().any()
    assert (u32(out["pair_pos"]) == 0xFFFFFFFF).all()
    # an empty bitmap is a valid superset of the (empty) D
    check_rebuild(ck, k, dev_keys(ck, rows), np.zeros(12, np.uint8))


def test_rebuild_varlen(ck):
    rng = np.random.default_rng(21)
    n, L = 8000, 24
    lens = rng.integers(1, L, n)
    rows = rng.choice(np.frombuffer(b"abc", np.uint8), (n, L))
    rows[np.arange(L)[None, :] >= lens[:, None]] = 0
    flat, offs = datagen.pack_varlen(rows, lens)
    k = O.Keys(flat, L=L, offsets=offs)
    dk = dev_keys(ck, flat=flat, offsets=offs, L=L)
    d_true = check_rebuild(ck, k, dk, None)
    check_rebuild(ck, k, dk, d_true)


def test_rebuild_batch_of_indexes(ck):
    specs, refs = [], []
    for x, (n, L) in enumerate([(3000, 8), (5000, 4), (4100, 12), (100, 48)]):
        rows = datagen.random_small_keys(n, L, 30 + x)
        k = O.Keys(rows)
        perm = O.full_sort(k)
        d, _ = O.dbits(k, perm)
        specs.append({"keys": dev_keys(ck, rows), "bitmap": d if x % 2 else None})
        refs.append((perm, d))
    outs = ck.ckey_rebuild_index(specs)
    for o, (perm, d) in zip(outs, refs):
        np.testing.assert_array_equal(u32(o["perm"]), perm)
        np.testing.assert_array_equal(o["bitmap"].cpu().numpy(), d)


# ------------------------------------------------------ paper workloads --

def test_uniform_prefix_2p20(ck):
    """16-byte keys, 6-byte constant prefix, 2^20 rows: full oracle parity."""
    rows = datagen.uniform_prefix_keys(1 << 20, seed=1)
    k = O.Keys(rows)
    dk = dev_keys(ck, rows)
    d_true = check_rebuild(ck, k, dk, None, want_ck=False)
    assert 30 <= int(np.unpackbits(d_true).sum()) <= 64
    check_rebuild(ck, k, dk, d_true)


def test_dna_windows_2p18(ck):
    rows = datagen.dna_window_keys(1 << 18, seed=1, seq_len=1 << 19)
    k = O.Keys(rows)
    dk = dev_keys(ck, rows)
    d_true = check_rebuild(ck, k, dk, None, want_ck=False)
    check_rebuild(ck, k, dk, d_true)
