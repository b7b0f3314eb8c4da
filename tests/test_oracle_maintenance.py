"""Pins of the oracle's DS-metadata maintenance (Sec. 4.3) against the plain
definitions: D of the grown key set by sorting (Python ``sorted``, Python
integers), the variant bitmap by a direct OR, Lemma 1, and a constructed
example meeting the paper's statements on inserts and deletes."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen


def as_int(row):
    return int.from_bytes(bytes(row), "big")


def true_d(rows, L):
    """D by definition: sort with Python, D-bit of each adjacent distinct pair."""
    srt = sorted(bytes(r) for r in rows)
    out = set()
    for a, b in zip(srt, srt[1:]):
        x = int.from_bytes(a, "big") ^ int.from_bytes(b, "big")
        if x:
            out.add(8 * L - x.bit_length())
    return out


def positions_of(bm):
    L = len(bm)
    v = as_int(bm)
    return {p for p in range(8 * L) if (v >> (8 * L - 1 - p)) & 1}


def bitmap_of(positions, L):
    bm = np.zeros(L, np.uint8)
    for p in positions:
        bm[p >> 3] |= 0x80 >> (p & 7)
    return bm


def variant_direct(rows, ref):
    v = 0
    for r in rows:
        v |= as_int(r) ^ as_int(ref)
    return v


def split_case(seed, n_old, n_new, L, alphabet=None):
    rows = datagen.random_small_keys(n_old + n_new, L, seed, alphabet)
    k = O.Keys(rows)
    old = np.arange(n_old, dtype=np.uint32)
    order = old[np.argsort([bytes(r) for r in rows[:n_old]], kind="stable")] if n_old else old
    ins = np.arange(n_old, n_old + n_new, dtype=np.uint32)
    return rows, k, order, ins


@pytest.mark.parametrize("seed", range(8))
def test_inserts_only_keep_d_exact(seed):
    """Sec. 4.3: with inserts only, the D-bitmap stays exactly D."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 5))
    n_old, n_new = int(rng.integers(0, 300)), int(rng.integers(1, 300))
    alphabet = None if seed % 2 else rng.integers(0, 256, 3)
    rows, k, order, ins = split_case(seed, n_old, n_new, L, alphabet)
    d0 = bitmap_of(true_d(rows[:n_old], L), L)
    d1, _ = O.insert(k, order, ins, d0)
    assert positions_of(d1) == true_d(rows, L)


@pytest.mark.parametrize("seed", range(4))
def test_inserts_from_empty_build_d(seed):
    """Inserting every key, in a random sequence, into an empty index gives D."""
    rng = np.random.default_rng(100 + seed)
    rows = datagen.random_small_keys(400, 3, seed, [0, 1, 0x40, 0x41, 0xFF])
    k = O.Keys(rows)
    ins = rng.permutation(len(rows)).astype(np.uint32)
    d, v = O.insert(k, np.zeros(0, np.uint32), ins, np.zeros(3, np.uint8), np.zeros(3, np.uint8), ref_row=5)
    assert positions_of(d) == true_d(rows, 3)
    assert as_int(v) == variant_direct(rows, rows[5])


@pytest.mark.parametrize("seed", range(4))
def test_variant_after_inserts(seed):
    rows, k, order, ins = split_case(seed, 150, 90, 4)
    ref = 3
    v0 = O.variant(O.Keys(rows[:150]), ref)
    _, v1 = O.insert(k, order, ins, np.zeros(4, np.uint8), v0, ref_row=ref)
    assert as_int(v1) == variant_direct(rows, rows[ref])
    assert (v1 == O.variant(k, ref)).all()


@pytest.mark.parametrize("seed", range(4))
def test_deletes_leave_a_superset(seed):
    """Sec. 4.3: after deletes the unchanged bitmaps still cover D and the
    variant positions (Lemma 1), and later inserts keep that true."""
    rng = np.random.default_rng(200 + seed)
    rows, k, order, ins = split_case(seed, 200, 100, 3, [0, 7, 0x80, 0x81])
    d0 = bitmap_of(true_d(rows[:200], 3), 3)
    d1, _ = O.insert(k, order, ins, d0)
    keep = rng.random(len(rows)) < 0.5
    live = rows[keep]
    assert true_d(live, 3) <= positions_of(d1)
    # insert the deleted keys back, into the shrunken index
    live_idx = np.nonzero(keep)[0].astype(np.uint32)
    live_order = live_idx[np.argsort([bytes(r) for r in live], kind="stable")]
    back = np.nonzero(~keep)[0].astype(np.uint32)
    d2, _ = O.insert(k, live_order, back, d1)
    assert positions_of(d2) >= true_d(rows, 3)
    assert positions_of(d2) == positions_of(d1) | true_d(rows, 3)


def test_varlen_inserts():
    strs = [b"AB", b"ABA", b"B", b"", b"ABAB", b"A", b"ABB", b"BA"]
    flat = np.frombuffer(b"".join(strs), np.uint8)
    offs = np.cumsum([0] + [len(s) for s in strs]).astype(np.uint64)
    k = O.Keys(flat, L=6, offsets=offs)
    padded = [s + b"\0" * (6 - len(s)) for s in strs]
    order = np.array(sorted(range(4), key=lambda i: padded[i]), np.uint32)
    d0 = bitmap_of(true_d([np.frombuffer(padded[i], np.uint8) for i in range(4)], 6), 6)
    d1, _ = O.insert(k, order, np.arange(4, 8, dtype=np.uint32), d0)
    assert positions_of(d1) == true_d([np.frombuffer(p, np.uint8) for p in padded], 6)


def test_constructed_maintenance_example(golden_dir):
    with open(os.path.join(golden_dir, "maintenance_constructed.json")) as f:
        g = json.load(f)
    rows = np.array([list(bytes.fromhex(h)) for h in g["keys_hex"]], np.uint8)
    L = g["key_bytes"]
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    assert d.tobytes().hex().upper() == g["dbitmap_hex"]
    assert O.variant(k, 0).tobytes().hex().upper() == g["variant_bitmap_hex"]
    # deleting key_3, then key_0: the true D and variant positions shrink as the
    # paper says, while the kept bitmaps still cover them
    for drop, want in (([3], g["after_delete_key3"]), ([3, 0], g["after_delete_key3_key0"])):
        live = np.delete(rows, drop, axis=0)
        assert true_d(live, L) == set(want["true_dbits"]) <= positions_of(d)
        ref = live[0]
        var = variant_direct(live, ref)
        assert {p for p in range(8 * L) if (var >> (8 * L - 1 - p)) & 1} == set(want["variant_positions"])
    # insert between the named neighbours: sets the larger of the two D-bits
    ins = g["insert"]
    allrows = np.vstack([rows, np.array([list(bytes.fromhex(ins["key_hex"]))], np.uint8)])
    k2 = O.Keys(allrows)
    a = g["keys_hex"].index(ins["between"][0])
    b = g["keys_hex"].index(ins["between"][1])
    assert O.dbit_pair(k2, a, 6) == ins["dbit_a_k"] and O.dbit_pair(k2, 6, b) == ins["dbit_k_b"]
    d2, _ = O.insert(k2, perm, np.array([6], np.uint32), d)
    assert d2.tobytes().hex().upper() == ins["dbitmap_after_hex"]
    assert positions_of(d2) == true_d(allrows, L)
