"""The host baseline (PEXT compression of Sec. 5.1 and the row-column sort of
Appendix A) against the oracle: the same compressed words and the full-key
order, for thread counts and cache sizes that exercise every phase (many
sub-blocks per init block, t > 1, empty split blocks, duplicates)."""
import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen, rowcol


CASES = [  # (n, L, threads, cache_bytes, alphabet)
    (0, 4, 4, 1 << 20, None), (1, 4, 4, 1 << 20, None), (2, 3, 2, 64, [0, 1]),
    (1000, 4, 1, 1 << 20, None), (1000, 4, 3, 160, None), (5000, 8, 8, 320, [0, 1, 0x80]),
    (20000, 16, 4, 4096, None), (30001, 6, 7, 1000, [0x41, 0x43, 0x47, 0x54]),
    (12345, 40, 5, 777, [0x61, 0x62, 0x63]), (4096, 64, 16, 2048, [0x41, 0x43, 0x47, 0x54]),
]


@pytest.mark.parametrize("case", CASES)
def test_matches_oracle(case):
    n, L, p, cache, alphabet = case
    rows = datagen.random_small_keys(n, L, n + L + p, alphabet)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm) if n else (np.zeros(L, np.uint8), 0)
    bm = d if d.any() else np.full(L, 0xFF, np.uint8)
    got, ck, t = rowcol.compress_sort(rows, bm, threads=p, cache_bytes=cache, want_ckeys=True)
    np.testing.assert_array_equal(got, perm)
    if n:
        np.testing.assert_array_equal(ck, O.compress(k, bm)[:, perm])


def test_superset_bitmap_and_dna():
    rows = datagen.dna_window_keys(20000, seed=3, seq_len=1 << 16)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    for bm in (np.full(64, 0x16, np.uint8), np.full(64, 0x17, np.uint8)):
        got, _, _ = rowcol.compress_sort(rows, bm, threads=6, cache_bytes=5000)
        np.testing.assert_array_equal(got, perm)


def test_stride_wider_than_key():
    rows = datagen.random_small_keys(3000, 12, 9, [1, 2, 3])
    k = O.Keys(rows, L=10)
    perm = O.full_sort(k)
    got, _, _ = rowcol.compress_sort(rows, np.full(10, 0xFF, np.uint8), threads=4, cache_bytes=999)
    np.testing.assert_array_equal(got, perm)


def test_rejects_bad_words():
    with pytest.raises(ValueError):
        rowcol.compress_sort(np.zeros((4, 80), np.uint8), np.full(80, 0xFF, np.uint8))  # 640 bits: > 8 words


@pytest.mark.parametrize("case", CASES)
def test_gnu_parallel_sorts_match_oracle(case):
    """The GCC parallel-mode baselines: compressed records and full keys give
    the oracle's full-key order (ties by record ID)."""
    n, L, p, _, alphabet = case
    rows = datagen.random_small_keys(n, L, n + L + p, alphabet)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm) if n else (np.zeros(L, np.uint8), 0)
    bm = d if d.any() else np.full(L, 0xFF, np.uint8)
    got, ck, _ = rowcol.gnu_compress_sort(rows, bm, threads=p, want_ckeys=True)
    np.testing.assert_array_equal(got, perm)
    if n:
        np.testing.assert_array_equal(ck, O.compress(k, bm)[:, perm])
    full, _ = rowcol.gnu_full_sort(rows, L, threads=p)
    np.testing.assert_array_equal(full, perm)
