"""The Zipf(s, n, m) generator of Sec. 6 against its definition and Table 4:
key layout, letter frequencies, the table's size arithmetic, and where the
distinction bits of such keys can lie (oracle, small n)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen


def test_table4_transcription(golden_dir):
    with open(os.path.join(golden_dir, "table4_zipf.json")) as f:
        g = json.load(f)
    assert [tuple(r[:6]) for r in g["rows"]] == [tuple(r) for r in datagen.ZIPF_TABLE4]
    for ds, s, L, m, full, comp, skr, wcr in g["rows"]:
        assert full == L + 8            # full key plus an 8-byte record ID
        assert round(full / comp, 2) == skr
        assert comp % 8 == 0 and 1.0 <= wcr <= 2.0


@pytest.mark.parametrize("s,L,m", [(2.5, 48, 0), (1.5, 40, 3), (1.5, 64, 5), (1.5, 20, 7), (2.5, 13, 2)])
def test_layout(s, L, m):
    rows = datagen.zipf_keys(3000, s, L, m, seed=4)
    assert rows.shape == (3000, L)
    pos = np.arange(L)
    fixed = rows[:, pos % 8 < m]
    letters = rows[:, pos % 8 >= m]
    if fixed.size:
        assert (fixed == fixed[0, 0]).all() and 0x21 <= fixed[0, 0] <= 0x7E
    assert ((letters >= ord("a")) & (letters <= ord("z"))).all()


@pytest.mark.parametrize("s", [1.5, 2.5])
def test_letter_frequencies(s):
    rows = datagen.zipf_keys(40000, s, 64, 0, seed=7)
    cnt = np.bincount(rows.reshape(-1) - ord("a"), minlength=26)
    N = cnt.sum()
    p = np.arange(1, 27, dtype=np.float64) ** -s
    p /= p.sum()
    sd = np.sqrt(N * p * (1 - p))
    assert (np.abs(cnt - N * p) <= 5 * sd + 1).all()
    assert cnt[0] == cnt.max()          # 'a' is the most frequent letter


@pytest.mark.parametrize("s,L,m", [(2.5, 48, 0), (1.5, 40, 2), (1.5, 64, 5)])
def test_dbits_only_in_letter_bits(s, L, m):
    """Letters a..z differ only in their low five bits (positions 3..7 of a
    byte) and the fixed bytes never differ, so D lies in those positions."""
    rows = datagen.zipf_keys(20000, s, L, m, seed=2)
    k = O.Keys(rows)
    d, desc = O.dbits(k, O.full_sort(k))
    assert not desc
    allowed = np.zeros(L, np.uint8)
    allowed[np.arange(L) % 8 >= m] = 0x1F
    assert ((d & ~allowed) == 0).all()
    assert d.any()
