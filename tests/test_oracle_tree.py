"""Pins of the oracle's index tree bulk load (Sec. 5.3): node sizes and
fanouts from the paper's arithmetic, tree shapes by a plain count, the
constructed distinction-bit example's offsets and partial key (Sec. 4.2), and
every field of every node re-derived in Python from the full keys (Python
integers), with inner offsets checked against Lemma 1."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen

FIRST, EQUAL = 0xFFFF, 0xFFFE


def u(b, off, size):
    return int.from_bytes(bytes(b[off:off + size]), "little")


def decode(nodes):
    out = []
    for nd in nodes:
        h = {"high_rid": u(nd, 0, 8), "count": u(nd, 8, 2), "level": u(nd, 10, 2),
             "zero": u(nd, 12, 4), "first": u(nd, 16, 8)}
        ents = []
        if h["level"] == 0:
            h["next"] = u(nd, 24, 8)
            for e in range(h["count"]):
                b = 32 + 16 * e
                ents.append({"pk": u(nd, b, 4), "dpos": u(nd, b + 4, 2), "len": u(nd, b + 6, 2),
                             "rid": u(nd, b + 8, 8)})
            tail = nd[32 + 16 * h["count"]:]
        else:
            for e in range(h["count"]):
                b = 24 + 24 * e
                ents.append({"pk": u(nd, b, 4), "dpos": u(nd, b + 4, 2), "len": u(nd, b + 6, 2),
                             "child": u(nd, b + 8, 8), "rid": u(nd, b + 16, 8)})
            tail = nd[24 + 24 * h["count"]:]
        h["entries"] = ents
        h["tail_zero"] = not tail.any()
        out.append(h)
    return out


def test_paper_fanouts():
    """Sec. 5.3: 256-byte nodes, 24-byte header, 8-byte next pointer, 16-byte
    leaf entries -> 14; 24-byte inner entries -> 9; fill 0.9 -> 12 and 8."""
    assert (256 - 24 - 8) // 16 == 14 and (256 - 24) // 24 == 9
    assert O.tree_fill(0.9) == (math.floor(14 * 0.9), math.floor(9 * 0.9)) == (12, 8)
    assert O.tree_fill(1.0) == (14, 9)


def plain_shape(n, lp, ip):
    if n == 0:
        return []
    lv = [-(-n // lp)]
    while lv[-1] > 1:
        lv.append(-(-lv[-1] // ip))
    return lv


@pytest.mark.parametrize("n", [0, 1, 11, 12, 13, 95, 96, 97, 768, 769, 10 ** 6, 10 ** 7])
@pytest.mark.parametrize("fill", [0.9, 1.0, 0.5, 0.1])
def test_shapes(n, fill):
    lp, ip = O.tree_fill(fill)
    assert O.tree_shape(n, fill) == plain_shape(n, lp, ip)
    assert O.tree_shape(97, 0.9) == [9, 2, 1]


def bits_after(row, L, dpos, pk):
    if dpos == EQUAL:
        return 0
    start = 0 if dpos == FIRST else dpos + 1
    v = int.from_bytes(bytes(row), "big")
    out = 0
    for t in range(pk):
        p = start + t
        if p < 8 * L and (v >> (8 * L - 1 - p)) & 1:
            out |= 1 << (31 - t)
    return out


def dbit(a, b, L):
    x = int.from_bytes(bytes(a), "big") ^ int.from_bytes(bytes(b), "big")
    return EQUAL if x == 0 else 8 * L - x.bit_length()


def check_tree(rows, lens, perm, pk, fill, nodes):
    n, L = rows.shape
    lp, ip = O.tree_fill(fill)
    shape = plain_shape(n, lp, ip)
    assert len(nodes) == sum(shape)
    dec = decode(nodes)
    first = np.cumsum([0] + shape)
    # leaves: chained, in key order, every field from the full keys
    leaves = dec[: shape[0]] if shape else []
    seq = [e for lf in leaves for e in lf["entries"]]
    assert [e["rid"] for e in seq] == list(perm)
    for i, e in enumerate(seq):
        r = perm[i]
        want_d = FIRST if i == 0 else dbit(rows[perm[i - 1]], rows[r], L)
        assert e["dpos"] == want_d
        assert e["pk"] == bits_after(rows[r], L, want_d, pk)
        assert e["len"] == lens[r]
    for j, lf in enumerate(leaves):
        assert lf["level"] == 0 and lf["zero"] == 0 and lf["tail_zero"]
        assert lf["next"] == (j + 1 if j + 1 < shape[0] else 2 ** 64 - 1)
        assert lf["first"] == j * lp and lf["high_rid"] == lf["entries"][-1]["rid"]
        assert lf["count"] == (lp if j + 1 < shape[0] else n - j * lp)
    # inner levels: children consecutive, offsets by Lemma 1 from the level below
    for lvl in range(1, len(shape)):
        nodes_l = dec[first[lvl]: first[lvl + 1]]
        ents = [e for nd in nodes_l for e in nd["entries"]]
        assert [e["child"] for e in ents] == list(range(first[lvl - 1], first[lvl]))
        for c, e in enumerate(ents):
            child = dec[e["child"]]
            assert e["rid"] == child["high_rid"]
            if c == 0:
                assert e["dpos"] == FIRST
            else:
                assert e["dpos"] == min(x["dpos"] for x in child["entries"])   # Lemma 1
                prev = dec[ents[c - 1]["child"]]["high_rid"]
                assert e["dpos"] == dbit(rows[prev], rows[e["rid"]], L)
            assert e["pk"] == bits_after(rows[e["rid"]], L, e["dpos"], pk)
            assert e["len"] == lens[e["rid"]]
        for nd in nodes_l:
            assert nd["level"] == lvl and nd["tail_zero"]
            assert nd["high_rid"] == nd["entries"][-1]["rid"]
    if shape:
        assert shape[-1] == 1


def test_constructed_example(golden_dir):
    with open(os.path.join(golden_dir, "fig_dbit_constructed.json")) as f:
        g = json.load(f)
    rows = np.array([list(bytes.fromhex(h)) for h in g["keys_hex"]], np.uint8)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    nodes = O.bulk_load(k, perm, pk=4, fill=0.9)
    leaf = decode(nodes)[0]
    assert [e["dpos"] for e in leaf["entries"]] == [FIRST] + g["adjacent_dbits"]
    want = int(g["partial_key_key1_pk4"], 2) << 28
    assert leaf["entries"][1]["pk"] == want          # Sec. 4.2: 1010 for key_1, pk = 4
    check_tree(rows, [2] * len(rows), list(perm), 4, 0.9, nodes)


@pytest.mark.parametrize("n,L,pk,fill", [(1, 3, 32, 0.9), (13, 2, 4, 0.9), (97, 4, 16, 0.9),
                                         (800, 3, 32, 1.0), (1500, 5, 7, 0.5), (3000, 2, 32, 0.9)])
def test_fixed_width(n, L, pk, fill):
    rows = datagen.random_small_keys(n, L, n + L, [0, 1, 0x80, 0xFF, 0x41])
    k = O.Keys(rows)
    perm = O.full_sort(k)
    check_tree(rows, [L] * n, list(perm), pk, fill, O.bulk_load(k, perm, pk, fill))


def test_varlen():
    rows = datagen.title_keys(2000, seed=6)
    lens = (rows != 0).sum(axis=1)
    flat, offs = datagen.pack_varlen(rows, lens)
    k = O.Keys(flat, L=48, offsets=offs)
    perm = O.full_sort(k)
    check_tree(rows, list(lens), list(perm), 32, 0.9, O.bulk_load(k, perm, 32, 0.9))


def test_empty():
    k = O.Keys(np.zeros((0, 4), np.uint8))
    assert len(O.bulk_load(k, np.zeros(0, np.uint32))) == 0
