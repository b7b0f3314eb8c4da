"""GPU parity of the index tree bulk load (Sec. 5.3) with the oracle: every
byte of every node, for fixed and variable-length keys, several fill factors
and partial-key lengths, partial-key bits taken from the compressed key, the
reference key or the key itself; and full-size properties at 2^26 keys."""
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


def rebuild(ck, dk, bitmap):
    return ck.ckey_rebuild_index([{"keys": dk, "bitmap": bitmap, "want_pair_pos": True,
                                   "want_ckeys": True}])[0]


def build_tree(ck, dk, bitmap, pk, fill, variant=None, ref=None):
    out = rebuild(ck, dk, bitmap)
    cb = np.full(dk.key_bytes, 0xFF, np.uint8) if bitmap is None else bitmap
    nodes, deref = ck.ckey_bulk_load(dk, out["perm"], out["ckeys"], cb, out.get("pair_pos"), pk=pk,
                                     fill=fill, variant=variant, ref=ref)
    return out, nodes.cpu().numpy(), int(deref.item())


CASES = [  # (n, L, pk, fill, alphabet)
    (1, 3, 32, 0.9, None), (2, 2, 8, 0.9, [0, 1]), (13, 4, 4, 0.9, None), (97, 4, 16, 0.9, None),
    (1500, 6, 32, 0.5, [0, 1, 0x80, 0xFF]), (5000, 8, 32, 1.0, None), (20000, 5, 13, 0.9, [0x41, 0x43]),
    (3000, 16, 32, 0.1, None), (777, 33, 32, 0.9, [7, 9]),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("source", ["first_build", "refresh", "refresh_variant"])
def test_nodes_match_oracle(ck, case, source):
    import torch
    n, L, pk, fill, alphabet = case
    rows = datagen.random_small_keys(n, L, n + L + pk, alphabet)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    want = O.bulk_load(k, perm, pk, fill)
    dk = ck.DeviceKeys.from_numpy(rows)
    d, _ = O.dbits(k, perm)
    bitmap = None if source == "first_build" else d
    variant = ref = None
    if source == "refresh_variant":
        variant = O.variant(k, 0)
        ref = torch.from_numpy(rows[0].copy()).cuda()
    out, nodes, deref = build_tree(ck, dk, bitmap, pk, fill, variant, ref)
    np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm)
    assert nodes.shape == want.shape
    np.testing.assert_array_equal(nodes, want)
    if source == "first_build":
        assert deref == 0   # every position is in the compressed key


def test_varlen_titles(ck):
    import torch
    rows = datagen.title_keys(6000, seed=12)
    lens = (rows != 0).sum(axis=1)
    flat, offs = datagen.pack_varlen(rows, lens)
    k = O.Keys(flat, L=48, offsets=offs)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    dk = ck.DeviceKeys.from_numpy(flat, key_bytes=48, offsets=offs)
    var = O.variant(k, 0)
    ref = torch.from_numpy(rows[0].copy()).cuda()
    _, nodes, deref = build_tree(ck, dk, d, 32, 0.9, var, ref)
    np.testing.assert_array_equal(nodes, O.bulk_load(k, perm, 32, 0.9))
    assert deref > 0    # title keys have variant bits outside D


def test_deref_count(ck):
    """An entry reads its key exactly when one of its partial-key positions is
    variant but outside the compression bitmap."""
    import torch
    rows = datagen.random_small_keys(4000, 6, 5, [0x41, 0x43, 0x47, 0x54])
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    var = O.variant(k, 0)
    _, nodes, deref = build_tree(ck, ck.DeviceKeys.from_numpy(rows), d, 32, 0.9, var,
                                 torch.from_numpy(rows[0].copy()).cuda())
    cls_c = np.unpackbits(var & ~d)
    want = 0
    for nd in nodes:
        cnt, level = int(nd[8:10].view(np.uint16)[0]), int(nd[10:12].view(np.uint16)[0])
        base, esz = (32, 16) if level == 0 else (24, 24)
        for e in range(cnt):
            dp = int(nd[base + esz * e + 4: base + esz * e + 6].view(np.uint16)[0])
            if dp == 0xFFFE:
                continue
            s = 0 if dp == 0xFFFF else dp + 1
            want += int(cls_c[s: min(s + 32, 48)].any())
    assert deref == want


def test_fullsize_dna(ck):
    """2^26 DNA windows, refreshed with D and the variant bitmap: tree shape,
    leaf chain = perm, inner D positions by Lemma 1 checked on the device, and
    4096 sampled leaf entries re-derived from the full keys on the host."""
    import torch
    n = 1 << 26
    rows = datagen.dna_window_keys(n, seed=1)
    dk = ck.DeviceKeys(torch.from_numpy(rows).cuda())
    d = np.full(64, 0x16, np.uint8)   # D of these keys (the 3 distinguishing bits per byte)
    var, ref = ck.ckey_variant_bitmap(dk)
    out, nodes_t, deref = None, None, None
    out = rebuild(ck, dk, d)
    assert (out["bitmap"].cpu().numpy() == d).all()
    nodes_t, deref_t = ck.ckey_bulk_load(dk, out["perm"], out["ckeys"], d, out["pair_pos"], pk=32, fill=0.9,
                                         variant=var.cpu().numpy(), ref=ref)
    shape = ck.ckey_tree_plan(n, 0.9)
    assert nodes_t.shape[0] == shape["total_nodes"] == sum(O.tree_shape(n, 0.9))
    nl = shape["level_nodes"][0]
    leaves = nodes_t[:nl]
    ent = leaves[:, 32:].reshape(nl, 14, 16)
    rid = ent[:, :12, 8:16].contiguous().view(torch.int64).reshape(-1)[:n]
    assert torch.equal(rid.to(torch.int32), out["perm"])
    dpos = ent[:, :12, 4:6].contiguous().view(torch.int16).reshape(-1)[:n].to(torch.int32) & 0xFFFF
    lvl1 = nodes_t[shape["level_first"][1]: shape["level_first"][1] + shape["level_nodes"][1]]
    e1 = lvl1[:, 24:240].reshape(-1, 9, 24)[:, :8].reshape(-1, 24)[:nl]
    d1 = e1[:, 4:6].contiguous().view(torch.int16).reshape(-1).to(torch.int32) & 0xFFFF
    pad = torch.full((nl * 12 - n,), 0xFFFE, dtype=torch.int32, device=dpos.device)
    mins = torch.cat([dpos, pad]).reshape(nl, 12).min(dim=1).values
    assert int(d1[0]) == 0xFFFF
    assert torch.equal(d1[1:], mins[1:])
    # sampled leaf entries against the full keys
    rng = np.random.default_rng(0)
    perm = out["perm"].cpu().numpy()
    pos = rng.integers(1, n, 4096)
    e = ent.reshape(-1, 16)[(pos // 12) * 14 + pos % 12].cpu().numpy()
    for q, i in enumerate(pos):
        a, b = rows[perm[i - 1]], rows[perm[i]]
        x = int.from_bytes(a.tobytes(), "big") ^ int.from_bytes(b.tobytes(), "big")
        dp = 0xFFFE if x == 0 else 512 - x.bit_length()
        assert int(e[q, 4:6].view(np.uint16)[0]) == dp
        if dp != 0xFFFE:
            v = int.from_bytes(b.tobytes(), "big")
            want = 0
            for t in range(32):
                p = dp + 1 + t
                if p < 512 and (v >> (511 - p)) & 1:
                    want |= 1 << (31 - t)
            assert int(e[q, 0:4].view(np.uint32)[0]) == want
        assert int(e[q, 8:16].view(np.uint64)[0]) == perm[i]
    assert int(deref_t.item()) > 0   # the last bit of each byte is variant, not D
