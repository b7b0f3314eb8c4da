"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and its host-only logic (planning, argument checks, workspace
queries) behaves as documented."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ckey_\w+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def ck():
    from paper_2009_11543_amd import ckey
    return ckey


def test_exports_every_declared_symbol(ck):
    names = declared_symbols()
    assert {"ckey_distinction_bits", "ckey_compress", "ckey_sort", "ckey_rebuild_index"} <= names
    lib = ctypes.CDLL(ck.LIB_PATH)
    for name in sorted(names):
        assert hasattr(lib, name), name


def test_every_declared_symbol_is_typed_on_each_load(ck):
    # An untyped ctypes call passes Python ints as C int: a device pointer
    # would be cut to 32 bits.  Every load must declare every signature.
    for lib in (ck.lib(), ck._load()):
        for name in sorted(declared_symbols()):
            f = getattr(lib, name)
            assert f.argtypes is not None, name
            assert f.restype is not None, name


def test_status_strings(ck):
    assert ck.status_string(0) == "ok"
    assert "workspace" in ck.status_string(3)


def test_plan_query_table3(ck, golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table3_indbtab_dbitmap.json")))
    bm = np.array([int(b, 2) for b in g["bytes_1_to_35"]], np.uint8)
    plan = ck.ckey_plan_query(bm)
    assert plan["nbits"] == 56 and plan["words"] == 1
    w = g["windows_sec51_rule"]
    assert [s for s, _ in plan["windows"]] == w["start_bytes_0based"]
    assert [format(m, "016x") for _, m in plan["windows"]] == w["masks_hex"]


@pytest.mark.parametrize("seed", range(20))
def test_plan_query_matches_oracle(ck, seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 300))
    bm = (rng.random(L) < rng.random()).astype(np.uint8) * rng.integers(0, 256, L, dtype=np.uint8)
    plan = ck.ckey_plan_query(bm)
    st, mk = O.windows(bm)
    assert plan["nbits"] == len(O.doffset(bm))
    assert plan["words"] == O.nwords(bm)
    assert [s for s, _ in plan["windows"]] == list(st)
    assert [m for _, m in plan["windows"]] == [int(x) for x in mk]


def test_argument_errors(ck):
    lib = ck.lib()
    need = ctypes.c_size_t(0)
    # null keys
    assert lib.ckey_compress(None, None, None, 1, None, None, None) == ck.CKEY_ERR_INVALID
    ks = ck.ckey_keys(None, None, 0, 0, 0)
    assert lib.ckey_distinction_bits(ctypes.byref(ks), None, None, None, None,
                                     ctypes.byref(need), None) == ck.CKEY_ERR_INVALID
    ks = ck.ckey_keys(None, None, 10, 16, 8)   # stride < key_bytes, bytes NULL
    assert lib.ckey_distinction_bits(ctypes.byref(ks), None, None, None, None,
                                     ctypes.byref(need), None) == ck.CKEY_ERR_INVALID
    ks = ck.ckey_keys(None, None, 4, 4, 4)   # real call (workspace given) with a null bitmap
    assert lib.ckey_distinction_bits(ctypes.byref(ks), None, None, None, ctypes.c_void_p(256),
                                     ctypes.byref(ctypes.c_size_t(256)), None) == ck.CKEY_ERR_INVALID
    ks = ck.ckey_keys(None, None, 0, ck.MAX_KEY_BYTES + 1, ck.MAX_KEY_BYTES + 1)
    bm = np.zeros(4, np.uint8)
    assert lib.ckey_distinction_bits(ctypes.byref(ks), None, bm.ctypes.data, None, None,
                                     ctypes.byref(need), None) == ck.CKEY_ERR_UNSUPPORTED
    o = ck.ckey_sort_opts(0, 9, 0, 0, None, None)   # digit width 9
    assert lib.ckey_sort(None, 1, 8, None, 0, ctypes.byref(o), None, ctypes.byref(need),
                         None) == ck.CKEY_ERR_INVALID
    o = ck.ckey_sort_opts(0, 8, 0, 0, None, None)
    assert lib.ckey_sort(None, 1, 65, None, 0, ctypes.byref(o), None, ctypes.byref(need),
                         None) == ck.CKEY_ERR_INVALID   # nbits > 64*words
    assert lib.ckey_sort(None, 1, 8, None, (1 << 30) + 1, ctypes.byref(o), None,
                         ctypes.byref(need), None) == ck.CKEY_ERR_UNSUPPORTED
    # compress: words below the plan's w
    keys = np.zeros((4, 16), np.uint8)
    ks = ck.ckey_keys(keys.ctypes.data, None, 4, 16, 16)
    full = np.full(16, 0xFF, np.uint8)
    assert lib.ckey_compress(ctypes.byref(ks), full.ctypes.data, keys.ctypes.data, 1, None, None,
                             None) == ck.CKEY_ERR_INVALID


def test_workspace_queries(ck):
    n = 1 << 20
    a = ck.ckey_sort_workspace(1, 40, n)
    b = ck.ckey_sort_workspace(3, 192, n)
    assert a >= n * 12 and b >= n * 28 and b > a
    lib = ck.lib()
    need = ctypes.c_size_t(0)
    ks = ck.ckey_keys(1, None, n, 64, 64)  # pointer never dereferenced by a query
    d = ck.ckey_index_desc(ks, None, 1, 1, None, None, None)
    assert lib.ckey_rebuild_index(ctypes.byref(d), 1, None, None, ctypes.byref(need), None) == 0
    assert need.value >= n * (64 + 4)  # first build: 8 words of ckeys + ping-pong
    small = ctypes.c_size_t(16)
    assert lib.ckey_rebuild_index(ctypes.byref(d), 1, None, ctypes.c_void_p(256),
                                  ctypes.byref(small), None) == ck.CKEY_ERR_WORKSPACE


def test_fused_table_queries_and_limits(ck):
    """The one-launch table rebuild: workspace query on the host, and its
    documented limits (indexes, key bytes, passes, method) refused up front."""
    lib = ck.lib()
    n = 1 << 20
    fused = ck.ckey_sort_opts(0, 8, 0, 0, None, None, 1)
    need = ctypes.c_size_t(0)

    def query(descs, opts=fused):
        arr = (ck.ckey_index_desc * len(descs))(*descs)
        need.value = 0
        return lib.ckey_rebuild_index(arr, len(descs), ctypes.byref(opts), None, ctypes.byref(need), None)

    def desc(L, rows=n, bitmap=None, opts=None):
        ks = ck.ckey_keys(1, None, rows, L, L)  # pointers never dereferenced by a query
        return ck.ckey_index_desc(ks, bitmap, 1, 1, None, None, None, opts)

    assert query([desc(16)]) == ck.CKEY_OK
    # first build of 16-byte keys: two 2-word ping-pong copies + row ids + two look-back arrays
    tiles = -(-n // 4096)
    assert need.value >= n * (2 * 16 + 4) + 2 * tiles * 1024
    one = need.value
    assert query([desc(16)] * 8) == ck.CKEY_OK and need.value >= 8 * (one - 4096)
    assert query([desc(16)] * 9) == ck.CKEY_ERR_UNSUPPORTED
    assert query([desc(65)]) == ck.CKEY_ERR_UNSUPPORTED
    assert query([desc(64)]) == ck.CKEY_OK  # 512 bits, 64 passes of 8 bits
    d1 = ck.ckey_sort_opts(0, 1, 0, 0, None, None, 0)
    assert query([desc(16, opts=ctypes.pointer(d1))]) == ck.CKEY_ERR_UNSUPPORTED  # 128 passes
    bm = np.zeros(16, np.uint8)
    bm[3] = 0x0F  # |D| = 4: four 1-bit passes
    assert query([desc(16, bitmap=bm.ctypes.data, opts=ctypes.pointer(d1))]) == ck.CKEY_OK
    lrn = ck.ckey_sort_opts(2, 0, 8, 0, 1, None, 0)
    assert query([desc(16, opts=ctypes.pointer(lrn))]) == ck.CKEY_ERR_UNSUPPORTED
    assert query([desc(16, rows=1 << 30)]) == ck.CKEY_ERR_UNSUPPORTED
    # the forked form's layout differs; graph creation checks the fused size
    assert query([desc(16)], ck.ckey_sort_opts(0, 8, 0, 0, None, None, 0)) == ck.CKEY_OK
    g = ctypes.c_void_p()
    arr = (ck.ckey_index_desc * 1)(desc(16))
    assert lib.ckey_graph_create(arr, 1, ctypes.byref(fused), ctypes.c_void_p(256), one - 1,
                                 ctypes.byref(g)) == ck.CKEY_ERR_WORKSPACE


def test_maintenance_argument_errors_and_queries(ck):
    lib = ck.lib()
    need = ctypes.c_size_t(0)
    ia = ck.ckey_keys(1, None, 100, 16, 16)
    ba = ck.ckey_keys(1, None, 10, 8, 8)   # key widths differ
    assert lib.ckey_insert_keys(ctypes.byref(ia), None, ctypes.byref(ba), None, None, None, None,
                                None, None, ctypes.byref(need), None) == ck.CKEY_ERR_INVALID
    bb = ck.ckey_keys(1, None, 1000, 16, 16)
    assert lib.ckey_insert_keys(ctypes.byref(ia), None, ctypes.byref(bb), ctypes.c_void_p(256), None,
                                None, None, None, None, ctypes.byref(need), None) == 0
    given = need.value
    assert given >= 1000 * 4  # places of the batch keys
    assert lib.ckey_insert_keys(ctypes.byref(ia), None, ctypes.byref(bb), None, None, None, None,
                                None, None, ctypes.byref(need), None) == 0
    assert need.value >= given + 1000 * (16 + 4)  # plus the batch's own full-key sort
    # real call without the D-bitmap, or with a variant bitmap but no reference
    ws = ctypes.c_void_p(256)
    big = ctypes.c_size_t(1 << 40)
    assert lib.ckey_insert_keys(ctypes.byref(ia), None, ctypes.byref(bb), None, None, None, None,
                                None, ws, ctypes.byref(big), None) == ck.CKEY_ERR_INVALID
    assert lib.ckey_insert_keys(ctypes.byref(ia), None, ctypes.byref(bb), None, ctypes.c_void_p(512),
                                ctypes.c_void_p(768), None, None, ws, ctypes.byref(big),
                                None) == ck.CKEY_ERR_INVALID
    assert lib.ckey_variant_bitmap(ctypes.byref(ia), None, None, None, None, None, ctypes.byref(need),
                                   None) == 0 and need.value >= 16
    assert lib.ckey_variant_bitmap(ctypes.byref(ia), None, None, None, None, ws, ctypes.byref(big),
                                   None) == ck.CKEY_ERR_INVALID   # no output bitmap
    small = ctypes.c_size_t(1)
    assert lib.ckey_variant_bitmap(ctypes.byref(ia), None, ctypes.c_void_p(512), None, None, ws,
                                   ctypes.byref(small), None) == ck.CKEY_ERR_WORKSPACE


def test_sort_noalloc_checks_before_any_gpu_call(ck):
    """ckey_sort_noalloc validates everything on the host before it touches the
    GPU: a sort whose workspace exceeds the static scratch array, a bucketing
    method, skip_trivial and more than 512 passes are refused as unsupported;
    bad words, digit widths and null pointers as invalid."""
    lib = ck.lib()
    U = ck.CKEY_ERR_UNSUPPORTED
    call = lambda o, words, nbits, n: lib.ckey_sort_noalloc(None, words, nbits, None, n, ctypes.byref(o), None)
    assert ck.ckey_sort_workspace(1, 60, 6_000_000) > ck.NOALLOC_SCRATCH_BYTES
    assert call(ck._opts(), 1, 60, 6_000_000) == U
    assert call(ck._opts(), 3, 192, 2_500_000) == U
    assert call(ck._opts(method=ck.CKEY_SORT_SPLITTER, bucket_log2=10), 1, 60, 100) == U
    assert call(ck._opts(method=ck.CKEY_SORT_LEARNED, bucket_log2=10), 1, 60, 100) == U
    assert call(ck._opts(skip_trivial=True), 1, 60, 100) == U
    assert call(ck._opts(digit_bits=1), 9, 576, 100) == U          # 576 one-bit passes
    assert call(ck._opts(), 1, 60, (1 << 30) + 1) == U                 # beyond CKEY_MAX_ROWS
    assert call(ck._opts(), 0, 0, 100) == ck.CKEY_ERR_INVALID
    assert call(ck._opts(), 1, 65, 100) == ck.CKEY_ERR_INVALID
    assert call(ck._opts(digit_bits=9), 1, 60, 100) == ck.CKEY_ERR_INVALID
    assert call(ck._opts(), 1, 60, 100) == ck.CKEY_ERR_INVALID      # null key and row-id pointers


def test_tile_option_checked(ck):
    """ckey_sort_opts.tile: radix 0..2, bucketing 0..3; anything else invalid
    (checked by the workspace query, before any GPU call)."""
    need = ctypes.c_size_t(0)
    def query(**kw):
        o = ck._opts(**kw)
        return ck.lib().ckey_sort(None, 1, 60, None, 1000, ctypes.byref(o), None, ctypes.byref(need), None)
    assert query(tile=2) == ck.CKEY_OK
    assert query(tile=3) == ck.CKEY_ERR_INVALID
    assert query(method=ck.CKEY_SORT_SPLITTER, bucket_log2=10, tile=3) == ck.CKEY_OK
    assert query(method=ck.CKEY_SORT_SPLITTER, bucket_log2=10, tile=4) == ck.CKEY_ERR_INVALID
    # the half pass tile doubles the radix sort's tile count, not its buffers
    full = ck.ckey_sort_workspace(1, 60, 1 << 20, tile=1)
    half = ck.ckey_sort_workspace(1, 60, 1 << 20, tile=2)
    assert full <= half < full + (1 << 20)

