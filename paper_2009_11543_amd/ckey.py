"""Python binding of libckey.so (declared in include/ckey.h).

Argument marshalling only: torch tensors supply device memory
(``data_ptr()``) and ``torch.cuda.current_stream()`` supplies the stream;
every step runs in the library's HIP kernels.  Importing this module fails
if the library has not been built (``python -m paper_2009_11543_amd.build``).
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libckey.so")

CKEY_OK, CKEY_ERR_INVALID, CKEY_ERR_UNSUPPORTED, CKEY_ERR_WORKSPACE, CKEY_ERR_HIP = range(5)
CKEY_FLAG_DESCENDING = 0x1
CKEY_FLAG_KEY_TOO_LONG = 0x2
CKEY_FLAG_SPIN_LIMIT = 0x4
CKEY_FLAG_BUCKET_OVERFLOW = 0x8
CKEY_SORT_RADIX, CKEY_SORT_LEARNED, CKEY_SORT_SPLITTER = 0, 1, 2
MAX_KEY_BYTES = 2048
TABLE_MAX_INDEXES, TABLE_MAX_KEY_BYTES, TABLE_MAX_PASSES = 8, 64, 64  # one-launch table rebuild


class CkeyError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn}: {status_string(status)} (status {status})")


class ckey_keys(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("key_bytes", ctypes.c_uint32), ("stride", ctypes.c_uint32)]


class ckey_sort_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_uint32), ("digit_bits", ctypes.c_uint32),
                ("bucket_log2", ctypes.c_uint32), ("skip_trivial", ctypes.c_uint32),
                ("model", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("fused_table", ctypes.c_uint32), ("tile", ctypes.c_uint32)]


class ckey_index_desc(ctypes.Structure):
    _fields_ = [("keys", ckey_keys), ("bitmap_in", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("bitmap_out", ctypes.c_void_p), ("pair_pos", ctypes.c_void_p),
                ("ckeys", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("opts", ctypes.POINTER(ckey_sort_opts))]


class ckey_tree_shape(ctypes.Structure):
    _fields_ = [("height", ctypes.c_uint32), ("leaf_entries", ctypes.c_uint32),
                ("inner_entries", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("level_nodes", ctypes.c_uint64 * 32), ("level_first", ctypes.c_uint64 * 32),
                ("total_nodes", ctypes.c_uint64)]


class ckey_tree_input(ctypes.Structure):
    _fields_ = [("keys", ckey_keys), ("perm", ctypes.c_void_p), ("ckeys", ctypes.c_void_p),
                ("words", ctypes.c_uint32), ("cbitmap", ctypes.c_void_p), ("pair_pos", ctypes.c_void_p),
                ("variant", ctypes.c_void_p), ("ref", ctypes.c_void_p)]


class ckey_cdf_train_opts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_11543_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, SZP = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t)
    lib.ckey_status_string.argtypes = [ctypes.c_int]
    lib.ckey_status_string.restype = ctypes.c_char_p
    lib.ckey_plan_query.argtypes = [P, U32, P, P, P, P, P, U32]
    lib.ckey_distinction_bits.argtypes = [ctypes.POINTER(ckey_keys), P, P, P, P, SZP, P]
    lib.ckey_compress.argtypes = [ctypes.POINTER(ckey_keys), P, P, U32, P, P, P]
    lib.ckey_sort.argtypes = [P, U32, U32, P, U64, ctypes.POINTER(ckey_sort_opts), P, SZP, P]
    lib.ckey_sort_noalloc.argtypes = [P, U32, U32, P, U64, ctypes.POINTER(ckey_sort_opts), P]
    lib.ckey_rebuild_index.argtypes = [ctypes.POINTER(ckey_index_desc), U32,
                                       ctypes.POINTER(ckey_sort_opts), P, SZP, P]
    lib.ckey_compress_sort.argtypes = [ctypes.POINTER(ckey_keys), P, P, U32, P,
                                       ctypes.POINTER(ckey_sort_opts), P, SZP, P]
    lib.ckey_graph_create.argtypes = [ctypes.POINTER(ckey_index_desc), U32,
                                      ctypes.POINTER(ckey_sort_opts), P, ctypes.c_size_t,
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.ckey_graph_launch.argtypes = [P, P]
    lib.ckey_graph_destroy.argtypes = [P]
    lib.ckey_tune_index.argtypes = [ctypes.POINTER(ckey_index_desc), ctypes.POINTER(ckey_sort_opts),
                                    U32, P, ctypes.c_size_t, P, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_float)]
    lib.ckey_variant_bitmap.argtypes = [ctypes.POINTER(ckey_keys), P, P, P, P, P, SZP, P]
    lib.ckey_insert_keys.argtypes = [ctypes.POINTER(ckey_keys), P, ctypes.POINTER(ckey_keys), P, P, P, P,
                                     P, P, SZP, P]
    lib.ckey_tree_plan.argtypes = [U64, ctypes.c_float, ctypes.POINTER(ckey_tree_shape)]
    lib.ckey_bulk_load.argtypes = [ctypes.POINTER(ckey_tree_input), U32, ctypes.c_float, P, P, P, SZP, P]
    lib.ckey_cdf_model_bytes.argtypes = [U32]
    lib.ckey_cdf_model_bytes.restype = ctypes.c_size_t
    lib.ckey_cdf_model_init.argtypes = [P, U32, U64, P]
    lib.ckey_cdf_fit.argtypes = [P, U32, P, U64, ctypes.POINTER(ckey_cdf_train_opts), P, P, SZP, P]
    lib.ckey_cdf_grad.argtypes = [P, P, P, U64, P, P, P, SZP, P]
    lib.ckey_cdf_bucket.argtypes = [P, U32, U32, P, U64, P, P, P, P]
    lib.ckey_profile_enable.argtypes = [ctypes.c_int]
    lib.ckey_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.ckey_profile_reset.argtypes = []
    lib.ckey_bench_copy.argtypes = [P, P, ctypes.c_size_t, P]
    for fn in ("ckey_plan_query", "ckey_distinction_bits", "ckey_compress", "ckey_sort", "ckey_sort_noalloc",
               "ckey_rebuild_index", "ckey_compress_sort", "ckey_graph_create", "ckey_graph_launch",
               "ckey_graph_destroy", "ckey_tune_index", "ckey_variant_bitmap", "ckey_insert_keys", "ckey_tree_plan", "ckey_bulk_load", "ckey_cdf_model_init", "ckey_cdf_fit",
               "ckey_cdf_grad", "ckey_cdf_bucket", "ckey_profile_enable", "ckey_profile_read",
               "ckey_profile_reset", "ckey_bench_copy"):
        getattr(lib, fn).restype = ctypes.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def status_string(s):
    return _lib.ckey_status_string(int(s)).decode()


def _check(fn, status):
    if status != CKEY_OK:
        raise CkeyError(fn, status)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host_bitmap(bitmap):
    a = np.ascontiguousarray(np.asarray(bitmap, dtype=np.uint8))
    return a, a.ctypes.data_as(ctypes.c_void_p)


class DeviceKeys:
    """Keys resident on the GPU.

    Fixed width: ``data`` is a uint8 tensor of shape (n, stride) whose first
    ``key_bytes`` bytes per row are the key.  Variable length: ``data`` is a
    flat uint8 tensor and ``offsets`` an int64 tensor of n+1 byte offsets.
    """

    def __init__(self, data, key_bytes=None, offsets=None):
        assert data.dtype == torch.uint8 and data.is_cuda and data.is_contiguous()
        self.data = data
        self.offsets = offsets
        if offsets is None:
            assert data.dim() == 2
            self.n = data.shape[0]
            self.stride = data.shape[1]
            self.key_bytes = self.stride if key_bytes is None else key_bytes
        else:
            assert offsets.dtype == torch.int64 and offsets.is_cuda and key_bytes is not None
            self.n = offsets.numel() - 1
            self.stride = 0
            self.key_bytes = key_bytes

    @classmethod
    def from_numpy(cls, arr, key_bytes=None, offsets=None, device="cuda"):
        data = torch.from_numpy(np.ascontiguousarray(arr)).to(device)
        off = None if offsets is None else torch.from_numpy(np.asarray(offsets, np.int64)).to(device)
        return cls(data, key_bytes, off)

    def c_struct(self):
        return ckey_keys(self.data.data_ptr() if self.n else None,
                         None if self.offsets is None else self.offsets.data_ptr(),
                         self.n, self.key_bytes, self.stride)


def _workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def ckey_plan_query(bitmap):
    """Host-only plan: dict(nbits, words, windows=[(start_byte, mask), ...])."""
    bm, p = _host_bitmap(bitmap)
    nb, w, nw = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check("ckey_plan_query", _lib.ckey_plan_query(p, len(bm), ctypes.byref(nb), ctypes.byref(w),
                                                   ctypes.byref(nw), None, None, 0))
    st = np.zeros(max(nw.value, 1), np.uint32)
    mk = np.zeros(max(nw.value, 1), np.uint64)
    _check("ckey_plan_query", _lib.ckey_plan_query(p, len(bm), None, None, None, st.ctypes.data,
                                                   mk.ctypes.data, nw.value))
    return {"nbits": nb.value, "words": w.value,
            "windows": [(int(s), int(m)) for s, m in zip(st[: nw.value], mk[: nw.value])]}


def ckey_distinction_bits(keys, order=None, flags=None, stream=None):
    """D-bitmap (uint8 tensor of key_bytes bytes on the device) of the keys taken
    in ``order`` (int32 tensor of row ids) or in row order."""
    ks = keys.c_struct()
    need = ctypes.c_size_t(0)
    _check("ckey_distinction_bits", _lib.ckey_distinction_bits(
        ctypes.byref(ks), _ptr(order), None, None, None, ctypes.byref(need), None))
    ws = _workspace(need.value, keys.data.device)
    bm = torch.empty(keys.key_bytes, dtype=torch.uint8, device=keys.data.device)
    _check("ckey_distinction_bits", _lib.ckey_distinction_bits(
        ctypes.byref(ks), _ptr(order), _ptr(bm), _ptr(flags), _ptr(ws), ctypes.byref(need),
        _stream(stream)))
    return bm


def ckey_variant_bitmap(keys, ref=None, flags=None, stream=None):
    """(variant bitmap, reference key): two uint8 device tensors of key_bytes
    bytes.  ``ref``: device uint8 tensor, or None for key 0 (Sec. 4.3)."""
    ks = keys.c_struct()
    need = ctypes.c_size_t(0)
    _check("ckey_variant_bitmap", _lib.ckey_variant_bitmap(ctypes.byref(ks), None, None, None, None,
                                                           None, ctypes.byref(need), None))
    dev = keys.data.device
    ws = _workspace(need.value, dev)
    var = torch.empty(keys.key_bytes, dtype=torch.uint8, device=dev)
    ref_out = torch.empty(keys.key_bytes, dtype=torch.uint8, device=dev)
    _check("ckey_variant_bitmap", _lib.ckey_variant_bitmap(
        ctypes.byref(ks), _ptr(ref), _ptr(var), _ptr(ref_out), _ptr(flags), _ptr(ws),
        ctypes.byref(need), _stream(stream)))
    return var, ref_out


def ckey_insert_keys(index, index_order, batch, dbitmap, variant=None, ref=None, batch_order=None,
                     flags=None, stream=None):
    """DS-metadata update for inserting ``batch`` into ``index`` (Sec. 4.3):
    ``dbitmap`` (and ``variant``, with ``ref``) -- device uint8 tensors of
    key_bytes bytes -- are updated in place.  ``index_order``/``batch_order``:
    int32 device tensors of row ids in key order, or None (stored in key order
    / sort the batch inside)."""
    ik, bk = index.c_struct(), batch.c_struct()
    need = ctypes.c_size_t(0)
    _check("ckey_insert_keys", _lib.ckey_insert_keys(
        ctypes.byref(ik), None, ctypes.byref(bk), _ptr(batch_order), None, None, None, None, None,
        ctypes.byref(need), None))
    ws = _workspace(need.value, dbitmap.device)
    _check("ckey_insert_keys", _lib.ckey_insert_keys(
        ctypes.byref(ik), _ptr(index_order), ctypes.byref(bk), _ptr(batch_order), _ptr(dbitmap),
        _ptr(variant), _ptr(ref), _ptr(flags), _ptr(ws), ctypes.byref(need), _stream(stream)))
    return dbitmap, variant


TREE_NODE_BYTES = 256
DPOS_FIRST, DPOS_EQUAL = 0xFFFF, 0xFFFE


def ckey_tree_plan(n, fill=0.9):
    """Shape of the index tree for n keys (host only)."""
    sh = ckey_tree_shape()
    _check("ckey_tree_plan", _lib.ckey_tree_plan(n, fill, ctypes.byref(sh)))
    h = sh.height
    return {"height": h, "leaf_entries": sh.leaf_entries, "inner_entries": sh.inner_entries,
            "level_nodes": list(sh.level_nodes[:h]), "level_first": list(sh.level_first[:h]),
            "total_nodes": sh.total_nodes}


def ckey_bulk_load(keys, perm, ckeys, cbitmap, pair_pos, pk=32, fill=0.9, variant=None, ref=None,
                   nodes=None, deref=None, stream=None):
    """Index tree (Sec. 5.3) from a rebuild's outputs: perm, the sorted
    compressed keys (words, n) made with host bitmap ``cbitmap``, and pair_pos.
    Returns (nodes: uint8 device tensor (total_nodes, 256), deref: int64[1])."""
    cb, cbp = _host_bitmap(cbitmap)
    var, varp = (None, None) if variant is None else _host_bitmap(variant)
    dev = keys.data.device
    shape = ckey_tree_plan(keys.n, fill)
    if nodes is None:
        nodes = torch.empty((shape["total_nodes"], TREE_NODE_BYTES), dtype=torch.uint8, device=dev)
    if deref is None:
        deref = torch.zeros(1, dtype=torch.int64, device=dev)
    inp = ckey_tree_input(keys.c_struct(), perm.data_ptr() if keys.n else None,
                          ckeys.data_ptr() if keys.n else None, ckeys.shape[0], cbp,
                          pair_pos.data_ptr() if pair_pos is not None and pair_pos.numel() else None,
                          varp, None if ref is None else ref.data_ptr())
    need = ctypes.c_size_t(0)
    _check("ckey_bulk_load", _lib.ckey_bulk_load(ctypes.byref(inp), pk, fill, None, None, None,
                                                 ctypes.byref(need), None))
    ws = _workspace(need.value, dev)
    _check("ckey_bulk_load", _lib.ckey_bulk_load(ctypes.byref(inp), pk, fill, _ptr(nodes), _ptr(deref),
                                                 _ptr(ws), ctypes.byref(need), _stream(stream)))
    return nodes, deref


def ckey_compress(keys, bitmap, words=None, out=None, rowids=None, flags=None, stream=None):
    """Compressed keys as an int64 tensor of shape (words, n) (bit patterns of
    the uint64 words) and the row ids 0..n-1 (int32)."""
    bm, p = _host_bitmap(bitmap)
    plan = ckey_plan_query(bm)
    w = plan["words"] if words is None else words
    dev = keys.data.device
    ck = torch.empty((w, keys.n), dtype=torch.int64, device=dev) if out is None else out
    rid = torch.empty(keys.n, dtype=torch.int32, device=dev) if rowids is None else rowids
    ks = keys.c_struct()
    _check("ckey_compress", _lib.ckey_compress(ctypes.byref(ks), p, _ptr(ck), w, _ptr(rid),
                                               _ptr(flags), _stream(stream)))
    return ck, rid


def _opts(method=CKEY_SORT_RADIX, digit_bits=0, bucket_log2=None, model=None, flags=None, skip_trivial=False,
          fused_table=False, tile=0):
    if bucket_log2 is None:
        bucket_log2 = model.bucket_log2 if model is not None else 0
    return ckey_sort_opts(method, digit_bits, bucket_log2, 1 if skip_trivial else 0,
                          None if model is None else model.handle,
                          None if flags is None else flags.data_ptr(), 1 if fused_table else 0, tile)


def ckey_compress_sort(keys, bitmap, out=None, rowids=None, words=None, workspace=None,
                       stream=None, **opts):
    """Compress and sort in one call: (sorted compressed keys (words, n) int64,
    row ids in full-key order int32)."""
    bm, p = _host_bitmap(bitmap)
    if words is None:
        words = out.shape[0] if out is not None else ckey_plan_query(bm)["words"]
    w = words
    dev = keys.data.device
    ck = torch.empty((w, keys.n), dtype=torch.int64, device=dev) if out is None else out
    rid = torch.empty(keys.n, dtype=torch.int32, device=dev) if rowids is None else rowids
    ks = keys.c_struct()
    o = _opts(**opts)
    if workspace is None:  # size query; a caller's workspace is checked by the library
        need = ctypes.c_size_t(0)
        _check("ckey_compress_sort", _lib.ckey_compress_sort(ctypes.byref(ks), p, None, w, None,
                                                             ctypes.byref(o), None, ctypes.byref(need),
                                                             None))
        workspace = _workspace(need.value, dev)
    ws = workspace
    need = ctypes.c_size_t(ws.numel())
    _check("ckey_compress_sort", _lib.ckey_compress_sort(ctypes.byref(ks), p, _ptr(ck), w, _ptr(rid),
                                                         ctypes.byref(o), _ptr(ws), ctypes.byref(need),
                                                         _stream(stream)))
    return ck, rid


def ckey_sort_workspace(words, nbits, n, **opts):
    o = _opts(**opts)
    need = ctypes.c_size_t(0)
    _check("ckey_sort", _lib.ckey_sort(None, words, nbits, None, n, ctypes.byref(o), None,
                                       ctypes.byref(need), None))
    return need.value


def ckey_sort(ck, nbits, rowids, workspace=None, stream=None, **opts):
    """Sort (ck[:, i], rowids[i]) in place by the top nbits of the word string."""
    words, n = ck.shape
    o = _opts(**opts)
    need = ctypes.c_size_t(ckey_sort_workspace(words, nbits, n, **opts))
    ws = _workspace(need.value, ck.device) if workspace is None else workspace
    need = ctypes.c_size_t(ws.numel())
    _check("ckey_sort", _lib.ckey_sort(_ptr(ck), words, nbits, _ptr(rowids), n, ctypes.byref(o),
                                       _ptr(ws), ctypes.byref(need), _stream(stream)))
    return ck, rowids


NOALLOC_SCRATCH_BYTES = 64 << 20


def ckey_sort_noalloc(ck, nbits, rowids, stream=None, **opts):
    """ckey_sort (radix method) with the library's static scratch array instead
    of a workspace: allocates nothing."""
    words, n = ck.shape
    o = _opts(**opts)
    _check("ckey_sort_noalloc", _lib.ckey_sort_noalloc(_ptr(ck), words, nbits, _ptr(rowids), n,
                                                       ctypes.byref(o), _stream(stream)))
    return ck, rowids


def _build_descs(indexes):
    """ctypes descriptors + output tensors for a list of index specs."""
    descs = (ckey_index_desc * len(indexes))()
    outs, hold = [], []
    for x, spec in enumerate(indexes):
        k = spec["keys"]
        dev = k.data.device
        bm = spec.get("bitmap")
        if bm is not None:
            bm, bp = _host_bitmap(bm)
            hold.append(bm)
            words = ckey_plan_query(bm)["words"]
        else:
            bp = None
            words = max(1, (8 * k.key_bytes + 63) // 64)
        o = {"perm": torch.empty(k.n, dtype=torch.int32, device=dev),
             "bitmap": torch.empty(k.key_bytes, dtype=torch.uint8, device=dev)}
        if spec.get("want_pair_pos"):
            o["pair_pos"] = torch.empty(max(k.n - 1, 0), dtype=torch.int32, device=dev)
        if spec.get("want_ckeys"):
            o["ckeys"] = torch.empty((words, k.n), dtype=torch.int64, device=dev)
        iopts = None
        if spec.get("opts") is not None:
            iopts = _opts(**spec["opts"])
            hold.append(iopts)
        descs[x] = ckey_index_desc(k.c_struct(), bp, o["perm"].data_ptr() if k.n else None,
                                   o["bitmap"].data_ptr(),
                                   o["pair_pos"].data_ptr() if "pair_pos" in o and k.n > 1 else None,
                                   o["ckeys"].data_ptr() if "ckeys" in o and k.n else None, None,
                                   None if iopts is None else ctypes.pointer(iopts))
        outs.append(o)
    return descs, outs, hold


def ckey_rebuild_index_workspace(indexes, **opts):
    descs, _, _hold = _build_descs(indexes)
    so = _opts(**opts)
    need = ctypes.c_size_t(0)
    _check("ckey_rebuild_index", _lib.ckey_rebuild_index(descs, len(indexes), ctypes.byref(so),
                                                         None, ctypes.byref(need), None))
    return need.value


def ckey_rebuild_index(indexes, workspace=None, stream=None, **opts):
    """Rebuild one or more indexes.

    ``indexes``: list of dicts with keys ``keys`` (DeviceKeys), ``bitmap``
    (host uint8 array or None for a first build), optional ``opts`` (dict of
    sort options for this index) and optional booleans ``want_pair_pos`` /
    ``want_ckeys``.  Returns a list of dicts with ``perm``, ``bitmap``
    (device) and optionally ``pair_pos`` / ``ckeys``.
    """
    descs, outs, _hold = _build_descs(indexes)
    so = _opts(**opts)
    need = ctypes.c_size_t(0)
    _check("ckey_rebuild_index", _lib.ckey_rebuild_index(descs, len(indexes), ctypes.byref(so),
                                                         None, ctypes.byref(need), None))
    ws = _workspace(need.value, indexes[0]["keys"].data.device) if workspace is None else workspace
    need = ctypes.c_size_t(ws.numel())
    _check("ckey_rebuild_index", _lib.ckey_rebuild_index(descs, len(indexes), ctypes.byref(so),
                                                         _ptr(ws), ctypes.byref(need),
                                                         _stream(stream)))
    return outs


class RebuildGraph:
    """A table rebuild (radix method) captured once into a HIP graph.

    ``launch()`` replays it on the current stream; outputs are the tensors in
    ``outs`` (overwritten by every replay)."""

    def __init__(self, indexes, **opts):
        self._descs, self.outs, self._hold = _build_descs(indexes)
        self._so = _opts(**opts)
        need = ctypes.c_size_t(0)
        _check("ckey_rebuild_index", _lib.ckey_rebuild_index(self._descs, len(indexes),
                                                             ctypes.byref(self._so), None,
                                                             ctypes.byref(need), None))
        self.workspace = _workspace(need.value, indexes[0]["keys"].data.device)
        self._keys = [spec["keys"] for spec in indexes]  # keep inputs alive
        g = ctypes.c_void_p()
        _check("ckey_graph_create", _lib.ckey_graph_create(self._descs, len(indexes),
                                                           ctypes.byref(self._so), _ptr(self.workspace),
                                                           self.workspace.numel(), ctypes.byref(g)))
        self._g = g

    def launch(self, stream=None):
        _check("ckey_graph_launch", _lib.ckey_graph_launch(self._g, _stream(stream)))

    def __del__(self):
        if getattr(self, "_g", None):
            _lib.ckey_graph_destroy(self._g)
            self._g = None


def ckey_tune_index(spec, candidates, stream=None):
    """Time one rebuild of index ``spec`` per candidate option dict on the
    device; returns (index of the fastest, list of times in ms)."""
    descs, _outs, hold = _build_descs([spec])
    copts = (ckey_sort_opts * len(candidates))(*[_opts(**c) for c in candidates])
    need = 0
    for c in candidates:
        d1, _, _h = _build_descs([dict(spec, opts=c)])
        so = _opts()
        n1 = ctypes.c_size_t(0)
        _check("ckey_rebuild_index", _lib.ckey_rebuild_index(d1, 1, ctypes.byref(so), None,
                                                             ctypes.byref(n1), None))
        need = max(need, n1.value)
    ws = _workspace(need, spec["keys"].data.device)
    best = ctypes.c_uint32(0)
    times = (ctypes.c_float * len(candidates))()
    _check("ckey_tune_index", _lib.ckey_tune_index(descs, copts, len(candidates), _ptr(ws), ws.numel(),
                                                   _stream(stream), ctypes.byref(best), times))
    return best.value, list(times)


def as_u64(t):
    """Device int64 tensor of word bit patterns -> host numpy uint64 array."""
    return t.cpu().numpy().view(np.uint64)


# ----------------------------------------------------- learned bucketing --

MODEL_PARAMS = 385
_OFF_M, _OFF_V, _OFF_T = 2048, 4096, 8192  # byte offsets of the model memory's parts


class CdfModel:
    """Device memory of a CDF model (thresholds + MLP), owned by torch."""

    def __init__(self, bucket_log2=14, seed=0, device="cuda", stream=None):
        nbytes = _lib.ckey_cdf_model_bytes(bucket_log2)
        if nbytes == 0:
            raise CkeyError("ckey_cdf_model_bytes", CKEY_ERR_INVALID)
        self.bucket_log2 = bucket_log2
        self.mem = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        _check("ckey_cdf_model_init", _lib.ckey_cdf_model_init(self.handle, bucket_log2, seed,
                                                               _stream(stream)))

    @property
    def handle(self):
        return self.mem.data_ptr()

    def params(self):
        return self.mem[: 4 * MODEL_PARAMS].view(torch.float32)

    def set_params(self, p):
        """Write 385 host parameters (ckey_cdf_grad's order) and zero both Adam moments."""
        t = torch.as_tensor(np.ascontiguousarray(p, np.float32))
        if t.numel() != MODEL_PARAMS:
            raise ValueError(f"expected {MODEL_PARAMS} parameters, got {t.numel()}")
        self.params().copy_(t.to(self.mem.device))
        self.mem[_OFF_M:_OFF_T].zero_()

    def thresholds(self):
        return self.mem[_OFF_T:].view(torch.int64)


def ckey_cdf_fit(model, sorted_prefix, steps=500, batch=1 << 14, lr=3e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, seed=1, stream=None):
    """Fit thresholds and train the network; returns the per-step loss (device)."""
    o = ckey_cdf_train_opts(steps, batch, lr, beta1, beta2, eps, seed)
    need = ctypes.c_size_t(0)
    _check("ckey_cdf_fit", _lib.ckey_cdf_fit(None, model.bucket_log2, None, 0, ctypes.byref(o), None,
                                             None, ctypes.byref(need), None))
    dev = model.mem.device
    ws = _workspace(need.value, dev)
    trace = torch.zeros(max(steps, 1), dtype=torch.float32, device=dev)
    need = ctypes.c_size_t(ws.numel())
    _check("ckey_cdf_fit", _lib.ckey_cdf_fit(model.handle, model.bucket_log2, _ptr(sorted_prefix),
                                             sorted_prefix.numel(), ctypes.byref(o), _ptr(trace),
                                             _ptr(ws), ctypes.byref(need), _stream(stream)))
    return trace[:steps]


def ckey_cdf_grad(model, prefix, target, stream=None):
    """(grad float32[385], loss float32[1]) of the network on an explicit batch."""
    need = ctypes.c_size_t(0)
    _check("ckey_cdf_grad", _lib.ckey_cdf_grad(None, None, None, prefix.numel(), None, None, None,
                                               ctypes.byref(need), None))
    dev = model.mem.device
    ws = _workspace(need.value, dev)
    grad = torch.zeros(MODEL_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    need = ctypes.c_size_t(ws.numel())
    _check("ckey_cdf_grad", _lib.ckey_cdf_grad(model.handle, _ptr(prefix), _ptr(target), prefix.numel(),
                                               _ptr(grad), _ptr(loss), _ptr(ws), ctypes.byref(need),
                                               _stream(stream)))
    return grad, loss


def ckey_cdf_bucket(model, prefix, method=CKEY_SORT_LEARNED, stream=None):
    """(exact bucket int32[n], network guess int32[n] or None, stats int64[2])."""
    dev = model.mem.device
    n = prefix.numel()
    bucket = torch.empty(n, dtype=torch.int32, device=dev)
    pred = torch.empty(n, dtype=torch.int32, device=dev) if method == CKEY_SORT_LEARNED else None
    stats = torch.zeros(2, dtype=torch.int64, device=dev)
    _check("ckey_cdf_bucket", _lib.ckey_cdf_bucket(model.handle, model.bucket_log2, method,
                                                   _ptr(prefix), n, _ptr(bucket), _ptr(pred),
                                                   _ptr(stats), _stream(stream)))
    return bucket, pred, stats
