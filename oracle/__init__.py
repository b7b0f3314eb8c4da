"""CPU oracle for the compressed key sort -- test infrastructure only.

Thin ctypes wrapper over ``oracle.c`` (plain C, built with gcc).  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may use it;
the HIP library never does.  Arrays in and out are numpy arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile oracle.c into liboracle.so (gcc -O2)."""
    subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        keys = [P, P, U64, U32, U32]
        lib.oracle_full_sort.argtypes = keys + [P]
        lib.oracle_dbits.argtypes = keys + [P, P]
        lib.oracle_dbit_pair.argtypes = keys + [U64, U64]
        lib.oracle_dbit_pair.restype = ctypes.c_int64
        lib.oracle_doffset.argtypes = [P, U32, P]
        lib.oracle_doffset.restype = U32
        lib.oracle_compress.argtypes = keys + [P, U32, P]
        lib.oracle_windows.argtypes = [P, U32, P, P]
        lib.oracle_windows.restype = U32
        lib.oracle_compress_windows.argtypes = keys + [P, U32, P]
        lib.oracle_csort.argtypes = [P, U32, U64, P]
        lib.oracle_refine.argtypes = [P, U32, U64, P, P, U32, P, P]
        lib.oracle_variant.argtypes = keys + [U64, P]
        lib.oracle_insert.argtypes = keys + [P, U64, P, U64, U64, P, P]
        lib.oracle_tree_fill.argtypes = [ctypes.c_double, P, P]
        lib.oracle_tree_shape.argtypes = [U64, ctypes.c_double, P]
        lib.oracle_tree_shape.restype = U32
        lib.oracle_bulk_load.argtypes = keys + [P, U32, ctypes.c_double, P]
        lib.oracle_mlp_loss_grad.argtypes = [P, P, P, U64, P]
        lib.oracle_mlp_loss_grad.restype = ctypes.c_double
        lib.oracle_mlp_forward.argtypes = [P, P, U64, P]
        D = ctypes.c_double
        lib.oracle_adam.argtypes = [P, P, P, P, U32, D, D, D, D, U32]
        lib.oracle_bucket.argtypes = [P, U64, P, U32, P]
        lib.oracle_thresholds.argtypes = [P, U64, U32, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Keys:
    """A key set as the oracle sees it: fixed-width rows or var-length bytes.

    ``fixed``: uint8 array of shape (n, stride) whose first ``L`` bytes per
    row are the key.  ``varlen``: (flat uint8 bytes, uint64 offsets[n+1]) with
    each key zero-padded to ``L`` bytes.
    """

    def __init__(self, data, L=None, offsets=None):
        if offsets is None:
            data = np.ascontiguousarray(data, dtype=np.uint8)
            assert data.ndim == 2
            self.bytes = data
            self.offsets = None
            self.n = data.shape[0]
            self.stride = data.shape[1]
            self.L = self.stride if L is None else L
        else:
            self.bytes = np.ascontiguousarray(data, dtype=np.uint8)
            self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
            self.n = len(self.offsets) - 1
            self.stride = 0
            assert L is not None
            self.L = L

    def args(self):
        return (_ptr(self.bytes), _ptr(self.offsets), self.n, self.L, self.stride)

    def padded(self):
        """(n, L) zero-padded copy of the keys."""
        if self.offsets is None:
            return np.ascontiguousarray(self.bytes[:, : self.L])
        out = np.zeros((self.n, self.L), np.uint8)
        for i in range(self.n):
            a, b = int(self.offsets[i]), int(self.offsets[i + 1])
            out[i, : b - a] = self.bytes[a:b]
        return out


def full_sort(k):
    perm = np.empty(k.n, np.uint32)
    _load().oracle_full_sort(*k.args(), _ptr(perm))
    return perm


def dbits(k, perm=None):
    """(bitmap uint8[L], descending flag) of keys in ``perm`` order."""
    bm = np.zeros(k.L, np.uint8)
    if perm is not None:
        perm = np.ascontiguousarray(perm, np.uint32)
    desc = _load().oracle_dbits(*k.args(), _ptr(perm), _ptr(bm))
    return bm, bool(desc)


def dbit_pair(k, a, b):
    return int(_load().oracle_dbit_pair(*k.args(), a, b))


def doffset(bitmap):
    bitmap = np.ascontiguousarray(bitmap, np.uint8)
    L = len(bitmap)
    nd = _load().oracle_doffset(_ptr(bitmap), L, None)
    out = np.zeros(max(nd, 1), np.uint32)
    _load().oracle_doffset(_ptr(bitmap), L, _ptr(out))
    return out[:nd]


def nwords(bitmap):
    return max(1, (len(doffset(bitmap)) + 63) // 64)


def compress(k, bitmap, w=None):
    """Word-major compressed keys, uint64 array of shape (w, n)."""
    bitmap = np.ascontiguousarray(bitmap, np.uint8)
    w = nwords(bitmap) if w is None else w
    ck = np.zeros((w, k.n), np.uint64)
    rc = _load().oracle_compress(*k.args(), _ptr(bitmap), w, _ptr(ck))
    assert rc == 0
    return ck


def windows(bitmap):
    """Sec. 5.1 masks: (start bytes, 64-bit masks)."""
    bitmap = np.ascontiguousarray(bitmap, np.uint8)
    L = len(bitmap)
    nw = _load().oracle_windows(_ptr(bitmap), L, None, None)
    st = np.zeros(max(nw, 1), np.uint32)
    mk = np.zeros(max(nw, 1), np.uint64)
    _load().oracle_windows(_ptr(bitmap), L, _ptr(st), _ptr(mk))
    return st[:nw], mk[:nw]


def compress_windows(k, bitmap, w=None):
    bitmap = np.ascontiguousarray(bitmap, np.uint8)
    w = nwords(bitmap) if w is None else w
    ck = np.zeros((w, k.n), np.uint64)
    rc = _load().oracle_compress_windows(*k.args(), _ptr(bitmap), w, _ptr(ck))
    assert rc == 0
    return ck


def csort(ck):
    ck = np.ascontiguousarray(ck, np.uint64)
    w, n = ck.shape
    perm = np.empty(n, np.uint32)
    _load().oracle_csort(_ptr(ck), w, n, _ptr(perm))
    return perm


def refine(ck, perm, bitmap_in):
    """(new bitmap, per-pair full-key D positions) from sorted compressed keys."""
    ck = np.ascontiguousarray(ck, np.uint64)
    perm = np.ascontiguousarray(perm, np.uint32)
    bitmap_in = np.ascontiguousarray(bitmap_in, np.uint8)
    w, n = ck.shape
    L = len(bitmap_in)
    out = np.zeros(L, np.uint8)
    pos = np.zeros(max(n - 1, 1), np.uint32)
    rc = _load().oracle_refine(_ptr(ck), w, n, _ptr(perm), _ptr(bitmap_in), L, _ptr(out), _ptr(pos))
    assert rc == 0
    return out, pos[: max(n - 1, 0)]


def variant(k, ref_row=0):
    out = np.zeros(k.L, np.uint8)
    _load().oracle_variant(*k.args(), ref_row, _ptr(out))
    return out


def insert(k, order, ins, dbitmap, variant=None, ref_row=0):
    """Sequential inserts (Sec. 4.3) of rows ``ins`` into the index whose rows in
    key order are ``order``.  Returns the updated (dbitmap, variant) copies."""
    order = np.ascontiguousarray(order, np.uint32)
    ins = np.ascontiguousarray(ins, np.uint32)
    d = np.array(dbitmap, np.uint8, copy=True)
    v = None if variant is None else np.array(variant, np.uint8, copy=True)
    rc = _load().oracle_insert(*k.args(), _ptr(order), len(order), _ptr(ins), len(ins), ref_row,
                               _ptr(d), _ptr(v))
    assert rc == 0
    return d, v


TREE_NODE = 256


def _f32(fill):
    """The fill factor as the library receives it (a C float)."""
    return float(np.float32(fill))


def tree_fill(fill):
    fill = _f32(fill)
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _load().oracle_tree_fill(fill, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def tree_shape(n, fill):
    """Nodes per level, leaves first (Sec. 5.3)."""
    lv = np.zeros(32, np.uint64)
    h = _load().oracle_tree_shape(n, _f32(fill), _ptr(lv))
    return [int(x) for x in lv[:h]]


def bulk_load(k, perm, pk=32, fill=0.9):
    """Index tree bulk load (Sec. 5.3): uint8 array (nodes, 256)."""
    perm = np.ascontiguousarray(perm, np.uint32)
    total = sum(tree_shape(k.n, fill))
    nodes = np.zeros((max(total, 1), TREE_NODE), np.uint8)
    rc = _load().oracle_bulk_load(*k.args(), _ptr(perm), pk, _f32(fill), _ptr(nodes))
    assert rc == 0
    return nodes[:total]


# ------------------------------------------------------------ CDF model --
MLP_H = 64
MLP_P = 6 * MLP_H + 1


def mlp_features(prefix):
    """(n, 4) float64 features: four 16-bit chunks of each 64-bit prefix, /65536."""
    x = np.asarray(prefix, np.uint64)
    cols = [((x >> np.uint64(48 - 16 * j)) & np.uint64(0xFFFF)).astype(np.float64) / 65536.0
            for j in range(4)]
    return np.ascontiguousarray(np.stack(cols, 1))


def mlp_forward(p, X):
    p = np.ascontiguousarray(p, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    y = np.zeros(len(X), np.float64)
    _load().oracle_mlp_forward(_ptr(p), _ptr(X), len(X), _ptr(y))
    return y


def mlp_loss_grad(p, X, t):
    p = np.ascontiguousarray(p, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.zeros(MLP_P, np.float64)
    loss = _load().oracle_mlp_loss_grad(_ptr(p), _ptr(X), _ptr(t), len(X), _ptr(g))
    return loss, g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays p, m, v."""
    g = np.ascontiguousarray(g, np.float64)
    _load().oracle_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), len(p), lr, b1, b2, eps, t)


def bucket(prefix, T):
    x = np.ascontiguousarray(prefix, np.uint64)
    T = np.ascontiguousarray(T, np.uint64)
    out = np.zeros(len(x), np.uint32)
    _load().oracle_bucket(_ptr(x), len(x), _ptr(T), len(T), _ptr(out))
    return out


def thresholds(sorted_prefix, B):
    """uint64[B]: T[0] = 0, T[b] = sorted_prefix[b*m // B] (m = len(sorted_prefix))."""
    x = np.ascontiguousarray(sorted_prefix, np.uint64)
    if len(x) == 0:
        raise ValueError("thresholds need a non-empty training set")
    T = np.zeros(B, np.uint64)
    _load().oracle_thresholds(_ptr(x), len(x), B, _ptr(T))
    return T
