"""Host-side baselines: PEXT compression (Sec. 5.1) and the row-column sort
(Appendix A) on the host cores, and the GCC parallel-mode sort of the same
records or of the full keys, built from ``rowcol.cpp`` with g++ (OpenMP).  Used
to set the paper's own CPU pipeline beside the GPU path; the GPU library never
calls it."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rowcol.cpp")
_LIB = os.path.join(_HERE, "librowcol.so")
_lib = None


def build():
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-Wall", "-shared", "-fPIC", "-pthread", "-fopenmp",
                           "-o", _LIB, _SRC])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        lib.rowcol_compress_sort.argtypes = [P, U64, U32, U32, P, U32, ctypes.c_int, U64, P, P, P]
        lib.rowcol_compress_sort.restype = ctypes.c_int
        lib.gnu_compress_sort.argtypes = [P, U64, U32, U32, P, U32, ctypes.c_int, P, P, P]
        lib.gnu_compress_sort.restype = ctypes.c_int
        lib.gnu_full_sort.argtypes = [P, U64, U32, U32, ctypes.c_int, P, P]
        lib.gnu_full_sort.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_cache_bytes(threads):
    """Last-level cache per thread (Appendix A's C), from sysfs; 2 MiB if unknown."""
    try:
        base = "/sys/devices/system/cpu/cpu0/cache"
        best = 0
        for ix in os.listdir(base):
            if not ix.startswith("index"):
                continue
            lvl = int(open(os.path.join(base, ix, "level")).read())
            size = open(os.path.join(base, ix, "size")).read().strip()
            mult = {"K": 1 << 10, "M": 1 << 20}.get(size[-1], 1)
            val = int(size.rstrip("KM")) * mult
            if lvl >= 3 or (lvl == 2 and best == 0):
                best = max(best, val)
        return max(1 << 16, best // max(1, threads))
    except (OSError, ValueError):
        return 2 << 20


def compress_sort(rows, bitmap, threads=None, cache_bytes=None, want_ckeys=False):
    """rows: (n, stride) uint8, keys are the first len(bitmap) bytes.  Returns
    (perm uint32[n], sorted compressed keys (words, n) or None, times dict)."""
    rows = np.ascontiguousarray(rows, np.uint8)
    bm = np.ascontiguousarray(bitmap, np.uint8)
    n, stride = rows.shape
    L = len(bm)
    threads = threads or min(16, os.cpu_count() or 1)
    cache_bytes = cache_bytes or default_cache_bytes(threads)
    nbits = int(np.unpackbits(bm).sum())
    words = max(1, -(-nbits // 64))
    perm = np.zeros(n, np.uint32)
    ck = np.zeros((words, n), np.uint64) if want_ckeys else None
    t = np.zeros(5, np.float64)
    rc = _load().rowcol_compress_sort(rows.ctypes.data if n else None, n, L, stride, bm.ctypes.data, words,
                                      threads, cache_bytes, perm.ctypes.data,
                                      None if ck is None else ck.ctypes.data, t.ctypes.data)
    if rc != 0:
        raise ValueError("rowcol_compress_sort: bad arguments")
    return perm, ck, {"compress_s": t[0], "sort_s": t[1], "phase_block_sort_s": t[2],
                      "phase_split_s": t[3], "phase_merge_s": t[4], "threads": threads,
                      "cache_bytes": cache_bytes}


def gnu_compress_sort(rows, bitmap, threads=None, want_ckeys=False):
    """Compression as compress_sort, then __gnu_parallel::sort of the
    (compressed key, record ID) records.  Returns (perm, ckeys or None, times)."""
    rows = np.ascontiguousarray(rows, np.uint8)
    bm = np.ascontiguousarray(bitmap, np.uint8)
    n, stride = rows.shape
    threads = threads or min(16, os.cpu_count() or 1)
    words = max(1, -(-int(np.unpackbits(bm).sum()) // 64))
    perm = np.zeros(n, np.uint32)
    ck = np.zeros((words, n), np.uint64) if want_ckeys else None
    t = np.zeros(5, np.float64)
    rc = _load().gnu_compress_sort(rows.ctypes.data if n else None, n, len(bm), stride, bm.ctypes.data, words,
                                   threads, perm.ctypes.data, None if ck is None else ck.ctypes.data,
                                   t.ctypes.data)
    if rc != 0:
        raise ValueError("gnu_compress_sort: bad arguments")
    return perm, ck, {"compress_s": t[0], "sort_s": t[1], "threads": threads}


def gnu_full_sort(rows, key_bytes, threads=None):
    """__gnu_parallel::sort of record IDs by memcmp of the first key_bytes
    bytes of each row, ties by record ID.  Returns (perm, seconds)."""
    rows = np.ascontiguousarray(rows, np.uint8)
    n, stride = rows.shape
    threads = threads or min(16, os.cpu_count() or 1)
    perm = np.zeros(n, np.uint32)
    sec = ctypes.c_double()
    rc = _load().gnu_full_sort(rows.ctypes.data if n else None, n, key_bytes, stride, threads,
                               perm.ctypes.data, ctypes.byref(sec))
    if rc != 0:
        raise ValueError("gnu_full_sort: bad arguments")
    return perm, sec.value
