"""CPU test of the bucket searches in csrc/bucket.h through a host build
(tests/emu/bucket_host.h stands in for the HIP definitions; one thread runs
each cooperative loop whole).  Every form of the search the kernels use is
checked against the definition of a key's bucket in the sorted threshold
table T (T[0] = 0): the largest b with T[b] <= x.

  * splitter, every threshold in LDS in breadth-first order: one key at a
    time and eight interleaved;
  * splitter, a 1-in-S sample in LDS then T in memory: one key at a time and
    eight interleaved (S = 16, 32 as chosen beyond 2^14 buckets, and a forced
    S at a small B);
  * learned: the outward exponential search, the fixed-depth window search
    and the four-key interleaved galloping search of T in memory, from
    arbitrary guesses (near, far, at either end);
  * the network's guess for one key and for four at once agree exactly;
  * the packed 16-bit LDS histogram flushed to the global one equals the
    bucket counts, with partial flushes on the way (every 500 keys, the pairs
    holding a count above 5) and the full one at the end.
An address sanitizer build checks that no search reads outside its LDS image
or T."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2009_11543_amd", "csrc", "bucket.h")
EMU = os.path.join(ROOT, "tests", "emu")
KH = 64


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("bucket_emu")
    src = open(SRC).read()
    assert src.count('#include "internal.h"') == 1
    open(d / "bucket.h", "w").write(src.replace('#include "internal.h"', '#include "bucket_host.h"'))
    exe = d / "emu"
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-I", str(d), "-I", EMU, "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                        os.path.join(EMU, "bucket_main.cpp")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def thresholds(rng, B, kind):
    if kind == "uniform":
        t = np.sort(rng.integers(0, 2**64 - 1, B - 1, dtype=np.uint64, endpoint=True))
    elif kind == "dups":  # long runs of equal thresholds
        t = np.sort(rng.choice(rng.integers(1, 2**62, max(2, B // 50), dtype=np.uint64), B - 1))
    else:  # clustered in a narrow range, some equal to the top value
        t = np.sort(np.uint64(7 << 40) + rng.integers(0, 1 << 20, B - 1, dtype=np.uint64))
        t[-3:] = np.uint64(2**64 - 1)
    return np.concatenate([np.zeros(1, np.uint64), t])


def run(emu, tmp_path, B, S, kind, seed):
    rng = np.random.default_rng(seed)
    T = thresholds(rng, B, kind)
    nx = 20000
    x = rng.integers(0, 2**64 - 1, nx, dtype=np.uint64, endpoint=True)
    x[:2000] = T[rng.integers(0, B, 2000)]                      # equal to a threshold
    x[2000:3000] = T[rng.integers(1, B, 1000)] - np.uint64(1)   # just below one
    x[3000:3200] = 0
    x[3200:3400] = np.uint64(2**64 - 1)
    if kind == "cluster":
        x[4000:12000] = np.uint64(7 << 40) + rng.integers(0, 1 << 21, 8000, dtype=np.uint64)
    exp = (np.searchsorted(T, x, side="right") - 1).astype(np.uint32)
    g = rng.integers(0, B, nx).astype(np.uint32)
    near = rng.integers(-600, 601, nx)
    g[::3] = np.clip(exp[::3].astype(np.int64) + near[::3], 0, B - 1).astype(np.uint32)
    g[1::7] = 0
    g[2::7] = B - 1
    params = (rng.standard_normal(6 * KH + 1) * 0.5).astype(np.float32)
    (tmp_path / "m.txt").write_text(f"{B} {S} {nx}\n")
    T.tofile(tmp_path / "T.bin")
    x.tofile(tmp_path / "x.bin")
    g.tofile(tmp_path / "g.bin")
    params.tofile(tmp_path / "p.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([str(emu), str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    out = {k: np.fromfile(tmp_path / f"{k}.bin", np.uint32)
           for k in ("one", "many", "lcorr", "lwin", "lmany", "pr1", "pr4", "hist")}
    for k in ("one", "many", "lcorr", "lwin", "lmany"):
        np.testing.assert_array_equal(out[k], exp, err_msg=f"{k} B={B} S={S} {kind}")
    np.testing.assert_array_equal(out["pr1"], out["pr4"])
    assert int(out["pr1"].max()) < B
    np.testing.assert_array_equal(out["hist"], np.bincount(exp, minlength=B).astype(np.uint32))


def splitter_stride(B):
    return 1 if B <= 1 << 14 else (B // 2048 if B // 16 > 2048 else 16)


@pytest.mark.parametrize("kind", ["uniform", "dups", "cluster"])
@pytest.mark.parametrize("B", [256, 1024, 1 << 14, 1 << 15, 1 << 16])
def test_bucket_searches(emu, tmp_path, B, kind):
    S = splitter_stride(B)
    assert (B > 1 << 14) == (S > 1) and S in (1, 16, 32)
    run(emu, tmp_path, B, S, kind, seed=B + len(kind))


@pytest.mark.parametrize("S", [2, 16, 64])
def test_sampled_search_small_table(emu, tmp_path, S):
    run(emu, tmp_path, 1024, S, "dups", seed=S)
