"""GPU test of ckey_sort_noalloc: the radix sort with the library's static
scratch array in place of a caller workspace, checked bit-exactly against
ckey_sort (the same sort with a workspace) and the oracle's order, on two calls
in a row, the second with a smaller input than the first."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11543_amd import ckey
    return ckey


def words_with_dups(n, words, nbits, seed):
    """Word-major (words, n) uint64 compressed keys: nbits meaningful bits,
    zero below them, one row in four a copy of another (ties by row id)."""
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 1 << 63, (words, n), dtype=np.uint64) * np.uint64(2) + rng.integers(
        0, 2, (words, n), dtype=np.uint64)
    for k in range(words):
        keep = min(64, max(0, nbits - 64 * k))
        mask = 0 if keep == 0 else ((1 << 64) - 1) ^ ((1 << (64 - keep)) - 1)
        w[k] &= np.uint64(mask)
    dup = rng.integers(0, n, n // 4)
    w[:, rng.integers(0, n, n // 4)] = w[:, dup]
    return w


def run_both(ck, w, nbits, digit_bits):
    import torch
    n = w.shape[1]
    a = torch.from_numpy(w.view(np.int64)).cuda()
    b = a.clone()
    ra = torch.arange(n, dtype=torch.int32, device="cuda")
    rb = ra.clone()
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(a, nbits, ra, digit_bits=digit_bits)
    ck.ckey_sort_noalloc(b, nbits, rb, digit_bits=digit_bits, flags=flags)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    return a, ra, b, rb


def test_noalloc_matches_workspace_sort_two_calls(ck):
    # first call: 2^20 + 333 rows of two words (100 meaningful bits), 8-bit digits
    w1 = words_with_dups((1 << 20) + 333, 2, 100, 1)
    print("noalloc call 1: n=2^20+333 words=2 nbits=100", flush=True)
    a, ra, b, rb = run_both(ck, w1, 100, 8)
    assert b.equal(a) and rb.equal(ra)
    # second call, smaller: 50001 rows of one word (40 bits), 5-bit digits;
    # the scratch array still holds the first call's contents
    w2 = words_with_dups(50001, 1, 40, 2)
    print("noalloc call 2: n=50001 words=1 nbits=40", flush=True)
    a, ra, b, rb = run_both(ck, w2, 40, 5)
    assert b.equal(a) and rb.equal(ra)
    np.testing.assert_array_equal(rb.cpu().numpy().view(np.uint32), O.csort(w2))


def test_noalloc_near_the_limit_and_tiny(ck):
    # the largest one-word sort the scratch array holds, then 2 rows and 0 rows
    n = 1 << 22
    assert ck.ckey_sort_workspace(1, 60, n) <= ck.NOALLOC_SCRATCH_BYTES
    for rows in (n, 2, 0):
        w = words_with_dups(max(rows, 1), 1, 60, rows)[:, :rows]
        print(f"noalloc: n={rows} words=1 nbits=60", flush=True)
        a, ra, b, rb = run_both(ck, np.ascontiguousarray(w), 60, 8)
        assert b.equal(a) and rb.equal(ra)
