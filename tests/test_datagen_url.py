"""The URL-like varchar workload (2^24 rows, 20-120 bytes zero-padded to 128):
its stated shape checked on a sample, with nothing of the method involved."""
import numpy as np

from paper_2009_11543_amd import datagen


def test_url_keys_shape():
    rows, lens = datagen.url_keys(20000, seed=1)
    assert rows.shape == (20000, 128) and rows.dtype == np.uint8
    assert lens.min() >= 20 and lens.max() <= 120
    assert abs(lens.mean() - 70) < 2                      # uniform in [20, 120]
    pad = np.arange(128)[None, :] >= lens[:, None]
    assert not rows[pad].any()                            # zero padding past the key
    body = rows[~pad]
    allowed = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789./", np.uint8)
    assert np.isin(body, allowed).all()
    assert (body != 0).all()                              # no NUL inside a key
    # hosts: the text before the first '/'; at most 256 of them, skewed (Zipf 1.1)
    hosts = {}
    for r, n in zip(rows[:5000], lens[:5000]):
        b = bytes(r[:n])
        h = b.split(b"/")[0]
        assert b"." not in b[len(h):]                     # path segments are [a-z0-9]
        if len(h) == n:
            continue                                      # the key ends inside its host
        assert 10 <= len(h) <= 30
        hosts[h] = hosts.get(h, 0) + 1
    assert len(hosts) <= 256
    counts = sorted(hosts.values(), reverse=True)
    assert counts[0] > 5 * counts[len(counts) // 2]


def test_url_keys_seeded():
    a, la = datagen.url_keys(3000, seed=7)
    b, lb = datagen.url_keys(3000, seed=7)
    c, _ = datagen.url_keys(3000, seed=8)
    assert np.array_equal(a, b) and np.array_equal(la, lb)
    assert not np.array_equal(a, c)
