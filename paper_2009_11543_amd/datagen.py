"""Seeded synthetic index keys.

Inputs only: nothing here computes distinction bits, compressed keys or sort
orders.  The same bytes feed the HIP library and the CPU oracle.  Randomness
comes from numpy's PCG64 generator seeded per workload.

Key formats follow the paper's index key format (Sec. 4.1): fixed strings as
they are, signed integers big-endian with the sign bit flipped so that byte
order equals numeric order, varchar keys zero-padded (the first pad byte is the
NUL terminator), multi-column keys concatenated.
"""
import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8).copy()
_ACGT_CODE = np.zeros(256, np.uint8)
_ACGT_CODE[ACGT] = np.arange(4, dtype=np.uint8)


def rng_for(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- encoders --

def encode_i32(v):
    """int32 values -> (n, 4) big-endian bytes with the sign bit toggled."""
    u = (np.asarray(v, np.int64).astype(np.uint32) ^ np.uint32(0x80000000)).astype(">u4")
    return u.view(np.uint8).reshape(-1, 4)


def encode_i64(v):
    """int64 values -> (n, 8) big-endian bytes with the sign bit toggled."""
    u = (np.asarray(v, np.int64).view(np.uint64) ^ np.uint64(1 << 63)).astype(">u8")
    return u.view(np.uint8).reshape(-1, 8)


def zipf_sampler(rng, s, K, size):
    """Ranks 0..K-1 with P(rank r) proportional to (r+1)^-s (inverse CDF)."""
    w = np.arange(1, K + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    return np.minimum(np.searchsorted(cdf, u, side="right"), K - 1)


# ------------------------------------------------------------ workloads --

def uniform_prefix_keys(n=1 << 20, seed=1, key_bytes=16, prefix_bytes=6):
    """16-byte binary keys: a fixed seeded prefix (bytes 0-5), the rest
    uniform (2^20 rows by default)."""
    rng = rng_for(seed)
    prefix = rng.integers(0, 256, prefix_bytes, dtype=np.uint8)
    keys = np.empty((n, key_bytes), np.uint8)
    keys[:, :prefix_bytes] = prefix
    keys[:, prefix_bytes:] = rng.integers(0, 256, (n, key_bytes - prefix_bytes), dtype=np.uint8)
    return keys


def dna_window_keys(n=1 << 26, seed=1, key_bytes=64, seq_len=1 << 27, p_mut=0.01):
    """64-byte ASCII keys over {A,C,G,T}: windows at uniform offsets into one
    seeded uniform sequence of 2^27 bases; each window position is then
    independently, with probability ``p_mut``, replaced by one of the other
    three bases chosen uniformly."""
    rng = rng_for(seed)
    seq = ACGT[rng.integers(0, 4, seq_len, dtype=np.uint8)]
    offs = rng.integers(0, seq_len - key_bytes + 1, n)
    win = np.lib.stride_tricks.sliding_window_view(seq, key_bytes)
    keys = win[offs]
    flat = keys.reshape(-1)
    total = flat.size
    if p_mut > 0 and total:
        pos_parts = []
        last = -1
        while True:
            m = int(total * p_mut * 1.05) + 1024
            gaps = rng.geometric(p_mut, size=m).astype(np.int64)
            pos = last + np.cumsum(gaps)
            pos_parts.append(pos[pos < total])
            if pos[-1] >= total:
                break
            last = int(pos[-1])
        pos = np.concatenate(pos_parts)
        shift = rng.integers(1, 4, pos.size, dtype=np.uint8)
        flat[pos] = ACGT[(_ACGT_CODE[flat[pos]] + shift) & 3]
    return keys


# Table 4 of the paper: (dataset, s, key bytes, m, full sort key bytes,
# compressed sort key bytes) of its Zipf(s, n, m) datasets of 10 million keys.
ZIPF_TABLE4 = [
    (1, 2.5, 48, 0, 56, 40), (2, 2.5, 56, 0, 64, 40), (3, 2.5, 64, 0, 72, 40),
    (4, 2.5, 72, 0, 80, 40), (5, 2.5, 80, 0, 88, 40), (6, 2.5, 88, 0, 96, 40),
    (7, 2.5, 96, 0, 104, 40), (8, 2.5, 104, 0, 112, 40), (9, 2.5, 112, 0, 120, 40),
    (10, 1.5, 40, 0, 48, 24), (11, 1.5, 40, 1, 48, 24), (12, 1.5, 40, 2, 48, 24),
    (13, 1.5, 40, 3, 48, 24), (14, 1.5, 40, 4, 48, 24),
    (15, 1.5, 64, 0, 72, 24), (16, 1.5, 64, 1, 72, 24), (17, 1.5, 64, 2, 72, 24),
    (18, 1.5, 64, 3, 72, 24), (19, 1.5, 64, 4, 72, 24), (20, 1.5, 64, 5, 72, 24),
]


def zipf_letter_table(s, bits=20):
    """Inverse-CDF table of Zipf(s, 26) over lower-case letters: entry u (of
    2^bits) is the letter of the uniform draw (u + 1/2) / 2^bits."""
    w = np.arange(1, 27, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w) / w.sum()
    u = (np.arange(1 << bits, dtype=np.float64) + 0.5) / float(1 << bits)
    return (0x61 + np.minimum(np.searchsorted(cdf, u, side="right"), 25)).astype(np.uint8)


def zipf_keys(n=10_000_000, s=2.5, key_bytes=64, m=0, seed=1):
    """The paper's Zipf(s, n, m) keys (Sec. 6): in every 8-byte word of a key
    the first m bytes hold one fixed printable ASCII byte (seeded) and the
    other 8 - m bytes are lower-case letters drawn from Zipf(s, 26) ('a' the
    most frequent), through a 2^20-entry inverse-CDF table of 32-bit draws."""
    rng = rng_for(seed)
    fixed = np.uint8(rng.integers(0x21, 0x7F))
    table = zipf_letter_table(s)
    pos = np.arange(key_bytes)
    lmask = (pos % 8) >= m
    nl = int(lmask.sum())
    out = np.empty((n, key_bytes), np.uint8)
    out[:, ~lmask] = fixed
    if nl:
        chunk = max(1, (1 << 25) // nl)
        for r0 in range(0, n, chunk):
            r1 = min(n, r0 + chunk)
            cnt = (r1 - r0) * nl
            raw = rng.bit_generator.random_raw((cnt + 1) // 2).view(np.uint32)[:cnt]
            letters = table[raw >> 12].reshape(r1 - r0, nl)
            if nl == key_bytes:
                out[r0:r1] = letters
            else:
                out[r0:r1, lmask] = letters
    return out


def uniform_keys(n=1 << 28, seed=1, key_bytes=32):  # noqa: D401
    """Uniform random bytes, ``key_bytes`` per row."""
    rng = rng_for(seed)
    return np.frombuffer(rng.bytes(n * key_bytes), np.uint8).reshape(n, key_bytes).copy()


def cluster_keys(n=1 << 28, seed=1, key_bytes=32, clusters=1 << 16):
    """Rows drawn from ``clusters`` random (key_bytes-1)-byte stems, each row's
    cluster uniform, its last byte uniform."""
    rng = rng_for(seed)
    stems = rng.integers(0, 256, (clusters, key_bytes - 1), dtype=np.uint8)
    cid = rng.integers(0, clusters, n)
    keys = np.empty((n, key_bytes), np.uint8)
    keys[:, : key_bytes - 1] = stems[cid]
    keys[:, key_bytes - 1] = rng.integers(0, 256, n, dtype=np.uint8)
    return keys


def random_small_keys(n, key_bytes, seed, alphabet=None):
    """Tiny test sets: bytes from ``alphabet`` (default all 256 values)."""
    rng = rng_for(seed)
    if alphabet is None:
        return rng.integers(0, 256, (n, key_bytes), dtype=np.uint8)
    alphabet = np.asarray(alphabet, np.uint8)
    return alphabet[rng.integers(0, len(alphabet), (n, key_bytes))]


def pack_varlen(rows, lengths):
    """(n, W) zero-padded rows + lengths -> (flat bytes, uint64 offsets[n+1])."""
    lengths = np.asarray(lengths, np.int64)
    offsets = np.zeros(len(lengths) + 1, np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    mask = np.arange(rows.shape[1])[None, :] < lengths[:, None]
    return np.ascontiguousarray(rows[mask]), offsets


_HOST_CHARS = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz.", np.uint8).copy()
_PATH_CHARS = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789", np.uint8).copy()


def url_keys(n=1 << 24, seed=1, width=128, min_len=20, max_len=120, hosts=256, host_s=1.1):
    """URL-like varchar keys.  256 seeded host prefixes of 10-30 chars over
    [a-z.]; each key takes one (Zipf s = 1.1 over the hosts) and appends 1-6
    path segments of 3-12 chars over [a-z0-9], each after a '/'.  The key's
    length is drawn uniformly in [20, 120]: the host + segments string is cut
    there, or its last segment is extended with more [a-z0-9] chars to reach
    it.  Returns (rows (n, width) zero-padded, lengths); pack_varlen gives the
    flat bytes + offsets of the variable-length form."""
    rng = rng_for(seed)
    hl = rng.integers(10, 31, hosts)
    host_rows = _HOST_CHARS[rng.integers(0, len(_HOST_CHARS), (hosts, 30))]
    h = zipf_sampler(rng, host_s, hosts, n)
    lens = rng.integers(min_len, max_len + 1, n)
    rows = _PATH_CHARS[rng.integers(0, len(_PATH_CHARS), (n, width), dtype=np.uint8)]
    rows[:, :30] = np.where(np.arange(30)[None, :] < hl[h][:, None], host_rows[h], rows[:, :30])
    nseg = rng.integers(1, 7, n)
    seg = rng.integers(3, 13, (n, 6))
    pos = hl[h][:, None] + np.arange(6)[None, :] + np.concatenate(
        [np.zeros((n, 1), np.int64), np.cumsum(seg, axis=1)[:, :-1]], axis=1)  # '/' before segment j
    ok = (np.arange(6)[None, :] < nseg[:, None]) & (pos < lens[:, None])
    r, c = np.nonzero(ok)
    rows[r, pos[r, c]] = ord("/")
    rows[np.arange(width)[None, :] >= lens[:, None]] = 0
    return rows, lens


def _title_vocab(rng, size=50000):
    """Unique [a-z]{2..12} words, first letter capitalised: (size, 12) bytes + lengths."""
    out, lens, seen = [], [], set()
    while len(out) < size:
        m = 2 * (size - len(out)) + 100
        L = rng.integers(2, 13, m)
        chars = rng.integers(ord("a"), ord("z") + 1, (m, 12), dtype=np.uint8)
        for i in range(m):
            w = bytes(chars[i, : L[i]])
            if w not in seen:
                seen.add(w)
                out.append(chars[i].copy())
                lens.append(L[i])
                if len(out) == size:
                    break
    vocab = np.stack(out)
    vocab[:, 0] -= 32  # capitalise
    lens = np.array(lens, np.int64)
    vocab[np.arange(12)[None, :] >= lens[:, None]] = 0
    return vocab, lens


def title_keys(n, seed, width=48, max_len=40, min_len=8, words_per_row=10, vocab_size=50000):
    """Title-like strings: words from a seeded synthetic vocabulary chosen by
    Zipf(1.0), joined by single spaces until at least the row's length
    l ~ U[min_len, max_len], truncated to l, zero-padded to `width` bytes."""
    rng = rng_for(seed)
    vocab, vlen = _title_vocab(rng, vocab_size)
    target = rng.integers(min_len, max_len + 1, n)
    w_cdf = np.cumsum(np.arange(1, vocab_size + 1, dtype=np.float64) ** -1.0)
    w_cdf /= w_cdf[-1]
    rows = np.zeros((n, width), np.uint8)
    flat = rows.reshape(-1)
    start = np.zeros(n, np.int64)
    act = np.arange(n, dtype=np.int64)  # rows still shorter than their target
    cols = np.arange(12, dtype=np.int64)[None, :]
    for j in range(words_per_row):
        if act.size == 0:
            break
        w = np.minimum(np.searchsorted(w_cdf, rng.random(act.size), side="right"), vocab_size - 1)
        wl = vlen[w]
        pos = start[act][:, None] + cols                      # (a, 12) target columns
        ok = (cols < wl[:, None]) & (pos < target[act][:, None])
        flat[(act[:, None] * width + pos)[ok]] = vocab[w][ok]
        sp = start[act] + wl
        oks = sp < target[act]
        flat[act[oks] * width + sp[oks]] = ord(" ")
        start[act] = sp + 1
        act = act[start[act] < target[act]]
    # a row that ends on a space keeps it; the zero padding ends the string
    return rows


def table_indexes(n=1 << 24, seed=1):
    """Eight indexes of one synthetic table (fixed-width key rows each):
    int64 uniform; int32 Zipf(1.2) over 2^20 distinct values; a 12-byte
    composite (int32 day in a 10-year range, int64 uniform id); 48-byte titles;
    two int32 and two int64 uniform columns."""
    rng = rng_for(seed)
    i64 = lambda: rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64,
                               endpoint=True)
    i32 = lambda: rng.integers(np.iinfo(np.int32).min, np.iinfo(np.int32).max, n, dtype=np.int64,
                               endpoint=True)
    vals = np.unique(rng.integers(0, 1 << 32, (1 << 20) + (1 << 16), dtype=np.int64))
    vals = rng.permutation(vals)[: 1 << 20] - (1 << 31)
    zipf_col = vals[zipf_sampler(rng, 1.2, 1 << 20, n)]
    day = rng.integers(16436, 16436 + 3652 + 1, n)
    return {
        "int64": encode_i64(i64()),
        "int32_zipf": encode_i32(zipf_col),
        "day_id": np.ascontiguousarray(np.concatenate([encode_i32(day), encode_i64(i64())], 1)),
        "title": title_keys(n, seed + 100),
        "int32_a": encode_i32(i32()),
        "int32_b": encode_i32(i32()),
        "int64_a": encode_i64(i64()),
        "int64_b": encode_i64(i64()),
    }
