"""GPU tests of the learned bucketing sort (an extension of the paper's
compressed key sort): network gradients and an Adam step against the fp64
oracle, exact bucket assignment against the oracle's threshold definition, and
the final permutation against the oracle's full-key sort."""
import numpy as np
import pytest

import oracle as O
from paper_2009_11543_amd import datagen

pytestmark = pytest.mark.gpu

MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11543_amd import ckey
    return ckey


def dna_prefixes(n, seed):
    """First compressed words of DNA-window keys, sorted (oracle-computed)."""
    rows = datagen.dna_window_keys(n, seed=seed, seq_len=4 * n)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    cko = O.compress(k, d)
    return rows, k, perm, d, cko


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def splitmix_index(seed, step, j, m):
    """The sampling rule documented for ckey_cdf_fit, in Python integers."""
    z = (seed + 0x9E3779B97F4A7C15 * ((step << 32) + j + 1)) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z % m


@pytest.mark.parametrize("n", [1, 65, 3000, 70000])
def test_grad_matches_oracle(ck, n):
    """Gradient and loss of an explicit batch against the fp64 oracle: one
    sample, 65 (a full wave and one sample), 3000 (a ragged last wave, twelve
    partial rows) and 70000 (274 partial rows, so the reduction's streams run
    their eight-load rounds)."""
    import torch
    model = ck.CdfModel(bucket_log2=10, seed=7)
    rng = np.random.default_rng(1)
    x = rng.integers(0, 2 ** 63, n, dtype=np.uint64) * np.uint64(2)
    t = rng.random(n).astype(np.float32)
    grad, loss = ck.ckey_cdf_grad(model, to_dev(x), torch.from_numpy(t).cuda())
    p = model.params().double().cpu().numpy()
    loss_ref, g_ref = O.mlp_loss_grad(p, O.mlp_features(x), t.astype(np.float64))
    g = grad.double().cpu().numpy()
    scale = np.abs(g_ref).max()
    np.testing.assert_allclose(g, g_ref, rtol=1e-3, atol=1e-4 * scale)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-4)


def host_params(seed):
    """A starting point for training made on the host (seeded), in the shape the
    library's own initialisation uses: unit k watches the top 16-bit chunk with
    its kink at k/64, the output starts near the first unit's identity."""
    rng = np.random.default_rng(seed)
    H = O.MLP_H
    p = np.zeros(O.MLP_P)
    p[:4 * H] = 1e-3 * rng.standard_normal(4 * H)
    p[0:4 * H:4] += 1.0
    p[4 * H:5 * H] = -np.arange(H) / H
    p[5 * H:6 * H] = 1e-3 * rng.standard_normal(H)
    p[5 * H] += 1.0
    return p.astype(np.float32).astype(np.float64)


def oracle_training(srt, p0, steps, batch, seed, lr, b1=0.9, b2=0.999, eps=1e-8):
    """`steps` oracle Adam steps on the batches ckey_cdf_fit documents (sample j
    of step s is row SplitMix64(seed + phi*((s << 32) + j + 1)) mod m, target
    (row + 0.5)/m); returns the parameters after every step and each loss."""
    m = len(srt)
    p, mm, vv = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    after, losses = [], []
    for s in range(1, steps + 1):
        idx = np.array([splitmix_index(seed, s, j, m) for j in range(batch)])
        X = O.mlp_features(srt[idx])
        tgt = (idx.astype(np.float64) + 0.5) / m
        loss, g = O.mlp_loss_grad(p, X, tgt)
        O.adam(p, g, mm, vv, s, lr, b1, b2, eps)
        after.append(p.copy())
        losses.append(loss)
    return after, losses


def test_adam_step_matches_oracle(ck):
    """One training step: sampled batch (documented SplitMix64 rule), gradient,
    Adam update -- all compared with the fp64 oracle from the same host-made
    starting parameters; the threshold table against the oracle's."""
    _, _, perm, _, cko = dna_prefixes(1 << 12, 3)
    srt = np.ascontiguousarray(cko[0, perm])
    model = ck.CdfModel(bucket_log2=8, seed=5)
    p0 = host_params(5)
    model.set_params(p0)
    batch, seed, lr = 2048, 11, 1e-2
    ck.ckey_cdf_fit(model, to_dev(srt), steps=1, batch=batch, lr=lr, seed=seed)
    p1 = model.params().double().cpu().numpy()
    (pr,), _ = oracle_training(srt, p0, 1, batch, seed, lr)
    # an fp32 gradient of 2048 terms moves a component by lr*sign(g) up to a
    # relative error of ~1e-4, except where g is tiny and the sign is noise
    idx = np.array([splitmix_index(seed, 1, j, len(srt)) for j in range(batch)])
    _, g = O.mlp_loss_grad(p0, O.mlp_features(srt[idx]), (idx + 0.5) / len(srt))
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    np.testing.assert_allclose((p1 - p0)[big], (pr - p0)[big], rtol=1e-3, atol=1e-6)
    T = model.thresholds().cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(T, O.thresholds(srt, 1 << 8))


def test_training_is_deterministic(ck):
    """The gradient sums run in a fixed order with no atomics: two fits from
    the same parameters on the same batches (2^16 samples, 256 partial rows
    a step) end in the same bytes, parameters and loss trace alike."""
    _, _, perm, _, cko = dna_prefixes(1 << 14, 4)
    srt = np.ascontiguousarray(cko[0, perm])
    p0 = host_params(7)
    runs = []
    for _ in range(2):
        model = ck.CdfModel(bucket_log2=8, seed=0)
        model.set_params(p0)
        trace = ck.ckey_cdf_fit(model, to_dev(srt), steps=20, batch=1 << 16, lr=1e-2, seed=3)
        runs.append((model.params().cpu().numpy().tobytes(), trace.cpu().numpy().tobytes()))
    assert runs[0] == runs[1]
    assert not np.array_equal(np.frombuffer(runs[0][0], np.float32), p0.astype(np.float32))


def test_training_ten_steps_matches_oracle(ck):
    """Ten steps of ckey_cdf_fit against ten oracle steps on the same SplitMix64
    batches from the same host-made parameters.  Bound: each fp32 step's update
    lr*m_hat/sqrt(v_hat) carries the relative error of a 2048-term fp32 sum
    (~1e-4 at most) and the error of earlier steps, so after s steps every
    parameter agrees within 1e-3*lr*s (an fp32 emulation of the same ten steps
    stays within 5e-5*lr); each step's loss within rtol 1e-4."""
    _, _, perm, _, cko = dna_prefixes(1 << 12, 3)
    srt = np.ascontiguousarray(cko[0, perm])
    batch, seed, lr, steps = 2048, 11, 1e-2, 10
    p0 = host_params(6)
    after, losses = oracle_training(srt, p0, steps, batch, seed, lr)
    for s in (1, 4, steps):
        model = ck.CdfModel(bucket_log2=8, seed=0)
        model.set_params(p0)
        trace = ck.ckey_cdf_fit(model, to_dev(srt), steps=s, batch=batch, lr=lr, seed=seed)
        got = model.params().double().cpu().numpy()
        np.testing.assert_allclose(got, after[s - 1], rtol=0, atol=1e-3 * lr * s)
        np.testing.assert_allclose(trace.double().cpu().numpy(), losses[:s], rtol=1e-4)
    # the ten steps really move the parameters (by about lr each)
    assert np.abs(after[-1] - p0).max() > 5 * lr


@pytest.mark.parametrize("method", ["learned", "splitter"])
def test_bucket_exact(ck, method):
    import torch
    _, _, perm, _, cko = dna_prefixes(1 << 14, 4)
    srt = np.ascontiguousarray(cko[0, perm])
    model = ck.CdfModel(bucket_log2=12, seed=1)
    ck.ckey_cdf_fit(model, to_dev(srt), steps=50, batch=4096)
    T = model.thresholds().cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(2)
    q = np.concatenate([cko[0], T, T - np.uint64(1), np.array([0, MASK64], np.uint64),
                        rng.integers(0, 2 ** 63, 5000, dtype=np.uint64) * np.uint64(2)])
    meth = ck.CKEY_SORT_LEARNED if method == "learned" else ck.CKEY_SORT_SPLITTER
    b, pred, stats = ck.ckey_cdf_bucket(model, to_dev(q), meth)
    np.testing.assert_array_equal(b.cpu().numpy().view(np.uint32), O.bucket(q, T))
    if method == "learned":
        assert int(stats[0].item()) > 0    # the search from the guess reads T
    else:
        assert int(stats[0].item()) == 0   # 2^12 thresholds: the whole search runs in LDS


def trained_model(ck, d, bucket_log2, n_train, steps=400, seed=2):
    """Model fitted to a training rebuild of a different seed, compressed with d."""
    import torch
    rows_t = datagen.dna_window_keys(n_train, seed=seed, seq_len=4 * n_train)
    dk = ck.DeviceKeys.from_numpy(rows_t)
    ckt, ridt = ck.ckey_compress(dk, d)
    plan = ck.ckey_plan_query(d)
    ck.ckey_sort(ckt, plan["nbits"], ridt)
    model = ck.CdfModel(bucket_log2=bucket_log2, seed=3)
    trace = ck.ckey_cdf_fit(model, ckt[0].contiguous(), steps=steps, batch=8192)
    torch.cuda.synchronize()
    return model, trace.cpu().numpy()


@pytest.mark.parametrize("method", ["learned", "splitter"])
@pytest.mark.parametrize("n", [1 << 15, (1 << 17) + 123])
def test_bucket_sort_parity(ck, method, n):
    import torch
    rows, k, perm, d, cko = dna_prefixes(n, 1)
    plan = ck.ckey_plan_query(d)
    model, _ = trained_model(ck, d, 8 if n < 1 << 16 else 10, 1 << 16)
    dk = ck.DeviceKeys.from_numpy(rows)
    ckd, rid = ck.ckey_compress(dk, d)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    meth = ck.CKEY_SORT_LEARNED if method == "learned" else ck.CKEY_SORT_SPLITTER
    ck.ckey_sort(ckd, plan["nbits"], rid, method=meth, model=model, flags=flags)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), cko[:, perm])


def test_bucket_overflow_falls_back(ck):
    """Buckets beyond the in-LDS capacity and long runs of equal prefixes go to
    the radix fallback; the permutation stays exact and the flag is raised."""
    import torch
    rng = np.random.default_rng(8)
    n = 1 << 18
    heavy = rng.integers(0, 256, (20, 16), dtype=np.uint8)
    rows = heavy[rng.integers(0, 20, n)]             # 90%: copies of 20 keys
    light = rng.random(n) < 0.1
    rows[light] = rng.integers(0, 256, (int(light.sum()), 16), dtype=np.uint8)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    plan = ck.ckey_plan_query(d)
    srt = np.ascontiguousarray(O.compress(k, d)[0, perm])
    model = ck.CdfModel(bucket_log2=8, seed=1)
    ck.ckey_cdf_fit(model, to_dev(srt), steps=20, batch=1024)
    dk = ck.DeviceKeys.from_numpy(rows)
    for meth in (ck.CKEY_SORT_LEARNED, ck.CKEY_SORT_SPLITTER):
        ckd, rid = ck.ckey_compress(dk, d)
        flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        ck.ckey_sort(ckd, plan["nbits"], rid, method=meth, model=model, flags=flags)
        np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
        assert int(flags.item()) & ck.CKEY_FLAG_BUCKET_OVERFLOW


def test_rebuild_with_learned_sort(ck):
    rows, k, perm, d, _ = dna_prefixes(1 << 15, 6)
    model, _ = trained_model(ck, d, 8, 1 << 15)
    dk = ck.DeviceKeys.from_numpy(rows)
    out = ck.ckey_rebuild_index([{"keys": dk, "bitmap": d}], method=ck.CKEY_SORT_LEARNED, model=model)[0]
    np.testing.assert_array_equal(out["perm"].cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(out["bitmap"].cpu().numpy(), d)


def test_trained_network_gain(ck):
    """What the trained network gains, against the untrained start (uniform
    CDF) and against the splitter, which needs no network: threshold probes
    per key -- the learned search reads T from the network's guess outward,
    the splitter searches all of T (log2 B levels) -- and the time of the
    whole sort with each method.  The trained network needs fewer probes than
    both; on this GPU its 64-unit fp32 evaluation costs more time than the
    probes it saves (the outcome is printed; both orders must equal the
    oracle's)."""
    import torch
    rows, k, perm, d, cko = dna_prefixes(1 << 16, 1)
    b_log2 = 10
    model, trace = trained_model(ck, d, b_log2, 1 << 16, steps=600)
    assert trace[-20:].mean() < 0.5 * trace[:5].mean()
    q = to_dev(cko[0])
    n = cko.shape[1]
    _, _, st_tr = ck.ckey_cdf_bucket(model, q, ck.CKEY_SORT_LEARNED)
    untrained = ck.CdfModel(bucket_log2=b_log2, seed=3)
    untrained.thresholds().copy_(model.thresholds())
    _, _, st_un = ck.ckey_cdf_bucket(untrained, q, ck.CKEY_SORT_LEARNED)
    probes_tr, err_tr = st_tr.cpu().numpy() / n
    probes_un, err_un = st_un.cpu().numpy() / n
    probes_sp = float(b_log2)  # every threshold in LDS: a full-depth search per key
    assert err_tr < 0.5 * err_un
    assert probes_tr < probes_un
    assert probes_tr < probes_sp
    # time of the whole compress + sort, learned vs splitter, same model
    dk = ck.DeviceKeys.from_numpy(rows)
    times = {}
    for name, meth in (("learned", ck.CKEY_SORT_LEARNED), ("splitter", ck.CKEY_SORT_SPLITTER)):
        _, rid = ck.ckey_compress_sort(dk, d, method=meth, model=model)
        np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            ck.ckey_compress_sort(dk, d, method=meth, model=model)
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 10
    print(f"probes/key: trained {probes_tr:.2f} (|err| {err_tr:.1f} buckets), untrained {probes_un:.2f} "
          f"(|err| {err_un:.1f}), splitter {probes_sp:.0f}; compress+sort of {n} keys: learned "
          f"{times['learned']:.3f} ms, splitter {times['splitter']:.3f} ms")


def test_bucket_spanning_a_gap_sorts_in_place(ck):
    """A bucket whose threshold range spans the gap between two clusters has no
    common prefix; its keys still differ below the 32 bits each cluster shares,
    so the in-LDS sort must finish it without the radix fallback."""
    import torch
    rng = np.random.default_rng(12)
    n = 1 << 17
    rows = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    hi = rng.random(n) < 0.5
    rows[:, 0] = np.where(hi, 0x80, 0x00)
    rows[:, 1:5] = np.where(hi[:, None], 0xFF, 0x00)   # 32 bits shared within a cluster
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    plan = ck.ckey_plan_query(d)
    srt = np.ascontiguousarray(O.compress(k, d)[0, perm])
    model = ck.CdfModel(bucket_log2=8, seed=1)
    ck.ckey_cdf_fit(model, to_dev(srt[::7].copy()), steps=20, batch=1024)
    T = model.thresholds().cpu().numpy().view(np.uint64)
    gap = [b for b in range(255) if (T[b] >> np.uint64(63)) != (T[b + 1] >> np.uint64(63))]
    assert gap, "expected a bucket spanning both clusters"
    dk = ck.DeviceKeys.from_numpy(rows)
    ckd, rid = ck.ckey_compress(dk, d)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, plan["nbits"], rid, method=ck.CKEY_SORT_SPLITTER, model=model, flags=flags)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    assert int(flags.item()) & ck.CKEY_FLAG_BUCKET_OVERFLOW == 0


@pytest.mark.parametrize("pattern", ["dup_runs", "few_digits", "all_equal_first_word"])
def test_bucket_sort_patterns(ck, pattern):
    """Buckets whose local keys vary in few digits, carry long runs of equal top
    digits (forcing the all-digit redo), or share one first word."""
    import torch
    rng = np.random.default_rng(hash(pattern) % 1000)
    n = 1 << 16
    rows = rng.integers(0, 256, (n, 24), dtype=np.uint8)
    if pattern == "dup_runs":        # 24 top bits shared by groups of ~40 keys
        rows[:, 0:3] = rng.integers(0, 1600, n).astype(">u4").view(np.uint8).reshape(n, 4)[:, 1:]
    elif pattern == "few_digits":    # only bits of two bytes vary in the first word
        rows[:, 0:6] = 7
        rows[:, 6:8] = rng.integers(0, 256, (n, 2))
    else:                            # first 8 bytes equal for runs of 20 keys
        rows[:, 0:8] = np.repeat(rng.integers(0, 256, (n // 20 + 1, 8)), 20, axis=0)[:n]
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    plan = ck.ckey_plan_query(d)
    srt = np.ascontiguousarray(O.compress(k, d)[0, perm])
    model = ck.CdfModel(bucket_log2=8, seed=1)
    ck.ckey_cdf_fit(model, to_dev(srt), steps=20, batch=1024)
    dk = ck.DeviceKeys.from_numpy(rows)
    ckd, rid = ck.ckey_compress(dk, d)
    ck.ckey_sort(ckd, plan["nbits"], rid, method=ck.CKEY_SORT_SPLITTER, model=model)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), O.compress(k, d)[:, perm])


@pytest.mark.parametrize("method", ["radix", "splitter", "learned"])
@pytest.mark.parametrize("layout", ["fixed16", "stride_odd", "varlen"])
def test_compress_sort_entry(ck, method, layout):
    """ckey_compress_sort (fused compression + bucket assignment where the keys
    allow it) against the oracle."""
    rng = np.random.default_rng(31)
    n, L = 50000, 24
    if layout == "varlen":
        lens = rng.integers(1, L + 1, n)
        rows = rng.choice(np.frombuffer(b"ACGT", np.uint8), (n, L))
        rows[np.arange(L)[None, :] >= lens[:, None]] = 0
        flat, offs = datagen.pack_varlen(rows, lens)
        k = O.Keys(flat, L=L, offsets=offs)
        dk = ck.DeviceKeys.from_numpy(flat, key_bytes=L, offsets=offs)
    else:
        rows = rng.choice(np.frombuffer(b"ACGT", np.uint8), (n, L))
        if layout == "stride_odd":
            rows = np.concatenate([rows, np.zeros((n, 3), np.uint8)], 1)
        k = O.Keys(rows, L=L)
        dk = ck.DeviceKeys.from_numpy(rows, key_bytes=L)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    cko = O.compress(k, d)
    opts = {}
    if method != "radix":
        model = ck.CdfModel(bucket_log2=8, seed=2)
        ck.ckey_cdf_fit(model, to_dev(np.ascontiguousarray(cko[0, perm])), steps=100, batch=4096)
        opts = dict(method=ck.CKEY_SORT_SPLITTER if method == "splitter" else ck.CKEY_SORT_LEARNED,
                    model=model)
    ckd, rid = ck.ckey_compress_sort(dk, d, **opts)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), cko[:, perm])


@pytest.mark.parametrize("words", [1, 2, 3, 5])
@pytest.mark.parametrize("per_bucket", [1024, 2048])
@pytest.mark.parametrize("pairs", [False, True])
def test_bucket_sort_group_paths(ck, words, per_bucket, pairs):
    """Direct word strings under evenly spaced thresholds (T[b] = b * 2^56):
    uniform first words (groups of equal top offset bits ranked in place),
    dense clusters of ~600 first words (a group beyond the in-place limit:
    the all-digit LSD), and repeated first words with differing later words
    (runs ordered by the later words and row ids).  1024 rows per bucket use
    the 512-thread kernel, 2048 the 1024-thread one; 5 words the kernel
    without a fixed word count.  With `pairs`, every first word appears
    twice, so run members exceed what is staged at once and runs are
    ordered array by array.  Expected order: lexicographic by
    (w0, ..., w_{k-1}, row id)."""
    import torch
    B = 256
    n = per_bucket * B + 77
    rng = np.random.default_rng(words * 10 + per_bucket + int(pairs))
    w = rng.integers(0, 1 << 63, (words, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    w += rng.integers(0, 2, (words, n), dtype=np.int64).astype(np.uint64)
    # clusters: 8 centres, 600 rows each, spread below 2^20
    centres = rng.integers(0, 1 << 63, 8, dtype=np.int64).astype(np.uint64)
    for c in range(8):
        idx = rng.choice(n, 600, replace=False)
        w[0, idx] = centres[c] + rng.integers(0, 1 << 20, 600, dtype=np.int64).astype(np.uint64)
    # repeated first words: runs of 2..12 rows
    src = rng.choice(n, n // 20, replace=False)
    for s in src[: n // 40]:
        w[0, rng.integers(0, n, int(rng.integers(1, 12)))] = w[0, s]
    if pairs:
        w[0, 1::2] = w[0, 0:n - 1:2]
    T = (np.arange(B, dtype=np.uint64) << np.uint64(56))
    model = ck.CdfModel(bucket_log2=8, seed=1)
    model.thresholds().copy_(to_dev(T))
    ckd = to_dev(w).reshape(words, n).contiguous()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, 64 * words, rid, method=ck.CKEY_SORT_SPLITTER, model=model, flags=flags)
    order = np.lexsort(tuple([np.arange(n)] + [w[k] for k in range(words - 1, -1, -1)]))
    np.testing.assert_array_equal(rid.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(ck.as_u64(ckd), w[:, order])
    assert int(flags.item()) & ck.CKEY_FLAG_SPIN_LIMIT == 0


@pytest.mark.parametrize("bucket_log2", [12, 15, 16])
def test_bucket_counts_many_buckets(ck, bucket_log2):
    """2^12 .. 2^16 evenly spaced thresholds: the bucket-start scan with
    16-byte loads and both forms of the pass histograms (staged in LDS up to
    2^15 buckets, read from global memory at 2^16)."""
    import torch
    n = (1 << 20) + 5
    rng = np.random.default_rng(bucket_log2)
    w = rng.integers(0, 1 << 63, (2, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    B = 1 << bucket_log2
    T = np.arange(B, dtype=np.uint64) << np.uint64(64 - bucket_log2)
    model = ck.CdfModel(bucket_log2=bucket_log2, seed=1)
    model.thresholds().copy_(to_dev(T))
    ckd = to_dev(w).reshape(2, n).contiguous()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, 128, rid, method=ck.CKEY_SORT_SPLITTER, model=model)
    order = np.lexsort((np.arange(n), w[1], w[0]))
    np.testing.assert_array_equal(rid.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(ck.as_u64(ckd), w[:, order])


def test_bucket_counts_beyond_16_bits_per_workgroup(ck):
    """2^25 one-word keys, 60 % of them one value: every assigning workgroup
    walks two chunks of 65535 keys and counts more than 65535 keys into the
    hot bucket in all, so its packed 16-bit counters are exact only when
    flushed after each chunk.  The bucket starts decide every destination:
    the permutation and keys equal a stable sort, and the hot bucket takes
    the radix fallback (CKEY_FLAG_BUCKET_OVERFLOW)."""
    import torch
    n = 1 << 25
    rng = np.random.default_rng(25)
    w = rng.integers(0, 1 << 62, n, dtype=np.int64)
    hot = rng.random(n) < 0.6
    w[hot] = 0x2D9B_5A1F_0C3E_7711
    B = 1 << 14
    sample = np.sort(w[rng.choice(n, 1 << 20, replace=False)])
    T = sample[(np.arange(B, dtype=np.int64) * sample.size) // B]
    T[0] = 0
    model = ck.CdfModel(bucket_log2=14, seed=1)
    model.thresholds().copy_(torch.from_numpy(T).cuda())
    ckd = torch.from_numpy(w).cuda().reshape(1, n).contiguous()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, 64, rid, method=ck.CKEY_SORT_SPLITTER, model=model, flags=flags)
    order = np.argsort(w, kind="stable")
    np.testing.assert_array_equal(rid.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(ckd[0].cpu().numpy(), w[order])
    f = int(flags.item())
    assert f & ck.CKEY_FLAG_BUCKET_OVERFLOW and not f & ck.CKEY_FLAG_SPIN_LIMIT


@pytest.mark.parametrize("words", [1, 3])
@pytest.mark.parametrize("too_big", [False, True])
def test_bucket_second_chance(ck, words, too_big):
    """Buckets beyond 5120 rows are sorted again by the 10240-row kernel (no
    overflow flag); one beyond 10240 rows goes on to the radix sort (flag)."""
    import torch
    B, per = 256, 4096
    n0 = B * per
    rng = np.random.default_rng(40 + words + 2 * int(too_big))
    w = rng.integers(0, 1 << 63, (words, n0), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    extra = [(5, 3000), (200, 1500)] + ([(9, 7000)] if too_big else [])
    parts = [w]
    for b, m in extra:
        e = rng.integers(0, 1 << 63, (words, m), dtype=np.int64).astype(np.uint64)
        e[0] = (np.uint64(b) << np.uint64(56)) | (e[0] >> np.uint64(8))
        parts.append(e)
    w = np.concatenate(parts, axis=1)
    n = w.shape[1]
    w = w[:, rng.permutation(n)]
    T = np.arange(B, dtype=np.uint64) << np.uint64(56)
    model = ck.CdfModel(bucket_log2=8, seed=1)
    model.thresholds().copy_(to_dev(T))
    ckd = to_dev(w).reshape(words, n).contiguous()
    rid = torch.arange(n, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    ck.ckey_sort(ckd, 64 * words, rid, method=ck.CKEY_SORT_SPLITTER, model=model, flags=flags)
    order = np.lexsort(tuple([np.arange(n)] + [w[k] for k in range(words - 1, -1, -1)]))
    np.testing.assert_array_equal(rid.cpu().numpy(), order.astype(np.int32))
    np.testing.assert_array_equal(ck.as_u64(ckd), w[:, order])
    assert bool(int(flags.item()) & ck.CKEY_FLAG_BUCKET_OVERFLOW) == too_big


@pytest.mark.parametrize("bucket_log2", [15, 16])
def test_fused_compress_sort_sampled_thresholds(ck, bucket_log2):
    """Beyond 2^14 buckets only a 1-in-S sample of the thresholds fits in LDS:
    the fused compress + bucket kernel searches the sample, then T, for four
    keys at once; the permutation equals the oracle's full-key order."""
    rows = datagen.uniform_keys(1 << 19, seed=3, key_bytes=32)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    rows_t = datagen.uniform_keys(1 << 18, seed=4, key_bytes=32)
    kt = ck.DeviceKeys.from_numpy(rows_t)
    ckt, ridt = ck.ckey_compress(kt, d)
    ck.ckey_sort(ckt, ck.ckey_plan_query(d)["nbits"], ridt)
    model = ck.CdfModel(bucket_log2=bucket_log2, seed=1)
    ck.ckey_cdf_fit(model, ckt[0].contiguous(), steps=20, batch=4096)
    for meth in (ck.CKEY_SORT_SPLITTER, ck.CKEY_SORT_LEARNED):
        ckd, rid = ck.ckey_compress_sort(ck.DeviceKeys.from_numpy(rows), d, method=meth, model=model)
        np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
        np.testing.assert_array_equal(ck.as_u64(ckd), O.compress(k, d)[:, perm])


def test_fused_compress_sort_wide_keys(ck):
    """Keys of 80 bytes sorted over all 640 bits (10 words): the fused path's
    grouping passes over more than 8 words, where the first pass generates
    the record IDs in the 256-thread pass kernel."""
    rng = np.random.default_rng(31)
    n = (1 << 15) + 3
    rows = rng.integers(0, 4, (n, 80), dtype=np.uint8) * np.uint8(0x40)  # few values: long shared prefixes
    rows[:, 70:] = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    bm = np.full(80, 0xFF, np.uint8)
    ckt, ridt = ck.ckey_compress(ck.DeviceKeys.from_numpy(rows), bm)
    ck.ckey_sort(ckt, 640, ridt)
    model = ck.CdfModel(bucket_log2=8, seed=1)
    ck.ckey_cdf_fit(model, ckt[0].contiguous(), steps=20, batch=4096)
    ckd, rid = ck.ckey_compress_sort(ck.DeviceKeys.from_numpy(rows), bm, method=ck.CKEY_SORT_SPLITTER,
                                     model=model)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), O.compress(k, bm)[:, perm])


@pytest.mark.parametrize("trained", [True, False])
def test_fused_learned_window_search(ck, trained):
    """The learned method's fused kernel (64-byte keys, 2^12 buckets: a
    fixed-depth search of the 1024 buckets around each guess, or of all of T
    for keys outside them).  A trained network puts most keys inside the
    window; an untrained one (same thresholds) sends most through the full
    search.  Either way the permutation and the compressed keys are the
    oracle's."""
    n = (1 << 20) + 333
    rows = datagen.dna_window_keys(n, seed=23, seq_len=1 << 21)
    k = O.Keys(rows)
    perm = O.full_sort(k)
    d, _ = O.dbits(k, perm)
    cko = O.compress(k, d)
    model = ck.CdfModel(bucket_log2=12, seed=2)
    ck.ckey_cdf_fit(model, to_dev(np.ascontiguousarray(cko[0, perm])), steps=300 if trained else 0, batch=1 << 14)
    if not trained:
        fresh = ck.CdfModel(bucket_log2=12, seed=9)
        fresh.thresholds().copy_(model.thresholds())
        model = fresh
    print(f"fused learned window search, trained={trained}, n={n}", flush=True)
    ckd, rid = ck.ckey_compress_sort(ck.DeviceKeys.from_numpy(rows), d, method=ck.CKEY_SORT_LEARNED, model=model)
    np.testing.assert_array_equal(rid.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(ck.as_u64(ckd), cko[:, perm])
