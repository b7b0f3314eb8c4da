#!/usr/bin/env python3
"""Benchmark of the compressed key sort on one MI355X.

A step is one pass of the timed hot path -- ckey_compress (gather of the
D-bitmap's bits into packed 64-bit words) followed by ckey_sort (stable
sort of the (compressed key, row id) pairs) -- over device-resident keys with
the D-bitmap given (it is index metadata computed by an earlier build, here a
first build over full keys done before the timed region).

Default workload: 2^26 keys of 64 ASCII bytes over {A,C,G,T}, windows at
uniform offsets into one seeded 2^27-base sequence with 1% point mutations.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compress+sort keys/s & HBM GB/s at 2^26 keys vs plain GPU full-key sort"
KERNEL_BYTES = ("compress", "compress_bucket", "hist", "onesweep", "assign_learned",
                "assign_splitter", "tile_counts", "bucket_pass", "bucket_sort")
PEAK_HBM_GBPS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def training_rows(name, n, seed=2):
    """Rows of the same generator at another seed (2: the training rebuild)."""
    from paper_2009_11543_amd import datagen
    if name == "dna64_2p26":
        return datagen.dna_window_keys(n, seed=seed)
    if name == "prefix16_2p20":
        return datagen.uniform_prefix_keys(n, seed=seed)
    if name == "uniform32_2p28":
        return datagen.uniform_keys(n, seed=seed)
    if name == "cluster32_2p28":
        return datagen.cluster_keys(n, seed=seed)
    if name == "url128_2p24":  # zero-padded rows compress to the same words as the varchar form
        return datagen.url_keys(n, seed=seed)[0]
    raise SystemExit(f"unknown workload {name}")


def workload(name):
    from paper_2009_11543_amd import datagen
    if name == "dna64_2p26":
        return datagen.dna_window_keys(1 << 26, seed=1), "2^26 x 64-byte DNA windows, 1% mutations, seed 1"
    if name == "prefix16_2p20":
        return datagen.uniform_prefix_keys(1 << 20, seed=1), "2^20 x 16-byte keys, 6-byte constant prefix, seed 1"
    if name == "uniform32_2p28":
        return datagen.uniform_keys(1 << 28, seed=1), "2^28 x 32 uniform bytes, seed 1"
    if name == "cluster32_2p28":
        return datagen.cluster_keys(1 << 28, seed=1), "2^28 x 32 bytes, 2^16 stems + uniform last byte, seed 1"
    if name == "url128_2p24":  # (zero-padded rows, lengths): the device gets flat bytes + offsets
        return datagen.url_keys(1 << 24, seed=1), ("2^24 URL-like keys of 20-120 bytes (mean 70), "
                                                   "zero-padded to 128, as flat bytes + offsets, seed 1")
    raise SystemExit(f"unknown workload {name}")


class Prof:
    def __init__(self, lib):
        self.lib = lib

    def on(self, flag=True):
        self.lib.ckey_profile_reset()
        self.lib.ckey_profile_enable(1 if flag else 0)

    def read(self, name):
        ms, cnt = ctypes.c_double(), ctypes.c_uint64()
        rc = self.lib.ckey_profile_read(name.encode(), ctypes.byref(ms), ctypes.byref(cnt))
        assert rc == 0
        return ms.value, cnt.value


def traffic_for(kernel, wl, src_file):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{wl}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(src_file, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


# The paper's own timings (Sec. 6, the INDBTAB sorting and index-building
# table), quoted for context only: another machine, another dataset (16,392k
# SAP HANA sales-document keys of 35 bytes, 16-byte compressed sort keys).
PAPER_CONTEXT = {
    "hardware": "Intel Xeon E7-8880 v4, 2.2 GHz; 1 core, and 16 cores of one socket",
    "workload": "INDBTAB, 16,392k keys",
    "one_core_s": {"extract": 0.543, "compressed_sort": 2.063, "full_key_sort": 4.251},
    "one_core_compress_sort_keys_per_s": 16_392_000 / (0.543 + 2.063),
    "sixteen_cores_s": {"extract": 0.034, "compressed_sort": 0.148, "full_key_sort": 0.310},
    "sixteen_cores_compress_sort_keys_per_s": 16_392_000 / (0.034 + 0.148),
    "use": "context only; not the target",
}


def cpu_baseline(rows_all, n_sample):
    """The CPU oracle, as it stands, on the first n_sample rows: compress with the
    sample's D-bitmap, then sort the compressed keys (single thread)."""
    import oracle as O
    rows = np.ascontiguousarray(rows_all[:n_sample])
    k = O.Keys(rows)
    d, _ = O.dbits(k, O.full_sort(k))
    t0 = time.perf_counter()
    ck = O.compress(k, d)
    perm = O.csort(ck)
    dt = time.perf_counter() - t0
    assert len(perm) == n_sample
    return {"value": n_sample / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} rows of the workload; oracle compress (bit by bit) + "
                      f"qsort of compressed keys, D-bitmap of the sample given; {dt:.1f} s",
            **host_cpu()}, d, perm


def host_cpu():
    """The host CPU the baselines ran on: model name, logical CPUs the process
    may use, and logical CPUs of the machine."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpus_total": os.cpu_count()}


def cpu_rowcol(rows_all, n_sample, d, perm_ref):
    """The paper's own CPU pipeline on the host cores: PEXT compression (Sec.
    5.1) and the row-column sort (Appendix A), on the same sample."""
    from paper_2009_11543_amd import rowcol
    rows = np.ascontiguousarray(rows_all[:n_sample])
    threads = min(16, os.cpu_count() or 1)
    perm, _, t = rowcol.compress_sort(rows, d, threads=threads)
    assert np.array_equal(perm, perm_ref), "row-column sort order differs from the oracle's"
    dt = t["compress_s"] + t["sort_s"]
    return {"value": n_sample / dt, "unit": "keys/s", "cores": threads,
            "kind": "row-column sort (Appendix A) + PEXT compression (Sec. 5.1)",
            "sample": f"first {n_sample} rows; compress {t['compress_s']:.3f} s + sort {t['sort_s']:.3f} s "
                      f"(C = {t['cache_bytes']} B per thread)", **host_cpu()}


def cpu_gnu(rows_all, n_sample, d, perm_ref):
    """The GCC parallel-mode sort on the host cores, same sample: of the full
    keys (memcmp, record-ID ties), and of the compressed records after the
    same compression."""
    from paper_2009_11543_amd import rowcol
    rows = np.ascontiguousarray(rows_all[:n_sample])
    threads = min(16, os.cpu_count() or 1)
    pf, sf = rowcol.gnu_full_sort(rows, rows.shape[1], threads=threads)
    assert np.array_equal(pf, perm_ref), "full-key parallel sort order differs from the oracle's"
    pc, _, t = rowcol.gnu_compress_sort(rows, d, threads=threads)
    assert np.array_equal(pc, perm_ref), "compressed parallel sort order differs from the oracle's"
    dt = t["compress_s"] + t["sort_s"]
    return {"full_keys": {"value": n_sample / sf, "unit": "keys/s", "seconds": sf},
            "compressed": {"value": n_sample / dt, "unit": "keys/s", "compress_s": t["compress_s"],
                           "sort_s": t["sort_s"]},
            "cores": threads, "kind": "__gnu_parallel::sort (OpenMP)", "sample": f"first {n_sample} rows",
            **host_cpu()}


def bench_table(args, torch, ckey, prof, dev):
    """Rebuild of all eight indexes of a 2^24-row table (refresh with the
    current D-bitmaps; radix sorts): eight separate calls, one batched call
    (indexes on forked streams), and a replay of the captured graph."""
    from paper_2009_11543_amd import datagen
    n = 1 << 24
    log("generating the 8-index table")
    tab = datagen.table_indexes(n, seed=1)
    keys = {k: ckey.DeviceKeys(torch.from_numpy(v).to(dev)) for k, v in tab.items()}
    widths = {k: v.shape[1] for k, v in tab.items()}
    del tab
    first = ckey.ckey_rebuild_index([{"keys": kk, "bitmap": None} for kk in keys.values()])
    bms = {k: o["bitmap"].cpu().numpy() for k, o in zip(keys, first)}
    dbits = {k: ckey.ckey_plan_query(b)["nbits"] for k, b in bms.items()}
    log(f"|D| per index: {dbits}")
    specs = [{"keys": keys[k], "bitmap": bms[k]} for k in keys]

    def timeit(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    wss = [torch.empty(ckey.ckey_rebuild_index_workspace([sp]), dtype=torch.uint8, device=dev)
           for sp in specs]
    seq_ms = timeit(lambda: [ckey.ckey_rebuild_index([sp], workspace=w) for sp, w in zip(specs, wss)],
                    args.steps)
    wsb = torch.empty(ckey.ckey_rebuild_index_workspace(specs), dtype=torch.uint8, device=dev)
    bat_ms = timeit(lambda: ckey.ckey_rebuild_index(specs, workspace=wsb), args.steps)
    g = ckey.RebuildGraph(specs)
    graph_ms = timeit(g.launch, args.steps)
    for (k, _), o in zip(keys.items(), g.outs):  # refreshed bitmaps equal the first build's
        assert np.array_equal(o["bitmap"].cpu().numpy(), bms[k]), k

    # Autotuned per-index options: radix digit widths and pass tiles, and the
    # splitter and learned bucketing sorts at two bucket counts (mean buckets
    # of 4096 and 2048 rows) and the in-LDS capacities that hold them, with
    # models fitted to the sorted compressed keys of the index's previous
    # rebuild; each index gets its fastest option.  The tuned table is then
    # also captured in one graph (the bucketing sorts decide overflow on the
    # device).
    from paper_2009_11543_amd import tune
    b_hi = max(8, min(16, n.bit_length() - 1 - 12))
    tuned, choices, models = [], {}, []
    for k, sp in zip(keys, specs):
        prev = ckey.ckey_rebuild_index([dict(sp, want_ckeys=True)])[0]
        ms_k = tune.fit_models(prev["ckeys"][0].contiguous(), (b_hi, min(16, b_hi + 1)), steps=300)
        models.append(ms_k)
        del prev
        choice, rec = tune.autotune(keys[k], bms[k], models=ms_k)
        choices[k] = rec["choice"]
        log(f"  {k}: {len(rec['candidates'])} candidates, fastest {min(rec['times_ms']):.3f} ms: {rec['choice']}")
        tuned.append(dict(sp, opts=choice))
    wst = torch.empty(ckey.ckey_rebuild_index_workspace(tuned), dtype=torch.uint8, device=dev)
    tuned_ms = timeit(lambda: ckey.ckey_rebuild_index(tuned, workspace=wst), args.steps)
    outs_t = ckey.ckey_rebuild_index(tuned, workspace=wst)
    for (k, _), o, og in zip(keys.items(), outs_t, g.outs):  # same results whatever the method
        assert np.array_equal(o["bitmap"].cpu().numpy(), bms[k]), k
        assert o["perm"].equal(og["perm"]), k
    del outs_t
    gt = ckey.RebuildGraph(tuned)
    tuned_graph_ms = timeit(gt.launch, args.steps)
    for (k, _), o, og in zip(keys.items(), gt.outs, g.outs):
        assert np.array_equal(o["bitmap"].cpu().numpy(), bms[k]), k
        assert o["perm"].equal(og["perm"]), k
    names = {ckey.CKEY_SORT_RADIX: "radix", ckey.CKEY_SORT_SPLITTER: "splitter", ckey.CKEY_SORT_LEARNED: "learned"}
    total = 8 * n
    forms = {"graph, radix": graph_ms, "batched call, autotuned options": tuned_ms,
             "graph, autotuned options": tuned_graph_ms}
    launch = min(forms, key=forms.get)
    best_ms = forms[launch]

    def describe(c):
        d = names[c["method"]]
        if c["method"] == ckey.CKEY_SORT_RADIX:
            return d + f" d={c['digit_bits']} tile={c.get('tile', 0)}"
        return d + f" B=2^{c['bucket_log2']} tile={c.get('tile', 0)}"
    out = {"metric": "table rebuild rows/s (8 indexes x 2^24 rows, D-bitmap refresh)",
           "value": total / (best_ms / 1e3), "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": best_ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "table8_2p24", "key_bytes": widths, "nbits": dbits,
                      "method": "radix d=8" if launch == "graph, radix" else
                      {k: describe(c) for k, c in choices.items()},
                      "launch": launch},
           "sequential_calls_ms": seq_ms, "batched_call_ms": bat_ms, "graph_replay_ms": graph_ms,
           "autotuned_batched_ms": tuned_ms, "autotuned_graph_ms": tuned_graph_ms}
    log(f"table: sequential {seq_ms:.2f} ms, batched {bat_ms:.2f} ms, graph {graph_ms:.2f} ms, "
        f"autotuned {tuned_ms:.2f} ms, autotuned graph {tuned_graph_ms:.2f} ms")
    print(json.dumps(out), flush=True)


def bench_zipf(args, torch, ckey, dev):
    """The paper's sensitivity datasets (Table 4): Zipf(s, n, m) keys, 10^7 rows
    each.  Per dataset: |D| from a full-key first build, the sort key sizes of
    Table 4, and the GPU time of the full-key sort against the compressed key
    sort (compress + radix sort with D), the analogue of the paper's total
    time ratio."""
    from paper_2009_11543_amd import datagen
    n = args.zipf_rows
    rid_bits = max(1, (n - 1).bit_length())

    def ev_time(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows_out = []
    tot_keys, tot_ms = 0, 0.0
    for (ds, s, L, m, full_b, comp_b) in datagen.ZIPF_TABLE4:
        if args.zipf_datasets and ds not in args.zipf_datasets:
            continue
        rows = datagen.zipf_keys(n, s, L, m, seed=1)
        keys = ckey.DeviceKeys(torch.from_numpy(rows).to(dev))
        del rows
        ones = np.full(L, 0xFF, np.uint8)
        wf = (8 * L + 63) // 64
        ckf = torch.empty((wf, n), dtype=torch.int64, device=dev)
        ridf = torch.empty(n, dtype=torch.int32, device=dev)
        wsf = torch.empty(ckey.ckey_sort_workspace(wf, 8 * L, n), dtype=torch.uint8, device=dev)

        def full_sort():
            ckey.ckey_compress(keys, ones, out=ckf, rowids=ridf)
            ckey.ckey_sort(ckf, 8 * L, ridf, workspace=wsf)
        full_ms = ev_time(full_sort, 2)
        d = ckey.ckey_distinction_bits(keys, order=ridf).cpu().numpy()
        del ckf, wsf
        plan = ckey.ckey_plan_query(d)
        nb, w = plan["nbits"], plan["words"]
        ck = torch.empty((w, n), dtype=torch.int64, device=dev)
        rid = torch.empty(n, dtype=torch.int32, device=dev)
        ws = torch.empty(ckey.ckey_sort_workspace(w, nb, n), dtype=torch.uint8, device=dev)

        def comp_sort():
            ckey.ckey_compress_sort(keys, d, out=ck, rowids=rid, workspace=ws)
        comp_ms = ev_time(comp_sort, 3)
        assert torch.equal(rid, ridf), f"Zipf dataset {ds}: compressed order differs"
        # Table 4's compressed sort key: |D| plus the record ID's variant bits,
        # in 8-byte words.  The rid variant bits r of the paper's rows are not
        # given; report the range of r for which |D| reproduces the table.
        ok_r = [r for r in range(0, 65) if -(-(nb + r) // 64) * 8 == comp_b]
        rows_out.append({"dataset": ds, "s": s, "key_bytes": L, "m": m, "nbits": nb,
                         "full_sort_key_bytes": L + 8, "table4_full": full_b,
                         "comp_sort_key_bytes_dense_rid": -(-(nb + rid_bits) // 64) * 8,
                         "table4_comp": comp_b, "rid_bits_matching_table4": [min(ok_r), max(ok_r)] if ok_r else None,
                         "full_key_sort_ms": full_ms, "compressed_sort_ms": comp_ms,
                         "gpu_time_ratio": full_ms / comp_ms})
        log(f"Zipf ds {ds} ({s},{L},{m}): |D|={nb} full {full_ms:.1f} ms comp {comp_ms:.2f} ms "
            f"ratio {full_ms / comp_ms:.1f}")
        tot_keys += n
        tot_ms += comp_ms
        del keys, ck, rid, ws, ridf
        torch.cuda.empty_cache()
    common = None
    for r in rows_out:
        rr = r["rid_bits_matching_table4"]
        if rr is None:
            common = (1, 0)
            break
        common = tuple(rr) if common is None else (max(common[0], rr[0]), min(common[1], rr[1]))
    out = {"metric": "compress+sort keys/s on the Zipf(s,n,m) datasets of Table 4",
           "value": tot_keys / (tot_ms / 1e3), "unit": "keys/s", "n_gpus": 1, "steps": 3,
           "warmup": 1, "ms_per_step": tot_ms / max(1, len(rows_out)), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "zipf_table4", "rows_per_dataset": n, "method": "radix"},
           "datasets": rows_out,
           "rid_bits_matching_every_dataset": None if common is None or common[0] > common[1] else list(common)}
    print(json.dumps(out), flush=True)


def bench_maintenance(torch, ckey, keys, ridf, d_bitmap, dev, batch_rows, model_opts=None,
                      method_name="radix", model_for=None):
    """DS-metadata calls at the workload's size (Sec. 4.3): the variant bitmap,
    a first build that takes the variant bitmap (a sort-free superset of D) in
    place of the all-ones bitmap, and a batched insert into the index."""
    n, L = keys.n, keys.key_bytes

    def ev_time(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    var = {}

    def variant():
        var["v"], var["r"] = ckey.ckey_variant_bitmap(keys)
    ms = ev_time(variant, 5)
    v_host = var["v"].cpu().numpy()
    assert all((int(v) & int(d)) == int(d) for v, d in zip(v_host, d_bitmap)), "variant must cover D"
    out["variant_bitmap"] = {"ms": ms, "gbps_key_bytes": n * L / (ms / 1e3) / 1e9,
                             "popcount": int(np.unpackbits(v_host).sum()),
                             "d_popcount": int(np.unpackbits(np.asarray(d_bitmap)).sum())}
    log(f"variant bitmap: {ms:.3f} ms, |V|={out['variant_bitmap']['popcount']}")

    # A CDF model for keys compressed with the variant bitmap (the first word
    # differs from the D-compressed one), trained like the main one.
    model_opts_v = None
    vname = "radix"
    if model_opts is not None and model_for is not None:
        model_opts_v = dict(model_opts)
        model_opts_v["model"] = model_for(v_host)
        vname = method_name

    res = {}

    def first_build():
        res["o"] = ckey.ckey_rebuild_index([{"keys": keys, "bitmap": v_host, "opts": model_opts_v}])[0]
    ms_fb = ev_time(first_build, 2)
    assert torch.equal(res["o"]["perm"], ridf), "first build from the variant bitmap: order differs"
    assert (res["o"]["bitmap"].cpu().numpy() == d_bitmap).all(), "first build: D differs"
    out["first_build_from_variant"] = {
        "ms": ms_fb + ms, "keys_per_s": n / ((ms_fb + ms) / 1e3),
        "what": f"ckey_variant_bitmap + ckey_rebuild_index(bitmap = variant, {vname}): perm and exact D"}
    log(f"first build via variant bitmap: {ms_fb + ms:.2f} ms")
    del res

    # Index reconstruction end to end (Sec. 5): a rebuild (compress, sort,
    # refreshed D, per-pair positions), then the tree (Sec. 5.3).  Partial-key
    # bits outside the compression bitmap are either read from the key by
    # record ID (option b, compression bitmap D) or not needed because the
    # compression bitmap is the variant bitmap, a superset of D that sorts the
    # same (option a).
    shape = ckey.ckey_tree_plan(n, 0.9)
    recon = {"tree_height": shape["height"], "tree_nodes": shape["total_nodes"]}
    tree = {}
    for label, cbm, mo, mname in (("option_b_D", np.asarray(d_bitmap), model_opts, method_name),
                                  ("option_a_variant", v_host, model_opts_v, vname)):
        rb = {}

        def rebuild():
            rb["o"] = ckey.ckey_rebuild_index([{"keys": keys, "bitmap": cbm, "want_pair_pos": True,
                                                "want_ckeys": True, "opts": mo}])[0]
        ms_rb = ev_time(rebuild, 3)
        o = rb["o"]
        assert torch.equal(o["perm"], ridf)
        assert (o["bitmap"].cpu().numpy() == d_bitmap).all()

        def bulk():
            tree["nodes"], tree["deref"] = ckey.ckey_bulk_load(keys, o["perm"], o["ckeys"], cbm, o["pair_pos"],
                                                               pk=32, fill=0.9, variant=v_host, ref=var["r"],
                                                               nodes=tree.get("nodes"))
        ms_bl = ev_time(bulk, 3)
        recon[label] = {"rebuild_ms": ms_rb, "bulk_load_ms": ms_bl, "total_ms": ms_rb + ms_bl,
                        "keys_per_s": n / ((ms_rb + ms_bl) / 1e3), "sort": mname,
                        "entries_reading_their_key": int(tree["deref"].item())}
        log(f"index reconstruction ({label}): rebuild {ms_rb:.2f} ms + bulk load {ms_bl:.2f} ms")
        del rb, o
    del tree
    recon["what"] = ("ckey_rebuild_index + ckey_bulk_load (pk 32, fill 0.9, variant bitmap and reference key); "
                     "option_b_D: compression bitmap D, partial-key bits outside it read by record ID; "
                     "option_a_variant: compression bitmap = variant bitmap")
    out["index_reconstruction"] = recon

    bk = ckey.DeviceKeys(torch.from_numpy(batch_rows).to(dev))
    dbm = torch.from_numpy(np.asarray(d_bitmap).copy()).to(dev)

    def insert():
        ckey.ckey_insert_keys(keys, ridf, bk, dbm)
    ms_in = ev_time(insert, 5)
    got = dbm.cpu().numpy()
    assert all((int(g) & int(d)) == int(d) for g, d in zip(got, d_bitmap))
    out["insert_batch"] = {"ms": ms_in, "batch": int(bk.n), "index": n,
                           "keys_per_s": bk.n / (ms_in / 1e3),
                           "what": "ckey_insert_keys: batch full-key sort, binary search, new pairs' D-bits"}
    log(f"insert {bk.n} keys into {n}: {ms_in:.3f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dna64_2p26")
    ap.add_argument("--method", default="auto", choices=["auto", "radix", "splitter", "learned"],
                    help="sort method for the timed steps; auto = the fastest after calibration")
    ap.add_argument("--bucket-log2", type=int, default=0,
                    help="log2 bucket count; 0 = about 4096 rows per bucket (2^14 at 2^26 rows)")
    ap.add_argument("--train-rows", type=int, default=1 << 24)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-key", action="store_true")
    ap.add_argument("--no-maintenance", action="store_true")
    ap.add_argument("--zipf-rows", type=int, default=10_000_000)
    ap.add_argument("--zipf-datasets", type=int, nargs="*", default=None,
                    help="Table 4 dataset numbers for --workload zipf_table4 (default all)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_11543_amd import ckey
    prof = Prof(ckey.lib())
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.workload.startswith("table8"):
        return bench_table(args, torch, ckey, prof, dev)
    if args.workload == "zipf_table4":
        return bench_zipf(args, torch, ckey, dev)
    log(f"generating workload {args.workload}")
    rows, desc = workload(args.workload)
    lens = None
    if isinstance(rows, tuple):  # varchar keys: the zero-padded rows serve the host baselines
        rows, lens = rows
    n, L = rows.shape
    if lens is None:
        keys = ckey.DeviceKeys(torch.from_numpy(rows).to(dev))
    else:
        from paper_2009_11543_amd import datagen
        flat, offs = datagen.pack_varlen(rows, lens)
        keys = ckey.DeviceKeys.from_numpy(flat, key_bytes=L, offsets=offs)
        del flat, offs
    torch.cuda.synchronize()
    log(f"keys resident: n={n} L={L}")
    if args.bucket_log2 == 0:
        args.bucket_log2 = max(8, min(16, n.bit_length() - 1 - 12))

    # copy probe: achievable HBM bandwidth
    buf_a = torch.empty(1 << 31, dtype=torch.uint8, device=dev)
    buf_b = torch.empty_like(buf_a)
    lib = ckey.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(2):
        lib.ckey_bench_copy(buf_b.data_ptr(), buf_a.data_ptr(), buf_a.numel(), st)
    prof.on()
    for _ in range(5):
        lib.ckey_bench_copy(buf_b.data_ptr(), buf_a.data_ptr(), buf_a.numel(), st)
    cms, cnt = prof.read("stream_copy")
    copy_gbps = 2 * buf_a.numel() / (cms / cnt / 1e3) / 1e9
    prof.on(False)
    del buf_a, buf_b
    log(f"copy probe: {copy_gbps:.0f} GB/s")

    # First build over full keys: the plain full-key GPU radix sort (timed as a
    # baseline) and D from its order (Sec. 4.3, first build).
    ones = np.full(L, 0xFF, np.uint8)
    wf = (8 * L + 63) // 64
    ckf = torch.empty((wf, n), dtype=torch.int64, device=dev)
    ridf = torch.empty(n, dtype=torch.int32, device=dev)
    wsf = torch.empty(ckey.ckey_sort_workspace(wf, 8 * L, n), dtype=torch.uint8, device=dev)
    full = None
    reps = 0 if args.no_full_key else 2
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ckey.ckey_compress(keys, ones, out=ckf, rowids=ridf)
        ckey.ckey_sort(ckf, 8 * L, ridf, workspace=wsf)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if r > 0:
            full = dt if full is None else min(full, dt)
        log(f"full-key sort rep {r}: {dt * 1e3:.1f} ms")
    # The same with passes over digits equal in every row skipped (found from
    # the upfront histograms: one stream synchronization).
    full_skip = None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ckey.ckey_compress(keys, ones, out=ckf, rowids=ridf)
        ckey.ckey_sort(ckf, 8 * L, ridf, workspace=wsf, skip_trivial=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if r > 0:
            full_skip = dt if full_skip is None else min(full_skip, dt)
    if full_skip is not None:
        log(f"full-key sort skipping trivial passes: {full_skip * 1e3:.1f} ms")
    d_bitmap = ckey.ckey_distinction_bits(keys, order=ridf).cpu().numpy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        ckey.ckey_distinction_bits(keys, order=ridf)
    torch.cuda.synchronize()
    dbits_ms = (time.perf_counter() - t0) / 3 * 1e3
    log(f"D-bitmap from the full-key order: {dbits_ms:.2f} ms")
    del ckf, wsf
    plan = ckey.ckey_plan_query(d_bitmap)
    nbits, w = plan["nbits"], plan["words"]
    log(f"|D|={nbits} words={w} windows={len(plan['windows'])}")

    # CDF model: trained on the sorted compressed keys of a rebuild of the same
    # generator at another seed, compressed with this D-bitmap.
    model = None
    if args.method in ("auto", "splitter", "learned"):
        from paper_2009_11543_amd import datagen
        log(f"training rebuild: {args.train_rows} rows, seed 2")
        rows_t = training_rows(args.workload, min(args.train_rows, n))
        keys_t = ckey.DeviceKeys(torch.from_numpy(rows_t).to(dev))
        del rows_t
        ckt, ridt = ckey.ckey_compress(keys_t, d_bitmap)
        ckey.ckey_sort(ckt, nbits, ridt)
        model = ckey.CdfModel(bucket_log2=args.bucket_log2, seed=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trace = ckey.ckey_cdf_fit(model, ckt[0].contiguous(), steps=args.train_steps, batch=1 << 16)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        trace = trace.cpu().numpy()
        del ckt, ridt, keys_t
        log(f"trained {args.train_steps} steps in {train_s:.2f} s; loss {trace[0]:.3e} -> {trace[-1]:.3e}")

    ck = torch.empty((w, n), dtype=torch.int64, device=dev)
    rid = torch.empty(n, dtype=torch.int32, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    method_opts = {"radix": dict(method=ckey.CKEY_SORT_RADIX)}
    if model is not None:
        method_opts["splitter"] = dict(method=ckey.CKEY_SORT_SPLITTER, model=model)
        method_opts["learned"] = dict(method=ckey.CKEY_SORT_LEARNED, model=model)
    cand = list(method_opts) if args.method == "auto" else [args.method]
    ws = torch.empty(max(ckey.ckey_sort_workspace(w, nbits, n, **method_opts[m]) for m in cand),
                     dtype=torch.uint8, device=dev)

    def step(m):
        ckey.ckey_compress_sort(keys, d_bitmap, out=ck, rowids=rid, workspace=ws, flags=flags,
                                **method_opts[m])

    def timed(m, steps):
        # The step time with the per-kernel event timing off (an event between
        # consecutive steps: the median step, and the mean over the region);
        # then the same steps again with it on, for the per-kernel times.
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(steps):
            step(m)
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        ms = float(np.median(per))
        timed.mean_ms = ev[0].elapsed_time(ev[steps]) / steps
        prof.on()
        for _ in range(steps):
            step(m)
        torch.cuda.synchronize()
        kern = {}
        for name in KERNEL_BYTES:
            t, c = prof.read(name)
            if c:
                kern[name] = {"ms_per_step": t / steps, "launches_per_step": c / steps,
                              "ms_per_launch": t / c}
        prof.on(False)
        return ms, kern

    results = {}
    for m in cand:
        for _ in range(args.warmup):
            step(m)
        torch.cuda.synchronize()
        assert torch.equal(rid, ridf), f"{m}: compressed-key order differs from full-key order"
        results[m] = timed(m, args.steps if len(cand) == 1 else max(3, args.steps // 2))
        log(f"{m}: {results[m][0]:.3f} ms/step; permutation equals the full-key order")
    best = min(results, key=lambda m: results[m][0])
    if len(cand) > 1:  # the timed region proper, on the chosen method
        for _ in range(args.warmup):
            step(best)
        results[best] = timed(best, args.steps)
    ms, kern = results[best]
    mean_ms = timed.mean_ms
    log(f"chosen {best}: {ms:.3f} ms/step (median; mean {mean_ms:.3f}); kernels {json.dumps(kern)}")
    assert int(flags.item()) & ckey.CKEY_FLAG_SPIN_LIMIT == 0

    # Algorithmic bytes per key of each kernel: what it must read and write once.
    key_bytes_read = len({b for s, _ in plan["windows"] for b in range(s, min(s + 8, L))})
    if lens is not None:  # varchar keys are staged whole, with their 8-byte offsets
        key_bytes_read = float(lens.mean()) + 8
    rec = 8 * w + 4
    # compress_bucket writes words + bucket id (the first bucket pass generates
    # the record IDs); the two bucket passes move rec + 2 bytes in and out,
    # less the record IDs pass 1 does not read, plus pass 1's bucket-id copy.
    # (the bucketing methods' compression writes no record IDs)
    # Kernel bytes as implemented (what each launch moves once) ...
    per_key = {"compress": key_bytes_read + (rec if best == "radix" else 8 * w),
               "compress_bucket": key_bytes_read + 8 * w + 2,
               "hist": 8 * w, "onesweep": 2 * rec,
               "assign_learned": 8 + 2, "assign_splitter": 8 + 2, "tile_counts": 2,
               "bucket_pass": 2 * rec,
               "bucket_sort": 2 * rec}
    moved_bytes = sum(per_key[k] * n * v["launches_per_step"] for k, v in kern.items())
    # ... and the method's bytes per key, which the GB/s figure is taken from:
    # key bytes read + compressed record written + (radix) one histogram read
    # of the words and a read and a write of every record per pass, or
    # (bucketing) a read of the first word for the bucket, the one scatter of
    # every record into its bucket, and the bucket sort's read and write.
    if best == "radix":
        npass = sum(-(-min(64, nbits - 64 * k) // 8) for k in range(w) if nbits > 64 * k)
        method_key = key_bytes_read + rec + 8 * w + 2 * npass * rec
    else:
        method_key = key_bytes_read + rec + 8 + 2 * rec + 2 * rec
    step_bytes = method_key * n
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    dom_bytes = per_key[dom] * n
    achieved = dom_bytes / (kern[dom]["ms_per_launch"] / 1e3) / 1e9
    src = os.path.join(ROOT, "paper_2009_11543_amd", "csrc",
                       "k_radix.hip" if dom in ("onesweep", "hist", "bucket_pass") else
                       "k_compress.hip" if dom in ("compress", "compress_bucket") else "k_learned.hip")
    traffic = traffic_for(dom, args.workload, src)

    out = {
        "metric": METRIC, "value": n / (ms / 1e3), "unit": "keys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "key_bytes": L,
                   "nbits": nbits, "words": w, "method": best,
                   "bucket_log2": args.bucket_log2 if best != "radix" else None,
                   "digit_bits": 8 if best == "radix" else None},
        "ms_per_step_mean": mean_ms,
        "hbm_gbps_algorithmic": step_bytes / (ms / 1e3) / 1e9,
        "bytes_per_key_algorithmic": step_bytes / n,
        "hbm_gbps_moved": moved_bytes / (ms / 1e3) / 1e9,
        "bytes_per_key_moved": moved_bytes / n,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved,
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS,
                     "traffic": traffic, "bytes_per_launch_algorithmic": dom_bytes,
                     "ms_per_launch": kern[dom]["ms_per_launch"], "copy_probe_gbps": copy_gbps},
        "kernels": kern,
        "methods_ms_per_step": {m: results[m][0] for m in results},
        "distinction_bits_ms": dbits_ms,
        "training": None if model is None else {"rows": args.train_rows, "seed": 2,
                                                "steps": args.train_steps, "batch": 1 << 16,
                                                "seconds": train_s, "loss_first": float(trace[0]),
                                                "loss_last": float(trace[-1])},
        "full_key_gpu": None if full is None else {
            "ms_per_step": full * 1e3, "keys_per_s": n / full,
            "speedup_of_compressed": full * 1e3 / ms,
            "speedup_of_compressed_radix": full * 1e3 / results["radix"][0] if "radix" in results else None,
            "what": "ckey_compress with an all-ones bitmap + ckey_sort over all 8L bits",
            "skip_trivial_ms_per_step": None if full_skip is None else full_skip * 1e3,
            "speedup_of_compressed_vs_skip": None if full_skip is None else full_skip * 1e3 / ms},
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_maintenance and full is not None:
        del ck, ws
        mo = None
        model_for = None
        if best != "radix":
            mo = dict(method_opts[best])

            def model_for(bitmap):
                rows_t = training_rows(args.workload, min(args.train_rows, n))
                kt = ckey.DeviceKeys(torch.from_numpy(rows_t).to(dev))
                del rows_t
                ckt, ridt = ckey.ckey_compress(kt, bitmap)
                ckey.ckey_sort(ckt, ckey.ckey_plan_query(bitmap)["nbits"], ridt)
                mv = ckey.CdfModel(bucket_log2=args.bucket_log2, seed=3)
                ckey.ckey_cdf_fit(mv, ckt[0].contiguous(), steps=args.train_steps, batch=1 << 16)
                return mv
        out["maintenance"] = bench_maintenance(torch, ckey, keys, ridf, d_bitmap, dev,
                                               training_rows(args.workload, 1 << 16, seed=5), mo, best,
                                               model_for)
    if not args.no_cpu_baseline:
        log(f"cpu baseline on {args.cpu_sample} rows")
        out["cpu_baseline"], d_s, perm_s = cpu_baseline(rows, min(args.cpu_sample, n))
        out["cpu_rowcol"] = cpu_rowcol(rows, min(args.cpu_sample, n), d_s, perm_s)
        log(f"cpu row-column: {out['cpu_rowcol']['value'] / 1e6:.1f} M keys/s on {out['cpu_rowcol']['cores']} threads")
        out["cpu_gnu_parallel"] = cpu_gnu(rows, min(args.cpu_sample, n), d_s, perm_s)
        g = out["cpu_gnu_parallel"]
        log(f"cpu gnu parallel sort: full keys {g['full_keys']['value'] / 1e6:.1f}, compressed "
            f"{g['compressed']['value'] / 1e6:.1f} M keys/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
