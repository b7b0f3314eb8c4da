// C ABI entry points of libckey.so: argument checks, planning and workspace
// layout on the host; all per-key work is enqueued as HIP kernels.
#include <string.h>

#include <mutex>
#include <vector>

#include "internal.h"

using namespace ckey;

namespace {

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

ckey_status check_keys(const ckey_keys *k) {
    if (!k) return CKEY_ERR_INVALID;
    if (k->key_bytes == 0) return CKEY_ERR_INVALID;
    if (k->key_bytes > CKEY_MAX_KEY_BYTES) return CKEY_ERR_UNSUPPORTED;
    if (k->n > CKEY_MAX_ROWS) return CKEY_ERR_UNSUPPORTED;
    if (k->n > 0 && !k->bytes) return CKEY_ERR_INVALID;
    if (!k->offsets && k->stride < k->key_bytes) return CKEY_ERR_INVALID;
    return CKEY_OK;
}

KeySrc key_src(const ckey_keys *k) {
    return KeySrc{k->bytes, k->offsets, k->n, k->key_bytes, k->stride};
}

uint32_t popcount_bitmap(const uint8_t *bm, uint32_t L) {
    uint32_t c = 0;
    for (uint32_t j = 0; j < L; ++j) c += __builtin_popcount(bm[j]);
    return c;
}

uint32_t words_for(uint32_t nbits) { return nbits ? (nbits + 63) / 64 : 1; }

ckey_status ws_check(void *ws, size_t *ws_bytes, size_t need, bool &query) {
    if (!ws_bytes) return CKEY_ERR_INVALID;
    if (!ws) {
        *ws_bytes = need;
        query = true;
        return CKEY_OK;
    }
    query = false;
    if (*ws_bytes < need) return CKEY_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return CKEY_ERR_INVALID;
    return CKEY_OK;
}

uint32_t digit_bits_of(const ckey_sort_opts *o) {
    uint32_t d = o ? o->digit_bits : 0;
    return d == 0 ? 8 : d;
}

uint32_t method_of(const ckey_sort_opts *o) { return o ? o->method : uint32_t(CKEY_SORT_RADIX); }

ckey_status check_sort_opts(const ckey_sort_opts *o, bool need_model) {
    const uint32_t m = method_of(o);
    if (m == CKEY_SORT_RADIX) {
        const uint32_t d = digit_bits_of(o);
        return (d >= 1 && d <= 8) ? CKEY_OK : CKEY_ERR_INVALID;
    }
    if (m != CKEY_SORT_LEARNED && m != CKEY_SORT_SPLITTER) return CKEY_ERR_INVALID;
    if (!learned_b_ok(o->bucket_log2)) return CKEY_ERR_INVALID;
    if (need_model && !o->model) return CKEY_ERR_INVALID;
    return CKEY_OK;
}

size_t sort_workspace(const ckey_sort_opts *o, uint32_t words, uint32_t nbits, uint64_t n) {
    if (method_of(o) == CKEY_SORT_RADIX) return radix_workspace(words, nbits, n, digit_bits_of(o));
    return learned_workspace(words, nbits, n, o->bucket_log2);
}

// skip_ok: the caller allows the radix sort's trivial-pass skip (a stream
// synchronization), i.e. it is ckey_sort / ckey_compress_sort, not a rebuild.
ckey_status sort_dispatch(const ckey_sort_opts *o, uint64_t *ck, uint32_t words, uint32_t nbits,
                          uint32_t *rid, uint64_t n, uint32_t *flags, void *ws, hipStream_t st,
                          bool skip_ok = false) {
    const uint32_t m = method_of(o);
    if (m == CKEY_SORT_RADIX)
        return radix_sort(ck, n, words, nbits, rid, n, digit_bits_of(o), 0, flags, ws, st,
                          skip_ok && o && o->skip_trivial);
    return learned_sort(ck, words, nbits, rid, n, m == CKEY_SORT_LEARNED ? 1 : 0, o->model,
                        o->bucket_log2, flags, ws, st);
}

// Compress then sort; for the bucketing methods the bucket of each key is
// found while it is compressed when the keys allow the fused kernel.
ckey_status compress_sort_dispatch(const ckey_sort_opts *o, const KeySrc &k, const uint8_t *bm,
                                   uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid,
                                   uint32_t *flags, void *ws, hipStream_t st, bool skip_ok = false) {
    const uint32_t m = method_of(o);
    if (m != CKEY_SORT_RADIX) {
        const ckey_status s = compress_learned_sort(k, bm, ck, words, nbits, rid,
                                                    m == CKEY_SORT_LEARNED ? 1 : 0, o->model,
                                                    o->bucket_log2, flags, ws, st);
        if (s != CKEY_ERR_UNSUPPORTED) return s;
    }
    CKEY_TRY(compress_launch(k, bm, ck, words, rid, flags, st));
    return sort_dispatch(o, ck, words, nbits, rid, k.n, flags, ws, st, skip_ok);
}

struct IndexPlan {
    std::vector<uint8_t> bm;  // bitmap used (all ones for a first build)
    uint32_t nbits, words;
    size_t off, bytes;        // this index's workspace part
};

struct RebuildPlan {
    std::vector<IndexPlan> ix;
    size_t total = 0;
};

ckey_status plan_rebuild(const ckey_index_desc *idx, uint32_t count, const ckey_sort_opts *opts,
                         bool real_call, RebuildPlan &plan) {
    if (!idx || count == 0) return CKEY_ERR_INVALID;
    plan.ix.resize(count);
    plan.total = 0;
    for (uint32_t x = 0; x < count; ++x) {
        const ckey_index_desc &D = idx[x];
        const ckey_sort_opts *o = D.opts ? D.opts : opts;
        CKEY_TRY(check_sort_opts(o, real_call));
        CKEY_TRY(check_keys(&D.keys));
        if (real_call && D.keys.n > 0 && !D.perm) return CKEY_ERR_INVALID;
        IndexPlan &P = plan.ix[x];
        const uint32_t L = D.keys.key_bytes;
        P.bm.assign(L, 0xFF);  // first build: every position (Sec. 4.3)
        if (D.bitmap_in) memcpy(P.bm.data(), D.bitmap_in, L);
        P.nbits = popcount_bitmap(P.bm.data(), L);
        P.words = words_for(P.nbits);
        const uint64_t n = D.keys.n;
        size_t s = align256((L + 3) / 4 * 4);
        if (!D.ckeys) s += align256(size_t(P.words) * n * 8);
        s += sort_workspace(o, P.words, P.nbits, n);
        P.bytes = s;
        // one index: the parts share offset 0; several: each its own part
        P.off = count == 1 ? 0 : plan.total;
        plan.total = count == 1 ? s : plan.total + align256(s);
    }
    return CKEY_OK;
}

ckey_status enqueue_one(const ckey_index_desc &D, const ckey_sort_opts *o, const IndexPlan &P,
                        uint8_t *ws, hipStream_t st) {
    const uint32_t L = D.keys.key_bytes;
    const uint64_t n = D.keys.n;
    uint8_t *p = ws + P.off;
    uint32_t *acc = reinterpret_cast<uint32_t *>(p);
    p += align256((L + 3) / 4 * 4);
    uint64_t *ck = D.ckeys;
    if (!ck) {
        ck = reinterpret_cast<uint64_t *>(p);
        p += align256(size_t(P.words) * n * 8);
    }
    uint32_t *flags = D.flags ? D.flags : (o ? o->flags : nullptr);
    CKEY_TRY(compress_sort_dispatch(o, key_src(&D.keys), P.bm.data(), ck, P.words, P.nbits, D.perm,
                                    flags, p, st));
    if (D.bitmap_out || D.pair_pos) {
        CKEY_TRY(fill_u32(acc, (L + 3) / 4, 0, st));
        CKEY_TRY(refine_launch(ck, P.words, n, P.bm.data(), L, acc, D.pair_pos, flags, st));
        if (D.bitmap_out) CKEY_TRY(bitmap_finalize(acc, D.bitmap_out, L, st));
    }
    return CKEY_OK;
}

constexpr bool kFusedTableEnabled = false;

// The whole table in one persistent launch (opts->fused_table): every index
// radix-sorted, key_bytes and pass count within the persistent kernel's limits.
// ws == nullptr: the workspace size into *ws_bytes.
ckey_status fused_rebuild(const ckey_index_desc *idx, uint32_t count, const ckey_sort_opts *opts,
                          bool real_call, void *ws, size_t *ws_bytes, hipStream_t st) {
    if (!idx || count == 0 || !ws_bytes) return CKEY_ERR_INVALID;
    if (count > CKEY_TABLE_MAX_INDEXES) return CKEY_ERR_UNSUPPORTED;
    TableIndex ti[CKEY_TABLE_MAX_INDEXES];
    uint8_t bms[CKEY_TABLE_MAX_INDEXES][CKEY_TABLE_MAX_KEY_BYTES];
    for (uint32_t x = 0; x < count; ++x) {
        const ckey_index_desc &D = idx[x];
        const ckey_sort_opts *o = D.opts ? D.opts : opts;
        CKEY_TRY(check_sort_opts(o, false));
        if (method_of(o) != CKEY_SORT_RADIX) return CKEY_ERR_UNSUPPORTED;
        CKEY_TRY(check_keys(&D.keys));
        const uint32_t L = D.keys.key_bytes;
        if (L > CKEY_TABLE_MAX_KEY_BYTES) return CKEY_ERR_UNSUPPORTED;
        if (real_call && D.keys.n > 0 && !D.perm) return CKEY_ERR_INVALID;
        memset(bms[x], 0xFF, L);  // first build: every position (Sec. 4.3)
        if (D.bitmap_in) memcpy(bms[x], D.bitmap_in, L);
        ti[x] = TableIndex{key_src(&D.keys), bms[x], digit_bits_of(o), D.perm, D.ckeys, D.pair_pos,
                           D.bitmap_out, D.flags ? D.flags : (o ? o->flags : nullptr)};
    }
    size_t need = 0;
    CKEY_TRY(table_fused_plan(ti, count, nullptr, &need, st));
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, need, query));
    if (query) return CKEY_OK;
    // Switched off: the persistent kernel's first run on the GPU ended in a
    // memory fault whose cause is not found (a host emulation of the same
    // kernel source shows no out-of-bounds access and the oracle's results).
    // Queries and argument checks stay; the launch is refused.
    if (!kFusedTableEnabled) return CKEY_ERR_UNSUPPORTED;
    return table_fused_plan(ti, count, ws, &need, st);
}

// Streams and events for fanning a table's indexes out from the caller's
// stream (created once, default priority, kept for the process lifetime).
constexpr int kForkStreams = 8;
std::mutex g_fork_mu;
hipStream_t g_fork[kForkStreams];
hipEvent_t g_fork_ev[kForkStreams + 1];
int g_fork_dev = -1;

ckey_status fork_resources() {
    int dev = 0;
    CKEY_HIP_TRY(hipGetDevice(&dev));
    if (g_fork_dev == dev) return CKEY_OK;
    if (g_fork_dev >= 0) return CKEY_ERR_UNSUPPORTED;  // one device per process
    for (int i = 0; i < kForkStreams; ++i)
        CKEY_HIP_TRY(hipStreamCreateWithFlags(&g_fork[i], hipStreamNonBlocking));
    for (int i = 0; i <= kForkStreams; ++i)
        CKEY_HIP_TRY(hipEventCreateWithFlags(&g_fork_ev[i], hipEventDisableTiming));
    g_fork_dev = dev;
    return CKEY_OK;
}

ckey_status enqueue_rebuild(const ckey_index_desc *idx, uint32_t count, const ckey_sort_opts *opts,
                            const RebuildPlan &plan, void *ws, hipStream_t st) {
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    if (count == 1) return enqueue_one(idx[0], idx[0].opts ? idx[0].opts : opts, plan.ix[0], w8, st);
    std::lock_guard<std::mutex> g(g_fork_mu);
    CKEY_TRY(fork_resources());
    CKEY_HIP_TRY(hipEventRecord(g_fork_ev[kForkStreams], st));
    const int ns = int(count < uint32_t(kForkStreams) ? count : kForkStreams);
    for (int i = 0; i < ns; ++i) CKEY_HIP_TRY(hipStreamWaitEvent(g_fork[i], g_fork_ev[kForkStreams], 0));
    // Radix indexes first: they enqueue without waiting, so they run while a
    // bucketing index's host synchronization (its overflow count) holds the
    // enqueue loop.
    ckey_status status = CKEY_OK;
    for (int pass = 0; pass < 2 && status == CKEY_OK; ++pass)
        for (uint32_t x = 0; x < count && status == CKEY_OK; ++x) {
            const ckey_sort_opts *o = idx[x].opts ? idx[x].opts : opts;
            if ((method_of(o) == CKEY_SORT_RADIX) != (pass == 0)) continue;
            status = enqueue_one(idx[x], o, plan.ix[x], w8, g_fork[x % kForkStreams]);
        }
    // Joined back even after an error, so the caller's stream still orders
    // after whatever was enqueued on the forks.
    for (int i = 0; i < ns; ++i) {
        CKEY_HIP_TRY(hipEventRecord(g_fork_ev[i], g_fork[i]));
        CKEY_HIP_TRY(hipStreamWaitEvent(st, g_fork_ev[i], 0));
    }
    return status;
}

}  // namespace

extern "C" {

const char *ckey_status_string(ckey_status s) {
    switch (s) {
        case CKEY_OK: return "ok";
        case CKEY_ERR_INVALID: return "invalid argument";
        case CKEY_ERR_UNSUPPORTED: return "unsupported (beyond library limits)";
        case CKEY_ERR_WORKSPACE: return "workspace too small";
        case CKEY_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

ckey_status ckey_plan_query(const uint8_t *bitmap, uint32_t L, uint32_t *nbits, uint32_t *words,
                            uint32_t *windows, uint32_t *window_start, uint64_t *window_mask,
                            uint32_t max_windows) {
    if (!bitmap || L == 0) return CKEY_ERR_INVALID;
    if (L > CKEY_MAX_KEY_BYTES) return CKEY_ERR_UNSUPPORTED;
    const uint32_t nb = popcount_bitmap(bitmap, L);
    if (nbits) *nbits = nb;
    if (words) *words = words_for(nb);
    // Sec. 5.1: each 8-byte mask starts at the byte holding the next 1 that
    // the previous mask does not cover.
    uint32_t nw = 0;
    for (uint32_t j = 0; j < L;) {
        if (!bitmap[j]) { ++j; continue; }
        uint64_t m = 0;
        for (uint32_t t = 0; t < 8; ++t) m = (m << 8) | (j + t < L ? bitmap[j + t] : 0u);
        if (nw < max_windows) {
            if (window_start) window_start[nw] = j;
            if (window_mask) window_mask[nw] = m;
        }
        ++nw;
        j += 8;
    }
    if (windows) *windows = nw;
    return CKEY_OK;
}

ckey_status ckey_distinction_bits(const ckey_keys *keys, const uint32_t *order, uint8_t *bitmap,
                                  uint32_t *flags, void *ws, size_t *ws_bytes, void *stream) {
    CKEY_TRY(check_keys(keys));
    const uint32_t nw = (keys->key_bytes + 3) / 4;
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, align256(nw * 4), query));
    if (query) return CKEY_OK;
    if (!bitmap) return CKEY_ERR_INVALID;
    hipStream_t st = as_stream(stream);
    uint32_t *acc = static_cast<uint32_t *>(ws);
    CKEY_TRY(fill_u32(acc, nw, 0, st));
    CKEY_TRY(dbits_launch(key_src(keys), order, acc, flags, st));
    return bitmap_finalize(acc, bitmap, keys->key_bytes, st);
}

ckey_status ckey_variant_bitmap(const ckey_keys *keys, const uint8_t *ref, uint8_t *variant,
                                uint8_t *ref_out, uint32_t *flags, void *ws, size_t *ws_bytes,
                                void *stream) {
    CKEY_TRY(check_keys(keys));
    const uint32_t nw = (keys->key_bytes + 3) / 4;
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, align256(nw * 4), query));
    if (query) return CKEY_OK;
    if (!variant) return CKEY_ERR_INVALID;
    hipStream_t st = as_stream(stream);
    uint32_t *acc = static_cast<uint32_t *>(ws);
    const KeySrc k = key_src(keys);
    CKEY_TRY(fill_u32(acc, nw, 0, st));
    CKEY_TRY(variant_launch(k, ref, acc, flags, st));
    CKEY_TRY(bitmap_finalize(acc, variant, keys->key_bytes, st));
    if (ref_out) {
        if (ref)
            CKEY_HIP_TRY(hipMemcpyAsync(ref_out, ref, keys->key_bytes, hipMemcpyDeviceToDevice, st));
        else
            CKEY_TRY(ref_copy_launch(k, ref_out, st));
    }
    return CKEY_OK;
}

namespace {
struct InsertLayout {
    size_t pos, acc_d, acc_v, ck, rid, sortws, total;
    uint32_t words, nbits;
};

InsertLayout insert_layout(const ckey_keys *batch, bool sort_batch) {
    InsertLayout l{};
    const uint64_t m = batch->n;
    const uint32_t nw = (batch->key_bytes + 3) / 4;
    size_t off = 0;
    l.pos = off;   off += align256(size_t(m) * 4);
    l.acc_d = off; off += align256(nw * 4);
    l.acc_v = off; off += align256(nw * 4);
    if (sort_batch) {  // full-key sort of the batch: compress with every position
        l.nbits = 8 * batch->key_bytes;
        l.words = words_for(l.nbits);
        l.ck = off;  off += align256(size_t(l.words) * m * 8);
        l.rid = off; off += align256(size_t(m) * 4);
        l.sortws = off;
        off += radix_workspace(l.words, l.nbits, m, 8);
    }
    l.total = off;
    return l;
}
}  // namespace

ckey_status ckey_insert_keys(const ckey_keys *index, const uint32_t *index_order,
                             const ckey_keys *batch, const uint32_t *batch_order, uint8_t *dbitmap,
                             uint8_t *variant, const uint8_t *ref, uint32_t *flags, void *ws,
                             size_t *ws_bytes, void *stream) {
    CKEY_TRY(check_keys(index));
    CKEY_TRY(check_keys(batch));
    if (index->key_bytes != batch->key_bytes) return CKEY_ERR_INVALID;
    const InsertLayout l = insert_layout(batch, batch_order == nullptr);
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, l.total, query));
    if (query) return CKEY_OK;
    if (!dbitmap || (variant && !ref)) return CKEY_ERR_INVALID;
    if (batch->n == 0) return CKEY_OK;
    hipStream_t st = as_stream(stream);
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    const KeySrc ix = key_src(index), bt = key_src(batch);
    const uint32_t L = batch->key_bytes, nw = (L + 3) / 4;
    const uint32_t *order = batch_order;
    if (!order) {
        const std::vector<uint8_t> ones(L, 0xFF);
        uint64_t *ck = reinterpret_cast<uint64_t *>(w8 + l.ck);
        uint32_t *rid = reinterpret_cast<uint32_t *>(w8 + l.rid);
        CKEY_TRY(compress_launch(bt, ones.data(), ck, l.words, rid, flags, st));
        CKEY_TRY(radix_sort(ck, batch->n, l.words, l.nbits, rid, batch->n, 8, 0, flags, w8 + l.sortws, st));
        order = rid;
    }
    uint32_t *pos = reinterpret_cast<uint32_t *>(w8 + l.pos);
    uint32_t *acc_d = reinterpret_cast<uint32_t *>(w8 + l.acc_d);
    CKEY_TRY(fill_u32(acc_d, nw, 0, st));
    CKEY_TRY(insert_launch(ix, index_order, bt, order, pos, acc_d, flags, st));
    CKEY_TRY(bitmap_or_finalize(acc_d, dbitmap, L, st));
    if (variant) {
        uint32_t *acc_v = reinterpret_cast<uint32_t *>(w8 + l.acc_v);
        CKEY_TRY(fill_u32(acc_v, nw, 0, st));
        CKEY_TRY(variant_launch(bt, ref, acc_v, flags, st));
        CKEY_TRY(bitmap_or_finalize(acc_v, variant, L, st));
    }
    return CKEY_OK;
}

ckey_status ckey_tree_plan(uint64_t n, float fill, ckey_tree_shape *shape) {
    if (!shape || !(fill > 0.0f && fill <= 1.0f)) return CKEY_ERR_INVALID;
    if (n > CKEY_MAX_ROWS) return CKEY_ERR_UNSUPPORTED;
    const TreePlan t = tree_plan(n, fill);
    memset(shape, 0, sizeof(*shape));
    shape->height = t.height;
    shape->leaf_entries = t.leaf_entries;
    shape->inner_entries = t.inner_entries;
    for (uint32_t l = 0; l < t.height; ++l) {
        shape->level_nodes[l] = t.level_nodes[l];
        shape->level_first[l] = t.level_first[l];
    }
    shape->total_nodes = t.total_nodes;
    return CKEY_OK;
}

ckey_status ckey_bulk_load(const ckey_tree_input *in, uint32_t pk_bits, float fill, void *nodes,
                           uint64_t *deref, void *ws, size_t *ws_bytes, void *stream) {
    if (!in) return CKEY_ERR_INVALID;
    CKEY_TRY(check_keys(&in->keys));
    if (pk_bits < 1 || pk_bits > 32 || !(fill > 0.0f && fill <= 1.0f)) return CKEY_ERR_INVALID;
    const uint32_t L = in->keys.key_bytes;
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, tree_workspace(L), query));
    if (query) return CKEY_OK;
    const uint64_t n = in->keys.n;
    if (n == 0) return CKEY_OK;
    if (!nodes || !in->perm || !in->ckeys || !in->cbitmap || (n > 1 && !in->pair_pos)) return CKEY_ERR_INVALID;
    if (in->variant && !in->ref) return CKEY_ERR_INVALID;
    if (in->words < words_for(popcount_bitmap(in->cbitmap, L))) return CKEY_ERR_INVALID;
    const TreePlan t = tree_plan(n, fill);
    return bulk_load_launch(key_src(&in->keys), in->perm, in->ckeys, in->words, in->cbitmap, in->pair_pos,
                            in->variant, in->ref, pk_bits, t, nodes,
                            reinterpret_cast<unsigned long long *>(deref), ws, as_stream(stream));
}

ckey_status ckey_compress(const ckey_keys *keys, const uint8_t *bitmap, uint64_t *ckeys,
                          uint32_t words, uint32_t *rowids, uint32_t *flags, void *stream) {
    CKEY_TRY(check_keys(keys));
    if (!bitmap) return CKEY_ERR_INVALID;
    if (keys->n > 0 && !ckeys) return CKEY_ERR_INVALID;
    if (words < words_for(popcount_bitmap(bitmap, keys->key_bytes))) return CKEY_ERR_INVALID;
    return compress_launch(key_src(keys), bitmap, ckeys, words, rowids, flags, as_stream(stream));
}

ckey_status ckey_sort(uint64_t *ckeys, uint32_t words, uint32_t nbits, uint32_t *rowids, uint64_t n,
                      const ckey_sort_opts *opts, void *ws, size_t *ws_bytes, void *stream) {
    if (n > CKEY_MAX_ROWS) return CKEY_ERR_UNSUPPORTED;
    if (words == 0 || nbits > 64ull * words) return CKEY_ERR_INVALID;
    CKEY_TRY(check_sort_opts(opts, ws != nullptr));
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, sort_workspace(opts, words, nbits, n), query));
    if (query) return CKEY_OK;
    if (n > 0 && (!ckeys || !rowids)) return CKEY_ERR_INVALID;
    return sort_dispatch(opts, ckeys, words, nbits, rowids, n, opts ? opts->flags : nullptr, ws,
                         as_stream(stream), true);
}

ckey_status ckey_compress_sort(const ckey_keys *keys, const uint8_t *bitmap, uint64_t *ckeys,
                               uint32_t words, uint32_t *rowids, const ckey_sort_opts *opts,
                               void *ws, size_t *ws_bytes, void *stream) {
    CKEY_TRY(check_keys(keys));
    if (!bitmap) return CKEY_ERR_INVALID;
    const uint32_t nbits = popcount_bitmap(bitmap, keys->key_bytes);
    if (words < words_for(nbits)) return CKEY_ERR_INVALID;
    CKEY_TRY(check_sort_opts(opts, ws != nullptr));
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, sort_workspace(opts, words, nbits, keys->n), query));
    if (query) return CKEY_OK;
    if (keys->n > 0 && (!ckeys || !rowids)) return CKEY_ERR_INVALID;
    return compress_sort_dispatch(opts, key_src(keys), bitmap, ckeys, words, nbits, rowids,
                                  opts ? opts->flags : nullptr, ws, as_stream(stream), true);
}

ckey_status ckey_rebuild_index(const ckey_index_desc *idx, uint32_t count,
                               const ckey_sort_opts *opts, void *ws, size_t *ws_bytes,
                               void *stream) {
    if (!ws_bytes) return CKEY_ERR_INVALID;
    if (opts && opts->fused_table)
        return fused_rebuild(idx, count, opts, ws != nullptr, ws, ws_bytes, as_stream(stream));
    RebuildPlan plan;
    CKEY_TRY(plan_rebuild(idx, count, opts, ws != nullptr, plan));
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, plan.total, query));
    if (query) return CKEY_OK;
    return enqueue_rebuild(idx, count, opts, plan, ws, as_stream(stream));
}

struct ckey_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

ckey_status ckey_graph_create(const ckey_index_desc *idx, uint32_t count, const ckey_sort_opts *opts,
                              void *ws, size_t ws_bytes, ckey_graph **out) {
    if (!out || !ws) return CKEY_ERR_INVALID;
    const bool fused = opts && opts->fused_table;
    RebuildPlan plan;
    if (fused) {
        size_t need = 0;
        CKEY_TRY(fused_rebuild(idx, count, opts, true, nullptr, &need, nullptr));
        if (ws_bytes < need) return CKEY_ERR_WORKSPACE;
    } else {
        CKEY_TRY(plan_rebuild(idx, count, opts, true, plan));
        for (uint32_t x = 0; x < count; ++x) {
            const ckey_sort_opts *o = idx[x].opts ? idx[x].opts : opts;
            if (method_of(o) != CKEY_SORT_RADIX) return CKEY_ERR_UNSUPPORTED;
        }
        if (ws_bytes < plan.total) return CKEY_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256) return CKEY_ERR_INVALID;
    hipStream_t cs = nullptr;
    CKEY_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    ckey_status st = CKEY_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return CKEY_ERR_HIP;
    }
    size_t wsb = ws_bytes;
    st = fused ? fused_rebuild(idx, count, opts, true, ws, &wsb, cs) : enqueue_rebuild(idx, count, opts, plan, ws, cs);
    const hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st != CKEY_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != CKEY_OK ? st : CKEY_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return CKEY_ERR_HIP;
    }
    *out = new ckey_graph{g, ex};
    return CKEY_OK;
}

ckey_status ckey_graph_launch(ckey_graph *g, void *stream) {
    if (!g) return CKEY_ERR_INVALID;
    CKEY_HIP_TRY(hipGraphLaunch(g->exec, as_stream(stream)));
    return CKEY_OK;
}

ckey_status ckey_graph_destroy(ckey_graph *g) {
    if (!g) return CKEY_OK;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return CKEY_OK;
}

ckey_status ckey_tune_index(const ckey_index_desc *idx, const ckey_sort_opts *cand, uint32_t ncand,
                            void *ws, size_t ws_bytes, void *stream, uint32_t *best,
                            float *times_ms) {
    if (!idx || !cand || ncand == 0 || !best || !ws) return CKEY_ERR_INVALID;
    hipStream_t st = as_stream(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CKEY_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CKEY_ERR_HIP;
    }
    ckey_status status = CKEY_OK;
    float best_ms = 0;
    for (uint32_t c = 0; c < ncand && status == CKEY_OK; ++c) {
        ckey_index_desc d = *idx;
        d.opts = &cand[c];
        const ckey_sort_opts *call = cand[c].fused_table ? &cand[c] : nullptr;  // one-launch form
        size_t need = ws_bytes;
        status = ckey_rebuild_index(&d, 1, call, ws, &need, stream);  // warm-up
        if (status != CKEY_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { status = CKEY_ERR_HIP; break; }
        status = ckey_rebuild_index(&d, 1, call, ws, &need, stream);
        if (status != CKEY_OK) break;
        float ms = 0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            status = CKEY_ERR_HIP;
            break;
        }
        if (times_ms) times_ms[c] = ms;
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            *best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

size_t ckey_cdf_model_bytes(uint32_t b_log2) { return learned_b_ok(b_log2) ? model_bytes(b_log2) : 0; }

ckey_status ckey_cdf_model_init(void *model, uint32_t b_log2, uint64_t seed, void *stream) {
    if (!model || reinterpret_cast<uintptr_t>(model) % 256) return CKEY_ERR_INVALID;
    if (!learned_b_ok(b_log2)) return CKEY_ERR_INVALID;
    return model_init(model, seed, as_stream(stream));
}

ckey_status ckey_cdf_fit(void *model, uint32_t b_log2, const uint64_t *sorted_prefix, uint64_t m,
                         const ckey_cdf_train_opts *o, float *loss_trace, void *ws,
                         size_t *ws_bytes, void *stream) {
    if (!o || !learned_b_ok(b_log2)) return CKEY_ERR_INVALID;
    if (o->batch == 0 || o->batch > (1u << 20)) return CKEY_ERR_INVALID;
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, grad_workspace(o->batch), query));
    if (query) return CKEY_OK;
    if (!model || !sorted_prefix || m == 0) return CKEY_ERR_INVALID;
    hipStream_t st = as_stream(stream);
    CKEY_TRY(model_thresholds(model, b_log2, sorted_prefix, m, st));
    return model_train(model, sorted_prefix, m, o->steps, o->batch, o->lr, o->beta1, o->beta2,
                       o->eps, o->seed, loss_trace, ws, st);
}

ckey_status ckey_cdf_grad(const void *model, const uint64_t *prefix, const float *target,
                          uint64_t m, float *grad, float *loss, void *ws, size_t *ws_bytes,
                          void *stream) {
    if (m == 0 || m > (1u << 20)) return CKEY_ERR_INVALID;
    bool query;
    CKEY_TRY(ws_check(ws, ws_bytes, grad_workspace(uint32_t(m)), query));
    if (query) return CKEY_OK;
    if (!model || !prefix || !target || (!grad && !loss)) return CKEY_ERR_INVALID;
    return model_grad(model, prefix, target, m, uint32_t(m), 0, 0, grad, loss, ws, as_stream(stream));
}

ckey_status ckey_cdf_bucket(const void *model, uint32_t b_log2, uint32_t method,
                            const uint64_t *prefix, uint64_t n, uint32_t *bucket,
                            uint32_t *predicted, uint64_t *stats, void *stream) {
    if (!learned_b_ok(b_log2)) return CKEY_ERR_INVALID;
    if (method != CKEY_SORT_LEARNED && method != CKEY_SORT_SPLITTER) return CKEY_ERR_INVALID;
    if (n > 0 && (!model || !prefix || !bucket)) return CKEY_ERR_INVALID;
    if (n > CKEY_MAX_ROWS) return CKEY_ERR_UNSUPPORTED;
    return model_bucket(model, b_log2, method == CKEY_SORT_LEARNED ? 1 : 0, prefix, n, bucket,
                        method == CKEY_SORT_LEARNED ? predicted : nullptr,
                        reinterpret_cast<unsigned long long *>(stats), as_stream(stream));
}

}  // extern "C"
