// Index tree bulk load (Sec. 5.3, index construction) from a rebuild's sorted
// output: leaves and inner levels of 256-byte nodes, built level by level,
// one thread per entry.
//
// Node layout (little-endian; unused bytes are zero):
//   header (24 B): record ID of the node's highest key u64, entry count u16,
//                  level u16 (0 = leaf), zero u32, sorted position of the
//                  node's first key u64
//   leaf:  next leaf's node index u64 (all ones for the last leaf), then up to
//          14 entries of 16 B: partial key u32, D position u16, key length u16,
//          record ID u64
//   inner: up to 9 entries of 24 B: partial key u32, D position u16, key
//          length u16, child node index u64, record ID of the child's highest
//          key u64
// Levels are stored leaves first, each level's nodes in key order.  A full
// node holds floor(fanout * fill) entries; the last node of a level the rest.
//
// An entry's D position is that of its key against the previous entry's key
// of the same level: for leaves the rebuild's per-pair positions (Sec. 5.3,
// D-offset of the compressed keys' D-bit); for an inner entry, by Lemma 1, the
// minimum over the entries of its child node (the child's first entry is
// taken against the previous child's last key).  0xFFFF marks the first entry
// of a level, 0xFFFE a key equal to the previous one.
//
// Partial key (Sec. 4.2): the pk bits after the D position, MSB-first and
// left-aligned in 32 bits (the first entry: the key's first pk bits; an equal
// key: zero).  Each bit comes, as Sec. 5.3 lists: A. from the compressed key
// if its position is in the compression bitmap; B. from the reference key if
// the variant bitmap has 0 there; C. otherwise from the key itself, read by
// record ID (option b), counted in `deref`.  Without a variant bitmap every
// position outside the compression bitmap is read from the key.
#include "internal.h"

namespace ckey {

namespace {

constexpr uint16_t kFirst = 0xFFFF, kEqual = 0xFFFE;
constexpr uint32_t kNode = CKEY_TREE_NODE_BYTES;

struct BitmapArg {
    uint8_t b[CKEY_MAX_KEY_BYTES];
};

// Workspace tables: compression bitmap, variant bitmap (all ones when none
// was given), rank of each byte's first position in the compression bitmap.
struct TreeTables {
    uint8_t *cb;
    uint8_t *var;
    uint16_t *rank;
};

__global__ void k_tree_table(BitmapArg bm, uint32_t L, uint8_t *__restrict__ dst, uint16_t *__restrict__ rank) {
    // one workgroup: copy the bitmap; with rank != null also its byte ranks (serial scan)
    for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) dst[j] = bm.b[j];
    if (rank && threadIdx.x == 0) {
        uint32_t c = 0;
        for (uint32_t j = 0; j < L; ++j) {
            rank[j] = uint16_t(c);
            c += __popc(uint32_t(bm.b[j]));
        }
    }
}

struct PkArgs {
    KeySrc keys;
    const uint32_t *perm;
    const uint64_t *ck;     // sorted compressed keys, word-major
    uint64_t n;
    uint32_t words;
    const uint8_t *ref;     // device reference key (null: no variant bitmap)
    uint32_t pk;
};

// Per-workgroup copies of the tables, indexed by key byte.
struct LdsTables {
    uint8_t cb[CKEY_MAX_KEY_BYTES];    // compression bitmap
    uint8_t var[CKEY_MAX_KEY_BYTES];   // variant bitmap (all ones: none given)
    uint8_t ref[CKEY_MAX_KEY_BYTES];   // reference key
    uint16_t rank[CKEY_MAX_KEY_BYTES]; // compressed index of each byte's first position
};

__device__ __forceinline__ uint16_t key_len_of(const KeySrc &k, uint64_t row) {
    if (!k.offsets) return uint16_t(k.L);
    const uint64_t len = k.offsets[row + 1] - k.offsets[row];
    return uint16_t(len < k.L ? len : k.L);
}

// The 32 bits at positions [start, start+32) of the key at sorted position pos
// (row `row`), assembled byte by byte over the (at most five) key bytes the
// window touches: class-A bits deposited from the compressed key's run of
// bits, class-B bits from the reference key, class-C bits from the key.
__device__ uint32_t partial_key(const PkArgs &a, const LdsTables &t, uint64_t pos, uint64_t row,
                                uint16_t dpos, bool &deref) {
    if (dpos == kEqual) return 0u;
    const uint32_t start = dpos == kFirst ? 0u : uint32_t(dpos) + 1u;
    const uint32_t L = a.keys.L;
    if (start >= 8 * L) return 0u;
    const uint32_t b0 = start >> 3, sh = start & 7u;
    uint32_t cbq[5], varq[5], wm[5];
    uint32_t c_any = 0, a_any = 0;
    const uint32_t end = min(start + a.pk, 8 * L);  // window [start, end)
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const uint32_t j = b0 + q;
        const uint32_t lo = max(start, 8 * j), hi = min(end, 8 * j + 8);  // window bits of byte j
        wm[q] = lo < hi ? (0xFFu >> (lo - 8 * j)) & ~(0xFFu >> (hi - 8 * j)) & 0xFFu : 0u;
        cbq[q] = j < L ? uint32_t(t.cb[j]) : 0u;
        varq[q] = j < L ? uint32_t(t.var[j]) : 0u;
        c_any |= varq[q] & ~cbq[q] & wm[q];
        a_any |= cbq[q] & wm[q];
    }
    uint32_t keyq[5] = {0, 0, 0, 0, 0};
    if (c_any) {  // option C (b): read the key by record ID
        deref = true;
        // The window's five bytes are loaded together, each at an index
        // clamped into the key (a byte past the key reads its last byte and
        // is replaced by zero, as are bytes outside the window by the masks).
        const uint8_t *kp;
        uint32_t klen;
        if (a.keys.offsets) {
            const uint64_t o0 = a.keys.offsets[row], o1 = a.keys.offsets[row + 1];
            kp = a.keys.bytes + o0;
            klen = uint32_t(min<uint64_t>(o1 - o0, L));
        } else {
            kp = a.keys.bytes + row * a.keys.stride;
            klen = L;
        }
        if (klen > 0) {
            uint32_t kb[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) kb[q] = kp[min(b0 + uint32_t(q), klen - 1)];
#pragma unroll
            for (int q = 0; q < 5; ++q) keyq[q] = b0 + uint32_t(q) < klen ? kb[q] : 0u;
        }
    }
    uint32_t F = 0;  // the compressed key's bits from the window's first class-A position on
    if (a_any) {
        const uint32_t c0 = uint32_t(t.rank[b0]) + __popc(cbq[0] & ~(0xFFu >> sh) & 0xFFu);
        const uint32_t k0 = c0 >> 6, o = c0 & 63u;
        const uint64_t w0 = a.ck[uint64_t(k0) * a.n + pos];
        const uint64_t w1 = (o && k0 + 1 < a.words) ? a.ck[uint64_t(k0 + 1) * a.n + pos] : 0ull;
        const uint64_t x = o ? (w0 << o) | (w1 >> (64 - o)) : w0;
        F = uint32_t(x >> 32);
    }
    uint64_t v40 = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        uint32_t byte = (uint32_t(t.ref[b0 + q < L ? b0 + q : 0]) & ~varq[q]) | (keyq[q] & varq[q] & ~cbq[q]);
        uint32_t m = cbq[q] & wm[q];
        while (m) {  // deposit the next compressed bits into this byte's class-A positions
            const uint32_t hb = 31u - __clz(m);
            byte |= (F >> 31) << hb;
            F <<= 1;
            m &= ~(1u << hb);
        }
        v40 = (v40 << 8) | (byte & wm[q]);
    }
    return uint32_t(v40 >> (8 - sh));  // bits past the window are zero
}

__device__ __forceinline__ void load_tables(const TreeTables &tt, const uint8_t *ref, uint32_t L,
                                            LdsTables &t) {
    for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
        t.cb[j] = tt.cb[j];
        t.var[j] = tt.var[j];
        t.ref[j] = ref ? ref[j] : uint8_t(0);
        t.rank[j] = tt.rank[j];
    }
}

// One global atomic per workgroup (a single counter shared by the whole grid).
__device__ __forceinline__ void count_deref(uint32_t mine, uint32_t *s_cnt, unsigned long long *cnt) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && cnt && *s_cnt) atomicAdd(cnt, (unsigned long long)*s_cnt);
}

constexpr uint32_t kTreeBlocks = 4096;  // grid-stride launches

inline uint32_t grid_blocks(uint64_t items) {
    const uint64_t b = (items + kWG - 1) / kWG;
    return uint32_t(b < kTreeBlocks ? b : kTreeBlocks);
}

__global__ __launch_bounds__(kWG) void k_leaf_level(PkArgs a, TreeTables tt,
                                                    const uint32_t *__restrict__ pair_pos,
                                                    uint32_t lp, uint64_t nleaves,
                                                    uint8_t *__restrict__ nodes,
                                                    unsigned long long *__restrict__ deref_cnt) {
    __shared__ LdsTables s_t;
    __shared__ uint32_t s_cnt;
    load_tables(tt, a.ref, a.keys.L, s_t);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    uint32_t nderef = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * kWG + threadIdx.x; i < a.n; i += uint64_t(gridDim.x) * kWG) {
        bool deref = false;
        const uint64_t j = i / lp, slot = i % lp;
        const uint64_t row = a.perm[i];
        uint16_t dpos = kFirst;
        if (i > 0) {
            const uint32_t pp = pair_pos[i - 1];
            dpos = pp == 0xFFFFFFFFu ? kEqual : uint16_t(pp);
        }
        const uint32_t pkv = partial_key(a, s_t, i, row, dpos, deref);
        nderef += deref ? 1u : 0u;
        uint64_t *nd = reinterpret_cast<uint64_t *>(nodes + j * kNode);
        nd[4 + 2 * slot] = uint64_t(pkv) | (uint64_t(dpos) << 32) | (uint64_t(key_len_of(a.keys, row)) << 48);
        nd[5 + 2 * slot] = row;
        if (slot == 0) {
            const uint64_t cnt = min<uint64_t>(lp, a.n - j * lp);
            nd[0] = a.perm[j * lp + cnt - 1];
            nd[1] = cnt;  // level 0
            nd[2] = j * lp;
            nd[3] = j + 1 < nleaves ? j + 1 : ~0ull;
            for (uint64_t q = 4 + 2 * cnt; q < kNode / 8; ++q) nd[q] = 0;  // unused entries
        }
    }
    count_deref(nderef, &s_cnt, deref_cnt);
}

// Level l >= 1: one thread per child node e of level l-1.
__global__ __launch_bounds__(kWG) void k_inner_level(PkArgs a, TreeTables tt, uint32_t level,
                                                     uint32_t ip, uint64_t nchildren,
                                                     uint64_t child_first, uint64_t child_span,
                                                     uint64_t span, uint64_t first,
                                                     uint8_t *__restrict__ nodes,
                                                     unsigned long long *__restrict__ deref_cnt) {
    __shared__ LdsTables s_t;
    __shared__ uint32_t s_cnt;
    load_tables(tt, a.ref, a.keys.L, s_t);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    uint32_t nderef = 0;
    for (uint64_t e = uint64_t(blockIdx.x) * kWG + threadIdx.x; e < nchildren; e += uint64_t(gridDim.x) * kWG) {
        bool deref = false;
        const uint64_t j = e / ip, slot = e % ip;
        const uint64_t pos = min<uint64_t>(a.n, (e + 1) * child_span) - 1;  // child's highest key
        const uint64_t row = a.perm[pos];
        const uint8_t *child = nodes + (child_first + e) * kNode;
        uint16_t dpos = kFirst;
        if (e > 0) {  // Lemma 1: the minimum over the child's entries
            const uint32_t cnt = *reinterpret_cast<const uint16_t *>(child + 8);
            const uint32_t base = level == 1 ? 32u : 24u, esz = level == 1 ? 16u : 24u;
            dpos = kEqual;
            for (uint32_t q = 0; q < cnt; ++q) {
                const uint16_t d = *reinterpret_cast<const uint16_t *>(child + base + esz * q + 4);
                dpos = d < dpos ? d : dpos;
            }
        }
        const uint32_t pkv = partial_key(a, s_t, pos, row, dpos, deref);
        nderef += deref ? 1u : 0u;
        uint64_t *nd = reinterpret_cast<uint64_t *>(nodes + (first + j) * kNode);
        nd[3 + 3 * slot] = uint64_t(pkv) | (uint64_t(dpos) << 32) | (uint64_t(key_len_of(a.keys, row)) << 48);
        nd[4 + 3 * slot] = child_first + e;
        nd[5 + 3 * slot] = row;
        if (slot == 0) {
            const uint64_t cnt = min<uint64_t>(ip, nchildren - j * ip);
            nd[0] = a.perm[min<uint64_t>(a.n, (j + 1) * span) - 1];
            nd[1] = cnt | (uint64_t(level) << 16);
            nd[2] = j * span;
            for (uint64_t q = 3 + 3 * cnt; q < kNode / 8; ++q) nd[q] = 0;  // unused entries, pad
        }
    }
    count_deref(nderef, &s_cnt, deref_cnt);
}

}  // namespace

TreePlan tree_plan(uint64_t n, float fill) {
    TreePlan t{};
    const double f = double(fill);
    const uint32_t a = uint32_t(floor(double(CKEY_TREE_LEAF_FANOUT) * f));
    const uint32_t b = uint32_t(floor(double(CKEY_TREE_INNER_FANOUT) * f));
    t.leaf_entries = a < 1 ? 1 : a;
    t.inner_entries = b < 2 ? 2 : b;
    if (n == 0) return t;
    uint64_t nodes = (n + t.leaf_entries - 1) / t.leaf_entries;
    uint64_t span = t.leaf_entries;
    for (;;) {
        t.level_first[t.height] = t.total_nodes;
        t.level_nodes[t.height] = nodes;
        t.span[t.height] = span;
        t.total_nodes += nodes;
        ++t.height;
        if (nodes <= 1) break;
        nodes = (nodes + t.inner_entries - 1) / t.inner_entries;
        span = span > n ? span : span * t.inner_entries;  // saturates once past n
    }
    return t;
}

size_t tree_workspace(uint32_t L) { return align256(size_t(L) * 4); }

ckey_status bulk_load_launch(const KeySrc &k, const uint32_t *perm, const uint64_t *ck,
                             uint32_t words, const uint8_t *cbitmap_host, const uint32_t *pair_pos,
                             const uint8_t *variant_host, const uint8_t *ref, uint32_t pk,
                             const TreePlan &t, void *nodes, unsigned long long *deref, void *ws,
                             hipStream_t st) {
    if (k.n == 0) return CKEY_OK;
    const uint32_t L = k.L;
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    TreeTables tt{w8, w8 + L, reinterpret_cast<uint16_t *>(w8 + 2 * L)};
    BitmapArg bm;
    for (uint32_t j = 0; j < CKEY_MAX_KEY_BYTES; ++j) bm.b[j] = j < L ? cbitmap_host[j] : 0;
    hipLaunchKernelGGL(k_tree_table, dim3(1), dim3(kWG), 0, st, bm, L, tt.cb, tt.rank);
    for (uint32_t j = 0; j < CKEY_MAX_KEY_BYTES; ++j) bm.b[j] = j < L ? (variant_host ? variant_host[j] : 0xFF) : 0;
    hipLaunchKernelGGL(k_tree_table, dim3(1), dim3(kWG), 0, st, bm, L, tt.var, nullptr);
    CKEY_TRY(launch_status());
    PkArgs a{k, perm, ck, k.n, words, ref, pk};
    uint8_t *nd = static_cast<uint8_t *>(nodes);
    const int pr = prof_begin(st, "tree_leaves");
    hipLaunchKernelGGL(k_leaf_level, dim3(grid_blocks(k.n)), dim3(kWG), 0, st, a, tt,
                       pair_pos, t.leaf_entries, t.level_nodes[0], nd, deref);
    prof_end(st, pr);
    CKEY_TRY(launch_status());
    for (uint32_t l = 1; l < t.height; ++l) {
        const uint64_t nch = t.level_nodes[l - 1];
        const int pr2 = prof_begin(st, "tree_inner");
        hipLaunchKernelGGL(k_inner_level, dim3(grid_blocks(nch)), dim3(kWG), 0, st, a, tt, l,
                           t.inner_entries, nch, t.level_first[l - 1], t.span[l - 1], t.span[l],
                           t.level_first[l], nd, deref);
        prof_end(st, pr2);
        CKEY_TRY(launch_status());
    }
    return CKEY_OK;
}

}  // namespace ckey
