// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <utility>

#include "../../include/ckey.h"

namespace ckey {

constexpr int kWG = 256;  // threads per workgroup (4 wave64s)

#define CKEY_TRY(expr)                      \
    do {                                    \
        ckey_status s_ = (expr);            \
        if (s_ != CKEY_OK) return s_;       \
    } while (0)

#define CKEY_HIP_TRY(expr)                  \
    do {                                    \
        hipError_t e_ = (expr);             \
        if (e_ != hipSuccess) return CKEY_ERR_HIP; \
    } while (0)

inline ckey_status launch_status() {
    return hipGetLastError() == hipSuccess ? CKEY_OK : CKEY_ERR_HIP;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Key source as the kernels see it.
struct KeySrc {
    const uint8_t *bytes;
    const uint64_t *offsets;  // nullptr: fixed width
    uint64_t n;
    uint32_t L;
    uint32_t stride;
};

// How a kernel may read key words.
enum LoadMode : int {
    kLoad16 = 0,  // fixed width, 16-byte aligned rows: 128-bit loads
    kLoad4 = 1,   // fixed width, 4-byte aligned rows: 32-bit loads
    kLoadBytes = 2  // anything else (variable length, odd strides): byte loads
};

inline int load_mode(const KeySrc &k) {
    if (k.offsets) return kLoadBytes;
    uintptr_t b = reinterpret_cast<uintptr_t>(k.bytes);
    if (k.stride % 16 == 0 && b % 16 == 0) return kLoad16;
    if (k.stride % 4 == 0 && b % 4 == 0) return kLoad4;
    return kLoadBytes;
}

// Big-endian 32-bit word j (bytes 4j..4j+3) of a key, bytes at or past `len`
// read as zero.  `p` points at the key's first byte.
__device__ __forceinline__ uint32_t key_word_bytes(const uint8_t *p, uint32_t j, uint32_t len) {
    uint32_t v = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t q = 4 * j + t;
        v = (v << 8) | (q < len ? uint32_t(p[q]) : 0u);
    }
    return v;
}

// Same for a 4-byte aligned fixed-width key of length len (len <= stride).
__device__ __forceinline__ uint32_t key_word_aligned(const uint8_t *p, uint32_t j, uint32_t len) {
    uint32_t v = __builtin_bswap32(*reinterpret_cast<const uint32_t *>(p + 4 * j));
    uint32_t have = len - 4 * j;  // bytes of this word inside the key (>= 1)
    if (have < 4) v &= ~(0xFFFFFFFFu >> (8 * have));
    return v;
}

// Bit for position p inside the little-endian u32 view of a bitmap
// (bitmap byte p/8 is byte (p/8)%4 of word p/32; the position is bit 7-p%8 of that byte).
__device__ __forceinline__ uint32_t bitmap_word_bit(uint32_t p) {
    return 1u << (8 * ((p >> 3) & 3) + (7 - (p & 7)));
}

// Dynamic LDS above 64 KB needs the kernel attribute raised, to the 160 KB
// of a CU less the kernel's static LDS: once per (device, kernel), remembered
// so that later calls pay nothing.
inline void raise_lds_limit(const void *fn) {
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    if (done.insert({dev, fn}).second) {
        hipFuncAttributes at{};
        const size_t stat = hipFuncGetAttributes(&at, fn) == hipSuccess ? at.sharedSizeBytes : 0;
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(160 * 1024 - stat));
    }
}

// Workgroups of `fn` that are resident on the current device at once: CUs x
// workgroups per CU at `threads` threads and `lds` bytes of dynamic LDS (at
// least 1).  Remembered per (device, kernel, threads, lds).
inline uint32_t resident_grid(const void *fn, int threads, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int, size_t>, uint32_t> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    const auto key = std::make_tuple(dev, fn, threads, lds);
    const auto it = done.find(key);
    if (it != done.end()) return it->second;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) per_cu = 1;
    const uint32_t grid = uint32_t(cus > 0 ? cus : 1) * uint32_t(per_cu > 0 ? per_cu : 1);
    done.emplace(key, grid);
    return grid;
}

// Event timing around a launch when profiling is enabled (profiler.hip).
int prof_begin(hipStream_t st, const char *name);
void prof_end(hipStream_t st, int idx);

// ----------------------------------------------------------------- launchers --
// Distinction bits (k_dbits.hip).
ckey_status dbits_launch(const KeySrc &k, const uint32_t *order, uint32_t *acc_words,
                         uint32_t *flags, hipStream_t st);
// Clear n u32 words (a fill kernel, safe inside graph capture).  gate: a
// device word read by the kernel, which writes nothing while it is 0.
ckey_status fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st, const uint32_t *gate = nullptr);
// Copy a little-endian u32 bitmap accumulator into a byte bitmap of L bytes.
ckey_status bitmap_finalize(const uint32_t *acc_words, uint8_t *bitmap, uint32_t L, hipStream_t st);

// Compression plan (host side, k_compress.hip).
struct HostPlan;
ckey_status compress_launch(const KeySrc &k, const uint8_t *bitmap_host, uint64_t *ckeys,
                            uint32_t words, uint32_t *rowids, uint32_t *flags, hipStream_t st);

// DS-metadata maintenance (k_maintain.hip).  acc_words: u32 view of a bitmap
// (zeroed by the caller), OR-ed into.
// Variant bitmap of k against ref (device, L bytes; nullptr: key 0 of k).
ckey_status variant_launch(const KeySrc &k, const uint8_t *ref, uint32_t *acc_words,
                           uint32_t *flags, hipStream_t st);
// Key 0 of k, zero-padded to L bytes (all zero when k is empty).
ckey_status ref_copy_launch(const KeySrc &k, uint8_t *out, hipStream_t st);
// OR a little-endian u32 bitmap accumulator into a byte bitmap of L bytes.
ckey_status bitmap_or_finalize(const uint32_t *acc_words, uint8_t *bitmap, uint32_t L, hipStream_t st);
// Batched insert of bt (in key order bt_order, or as stored) into the index ix
// (key order ix_order, or as stored): pos[j] receives the place of batch key j,
// acc_words the D-bits of the new adjacent pairs.
ckey_status insert_launch(const KeySrc &ix, const uint32_t *ix_order, const KeySrc &bt,
                          const uint32_t *bt_order, uint32_t *pos, uint32_t *acc_words,
                          uint32_t *flags, hipStream_t st);

// Index tree bulk load (k_tree.hip).
struct TreePlan {
    uint32_t height, leaf_entries, inner_entries;
    uint64_t level_nodes[CKEY_TREE_MAX_LEVELS];
    uint64_t level_first[CKEY_TREE_MAX_LEVELS];
    uint64_t span[CKEY_TREE_MAX_LEVELS];  // keys under a full node of each level (saturating past n)
    uint64_t total_nodes;
};
TreePlan tree_plan(uint64_t n, float fill);
size_t tree_workspace(uint32_t L);
ckey_status bulk_load_launch(const KeySrc &k, const uint32_t *perm, const uint64_t *ckeys,
                             uint32_t words, const uint8_t *cbitmap_host, const uint32_t *pair_pos,
                             const uint8_t *variant_host, const uint8_t *ref, uint32_t pk,
                             const TreePlan &t, void *nodes, unsigned long long *deref, void *ws,
                             hipStream_t st);

// Refresh of the D-bitmap from sorted compressed keys (k_refine.hip).
ckey_status refine_launch(const uint64_t *ckeys, uint32_t words, uint64_t n,
                          const uint8_t *bitmap_in_host, uint32_t L, uint32_t *acc_words,
                          uint32_t *pair_pos, uint32_t *flags, hipStream_t st);

// Radix sort (k_radix.hip): stable LSD sort of rows [0, n) of word-major keys
// (word k of row i at ckeys[k*ld + i]) by their top nbits, moving rowids
// along.  rid_bits > 0 first sorts by the low rid_bits bits of the row ids,
// so that ties end up in row-id order whatever the input order.
// half_tile: passes over 1..8 words take half the rows per workgroup (512
// threads); an option the autotuner may choose.
size_t radix_workspace(uint32_t words, uint32_t nbits, uint64_t n, uint32_t digit_bits,
                       uint32_t rid_bits = 0, bool half_tile = false);
// Passes of a sort of the top nbits of `words` words with digit_bits-bit
// digits.  A sort of at most kRadixInlinePasses passes (no skip_trivial)
// makes no heap allocation on the host.
constexpr uint32_t kRadixInlinePasses = 512;
uint32_t radix_pass_count(uint32_t words, uint32_t nbits, uint32_t digit_bits);
// skip_trivial: read the pass histograms back (one stream synchronization)
// and skip every pass whose digit is the same for all n rows.
// gate (device word, or nullptr): every kernel of the sort returns at once
// while it is 0 -- a sort enqueued whether or not it turns out to be needed
// (a captured graph cannot ask the host).
ckey_status radix_sort(uint64_t *ckeys, uint64_t ld, uint32_t words, uint32_t nbits,
                       uint32_t *rowids, uint64_t n, uint32_t digit_bits, uint32_t rid_bits,
                       uint32_t *flags, void *ws, hipStream_t st, bool skip_trivial = false,
                       const uint32_t *gate = nullptr, bool half_tile = false);

// Stable sort of rows [0, n) by a 16-bit aux key of aux_bits bits (two
// one-sweep passes; the aux array is read, not reordered), moving the words
// and row ids; the result is back in ck/rid.  rid_identity: the row ids are
// 0..n-1 in order and are generated by the first pass instead of read (rid
// is then only written).
size_t aux_sort_workspace(uint32_t words, uint64_t n);
// aux_full_hist (optional): histogram over all 2^aux_bits values, from which
// the passes' histograms are derived instead of re-reading aux.
ckey_status aux_sort(uint64_t *ck, uint32_t *rid, bool rid_identity, const uint16_t *aux, uint64_t n,
                     uint32_t words, uint32_t aux_bits, const uint32_t *aux_full_hist, uint32_t *flags,
                     void *ws, hipStream_t st);

// OR a value into a device flags word (a kernel, so it is stream-ordered).
ckey_status fill_flag_or(uint32_t *flags, uint32_t v, hipStream_t st);

// One index of a table rebuilt by the persistent launch (k_table.hip).
struct TableIndex {
    KeySrc keys;
    const uint8_t *bitmap;  // host, keys.L bytes: the bitmap to compress with
    uint32_t digit_bits;
    uint32_t *perm;         // device [n] out
    uint64_t *ckeys_out;    // device [words*n] out or nullptr
    uint32_t *pair_pos;     // device [n-1] out or nullptr
    uint8_t *bitmap_out;    // device [L] out or nullptr
    uint32_t *flags;        // device or nullptr
};
// ws == nullptr: *need = workspace bytes (host only).  Else enqueue one fill
// kernel and the persistent launch on st.
ckey_status table_fused_plan(const TableIndex *ti, uint32_t count, void *ws, size_t *need,
                             hipStream_t st);

// Learned bucketing (k_learned.hip).  mode 1 = learned (MLP + correction),
// mode 0 = splitter search.
bool learned_b_ok(uint32_t b_log2);
size_t learned_workspace(uint32_t words, uint32_t nbits, uint64_t n, uint32_t b_log2);
// cap: the in-LDS capacity of a bucket, 1 = 2560 rows, 2 = 5120, 3 = 10240,
// 0 = chosen from the mean bucket size.
ckey_status learned_sort(uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid, uint64_t n,
                         int mode, const void *model, uint32_t b_log2, uint32_t *flags, void *ws,
                         hipStream_t st, uint32_t cap = 0);
// Compression and bucketing sort with the record IDs generated by the first
// grouping pass.  Learned (mode 1): the bucket of each key is found while it
// is compressed; CKEY_ERR_UNSUPPORTED when the keys do not allow that fused
// kernel (then compress and sort separately).  Splitter (mode 0): a plain
// compression, then the assignment over the first words.
ckey_status compress_learned_sort(const KeySrc &k, const uint8_t *bitmap_host, uint64_t *ck,
                                  uint32_t words, uint32_t nbits, uint32_t *rid, int mode,
                                  const void *model, uint32_t b_log2, uint32_t *flags, void *ws,
                                  hipStream_t st, uint32_t cap = 0);
size_t model_bytes(uint32_t b_log2);
ckey_status model_init(void *model, uint64_t seed, hipStream_t st);
ckey_status model_thresholds(void *model, uint32_t b_log2, const uint64_t *sorted, uint64_t m,
                             hipStream_t st);
size_t grad_workspace(uint32_t M);
ckey_status model_grad(const void *model, const uint64_t *prefix, const float *target, uint64_t m,
                       uint32_t M, uint64_t seed, uint32_t step, float *grad, float *loss, void *ws,
                       hipStream_t st);
ckey_status model_train(void *model, const uint64_t *prefix, uint64_t m, uint32_t steps, uint32_t M,
                        float lr, float b1, float b2, float eps, uint64_t seed, float *loss_trace,
                        void *ws, hipStream_t st);
ckey_status model_bucket(const void *model, uint32_t b_log2, int mode, const uint64_t *prefix,
                         uint64_t n, uint32_t *bucket, uint32_t *pred, unsigned long long *stats,
                         hipStream_t st);

}  // namespace ckey

#include "scan.h"
