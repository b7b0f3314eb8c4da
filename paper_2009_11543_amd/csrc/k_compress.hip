// Key compression (Sec. 3.2; extraction procedure of Sec. 5.1).
//
// The paper cuts the D-bitmap into 8-byte masks and applies x86 PEXT to each
// 8-byte slice of the key, joining the pieces with shift and OR.  gfx950 has
// no PEXT.  The masks are the same for every key, so the host prepares, for
// each 32-bit big-endian source word that holds D bits, its mask m, the five
// "move" masks of the log-step compress of Hacker's Delight (Warren, 2nd ed.,
// Sec. 7-4: after x &= m, step i moves the selected bits right by 2^i), the
// number of selected bits and their offset in the compressed string.  Each key
// then costs, per such word, one AND plus five (AND, XOR, shift-OR) steps and
// a 64-bit shift-OR into the output word -- a fixed cost, independent of how
// fragmented the mask is, with all per-word constants in scalar registers.
// Source words are fetched with 128-bit loads, four 16-byte chunks at a time.
#include <algorithm>
#include <vector>

#include "bucket.h"
#include "internal.h"

namespace ckey {

namespace {

constexpr int kMaxChunks = 24;  // 16-byte chunks per launch (longer keys take several launches)

// One 32-bit source word (slot q of chunk c).  m == 0: the word holds no D bit.
struct WordOp {
    uint32_t m;       // D bits of the word (big-endian word of the bitmap)
    uint32_t mv[5];   // bits moved right by 1, 2, 4, 8, 16
    uint32_t pc;      // popcount(m)
    uint32_t off;     // offset of the word's first selected bit in the compressed string
};

struct CompressPlan {
    uint32_t n_chunks;
    uint32_t word_begin;     // this launch writes output words [word_begin, word_end)
    uint32_t word_end;
    uint32_t zero_end;       // and zero-fills [word_end, zero_end)
    uint32_t kw_init;        // output word of the first source word's first bit
    uint32_t write_rowids;
    uint32_t chunk[kMaxChunks];    // 16-byte chunk index in the key
    WordOp op[kMaxChunks * 4];
};

// Move masks of the log-step compress for mask m (Hacker's Delight Sec. 7-4).
void compress_masks(uint32_t m, uint32_t mv[5]) {
    uint32_t mk = ~m << 1;  // counts the zeros to the right of each bit
    for (int i = 0; i < 5; ++i) {
        uint32_t mp = mk ^ (mk << 1);  // parallel suffix (prefix XOR from the right)
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        const uint32_t v = mp & m;     // bits to move in this step
        mv[i] = v;
        m = (m ^ v) | (v >> (1u << i));
        mk &= ~mp;
    }
}

struct SrcWord {
    uint32_t j, m, off;
};

// Gather of one key's D bits into its output words, for a loader that
// fills the four words of a 16-byte chunk: big-endian, or as loaded from
// memory (little-endian, Loader::kRaw) so that no load's value is needed
// before the group's other loads are issued.
// Returns output word 0 when this launch writes it (else 0).
template <typename Loader>
__device__ __forceinline__ uint64_t compress_key(const CompressPlan &plan, const Loader &ld,
                                                 uint64_t *__restrict__ ck, uint64_t n, uint64_t i) {
    uint64_t acc = 0, w0 = 0;
    uint32_t kw = plan.kw_init;
    // Stores outside [word_begin, word_end) belong to a neighbouring launch.
    auto store = [&](uint32_t kk, uint64_t val) {
        if (kk >= plan.word_begin && kk < plan.word_end) ck[uint64_t(kk) * n + i] = val;
        if (kk == 0) w0 = val;
    };
    // Chunks are taken four at a time: all loads of a group are issued before
    // any of its output stores, so they overlap.
    for (uint32_t c0 = 0; c0 < plan.n_chunks; c0 += 4) {
        uint32_t x[4][4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t c = c0 + g;
            if constexpr (Loader::kRaw) {
                // Memory loads are issued unconditionally (a chunk past the
                // last one reloads the last; its words are not used), so that
                // no branch separates them.
                ld(plan, c < plan.n_chunks ? c : plan.n_chunks - 1, g, x[g]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) x[g][q] = 0;
                if (c < plan.n_chunks) ld(plan, c, g, x[g]);
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t c = c0 + g;
            if (c >= plan.n_chunks) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const WordOp &op = plan.op[4 * c + q];
                if (op.m == 0) continue;
                uint32_t v = (Loader::kRaw ? __builtin_bswap32(x[g][q]) : x[g][q]) & op.m;
                if (op.m != 0xFFFFFFFFu) {
#pragma unroll
                    for (int s = 0; s < 5; ++s) {
                        const uint32_t t = v & op.mv[s];
                        v = (v ^ t) | (t >> (1u << s));
                    }
                }
                // append the op.pc low bits of v at bit op.off of the compressed string
                const uint32_t o = op.off & 63u, end = o + op.pc;
                if ((op.off >> 6) != kw) {  // the previous output word is complete
                    store(kw, acc);
                    acc = 0;
                    kw = op.off >> 6;
                }
                if (end <= 64) {
                    acc |= uint64_t(v) << (64 - end);
                } else {  // straddles two output words
                    store(kw, acc | (uint64_t(v) >> (end - 64)));
                    ++kw;
                    acc = uint64_t(v) << (128 - end);
                }
            }
        }
    }
    store(kw, acc);
    for (uint32_t kk = plan.word_end; kk < plan.zero_end; ++kk) ck[uint64_t(kk) * n + i] = 0;
    return w0;
}

template <int MODE>
struct GlobalLoader {
    static constexpr bool kRaw = MODE != kLoadBytes;  // words as loaded (little-endian)
    const uint8_t *p;
    uint32_t len;
    __device__ __forceinline__ void operator()(const CompressPlan &plan, uint32_t c, int, uint32_t *x) const {
        const uint32_t cb = plan.chunk[c];
        if (MODE == kLoad16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p + 16 * cb);
            x[0] = v.x;
            x[1] = v.y;
            x[2] = v.z;
            x[3] = v.w;
        } else if (MODE == kLoad4) {
            // A word without D bits may lie past the row: it rereads the
            // key's first word instead (its value is not used).
#pragma unroll
            for (int q = 0; q < 4; ++q)
                x[q] = *reinterpret_cast<const uint32_t *>(plan.op[4 * c + q].m ? p + 16 * cb + 4 * q : p);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (plan.op[4 * c + q].m) x[q] = key_word_bytes(p, 4 * cb + q, len);
        }
    }
};

template <int MODE>
__global__ __launch_bounds__(kWG) void k_compress(KeySrc k, CompressPlan plan,
                                                  uint64_t *__restrict__ ck,
                                                  uint32_t *__restrict__ rowids,
                                                  uint32_t *__restrict__ flags) {
    const uint64_t i = uint64_t(blockIdx.x) * kWG + threadIdx.x;
    if (i >= k.n) return;
    GlobalLoader<MODE> ld{nullptr, k.L};
    if (MODE == kLoadBytes && k.offsets) {
        const uint64_t o0 = k.offsets[i], o1 = k.offsets[i + 1];
        ld.p = k.bytes + o0;
        if (o1 - o0 > k.L) {
            if (flags) atomicOr(flags, CKEY_FLAG_KEY_TOO_LONG);
        } else {
            ld.len = uint32_t(o1 - o0);
        }
    } else {
        ld.p = k.bytes + i * k.stride;
    }
    compress_key(plan, ld, ck, k.n, i);
    if (plan.write_rowids && rowids) rowids[i] = uint32_t(i);
}

// Variable-length keys: the workgroup's 256 keys occupy one contiguous byte
// range, which is copied to LDS with 16-byte loads; each thread then reads its
// key's words from LDS (byte-aligned, zero past the key's length).
constexpr uint32_t kVarTileBytes = 256 * 128;  // keys up to 128 bytes on average per tile

struct LdsLoader {
    static constexpr bool kRaw = false;
    const uint32_t *s;  // LDS tile, little-endian words
    uint32_t o;         // key's first byte in the tile
    uint32_t len;
    __device__ __forceinline__ uint32_t word(uint32_t j) const {
        const int32_t have = int32_t(len) - int32_t(4 * j);  // key bytes in this word
        if (have <= 0) return 0u;
        const uint32_t b = o + 4 * j;  // byte offset of the word in the tile (< o + len)
        const uint32_t lo = s[b >> 2], hi = s[(b >> 2) + 1];
        const uint32_t sh = 8 * (b & 3);
        const uint32_t le = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;  // bytes b..b+3, little-endian
        uint32_t v = __builtin_bswap32(le);
        if (have < 4) v &= ~(0xFFFFFFFFu >> (8 * have));
        return v;
    }
    __device__ __forceinline__ void operator()(const CompressPlan &plan, uint32_t c, int, uint32_t *x) const {
        const uint32_t cb = plan.chunk[c];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (plan.op[4 * c + q].m) x[q] = word(4 * cb + q);
    }
};

// A variable-length key read from the LDS tile (s non-null) or, for a
// workgroup whose keys exceed the tile, byte by byte from global memory.
struct VarLoader {
    static constexpr bool kRaw = false;
    const uint32_t *s;
    uint32_t o;
    uint32_t len;
    const uint8_t *p;
    __device__ __forceinline__ void operator()(const CompressPlan &plan, uint32_t c, int g, uint32_t *x) const {
        if (s) {
            LdsLoader{s, o, len}(plan, c, g, x);
        } else {
            const uint32_t cb = plan.chunk[c];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (plan.op[4 * c + q].m) x[q] = key_word_bytes(p, 4 * cb + q, len);
        }
    }
};

__global__ __launch_bounds__(kWG) void k_compress_var(KeySrc k, CompressPlan plan,
                                                      uint64_t *__restrict__ ck,
                                                      uint32_t *__restrict__ rowids,
                                                      uint32_t *__restrict__ flags) {
    // tile bytes + 16 for alignment + 8 zero bytes past the end for the word reads
    __shared__ uint32_t s_tile[(kVarTileBytes + 32) / 4];
    const uint64_t t0 = uint64_t(blockIdx.x) * kWG;
    const uint64_t t1 = min<uint64_t>(k.n, t0 + kWG);
    const uint64_t b0 = k.offsets[t0], b1 = k.offsets[t1];
    const uintptr_t base = reinterpret_cast<uintptr_t>(k.bytes);
    const uintptr_t a0 = (base + b0) & ~uintptr_t(15);  // aligned start (may precede b0)
    const uint64_t span = (base + b1) - a0;
    const bool fits = span <= kVarTileBytes;  // uniform
    if (fits) {
        // 16-byte chunks fully inside [base + b0 - pad, base + b1) are loaded as
        // vectors when they lie inside the key buffer; edge chunks byte by byte.
        // Every inside chunk's load is issued before any is stored, so a
        // thread's loads are in flight together; the edge chunks follow.
        const uint64_t nch = (span + 15) / 16;
        constexpr int kCh = (kVarTileBytes / 16 + kWG) / kWG;  // chunks per thread at most
        uint4 v[kCh];
#pragma unroll
        for (int q = 0; q < kCh; ++q) {
            const uint64_t c = threadIdx.x + uint64_t(q) * kWG;
            const uintptr_t addr = a0 + 16 * c;
            if (c < nch && addr >= base + b0 && addr + 16 <= base + b1) v[q] = *reinterpret_cast<const uint4 *>(addr);
        }
#pragma unroll
        for (int q = 0; q < kCh; ++q) {
            const uint64_t c = threadIdx.x + uint64_t(q) * kWG;
            if (c >= nch) break;
            const uintptr_t addr = a0 + 16 * c;
            if (addr < base + b0 || addr + 16 > base + b1) {
                uint32_t w[4] = {0, 0, 0, 0};
                for (int t = 0; t < 16; ++t) {
                    const uintptr_t bt = addr + t;
                    if (bt >= base + b0 && bt < base + b1)
                        w[t >> 2] |= uint32_t(*reinterpret_cast<const uint8_t *>(bt)) << (8 * (t & 3));
                }
                v[q] = make_uint4(w[0], w[1], w[2], w[3]);
            }
            s_tile[4 * c + 0] = v[q].x;
            s_tile[4 * c + 1] = v[q].y;
            s_tile[4 * c + 2] = v[q].z;
            s_tile[4 * c + 3] = v[q].w;
        }
        for (uint64_t c = 4 * nch + threadIdx.x; c < 4 * nch + 8; c += kWG) s_tile[c] = 0;
    }
    __syncthreads();
    const uint64_t i = t0 + threadIdx.x;
    if (i >= t1) return;
    const uint64_t o0 = k.offsets[i], o1 = k.offsets[i + 1];
    uint32_t len = uint32_t(min<uint64_t>(o1 - o0, k.L));
    if (o1 - o0 > k.L && flags) atomicOr(flags, CKEY_FLAG_KEY_TOO_LONG);
    // One loader for both cases (one compress_key instance keeps the plan in
    // the kernel-argument segment instead of a per-lane copy).
    VarLoader ld{fits ? s_tile : nullptr, uint32_t(fits ? base + o0 - a0 : 0), len, k.bytes + o0};
    compress_key(plan, ld, ck, k.n, i);
    if (plan.write_rowids && rowids) rowids[i] = uint32_t(i);
}

// Chunks already in registers, for keys of at most four 16-byte chunks (the
// compress loop then runs one group, whose slot g is the chunk index).
struct RegLoader {
    static constexpr bool kRaw = false;
    const uint4 *v;
    __device__ __forceinline__ void operator()(const CompressPlan &, uint32_t, int g, uint32_t *x) const {
        const uint4 u = v[g];
        x[0] = __builtin_bswap32(u.x);
        x[1] = __builtin_bswap32(u.y);
        x[2] = __builtin_bswap32(u.z);
        x[3] = __builtin_bswap32(u.w);
    }
};

// Compression fused with bucket assignment: persistent, each workgroup loads
// its thresholds into LDS once and takes the chunks of kFusedChunk keys
// blockIdx.x, + gridDim.x, ... (grid-stride over its threads); it finds
// each key's bucket from its first compressed word while it is in registers
// (learned: the network's guess, then the exact bucket; splitter: a search of
// the threshold sample in LDS, then of T in memory), and keeps a packed 16-bit
// bucket histogram in LDS, adding a pair of counters to the global histogram
// between chunks only where one of them could pass 65535 with the next
// chunk, and every pair after its last chunk.  (With every threshold in LDS the splitter's search
// is cheap enough that a separate assignment kernel over the first words,
// after a plain compression, is faster than this one-workgroup-per-CU kernel;
// with a sample, the search's reads of T overlap the compression's loads here.)
constexpr uint64_t kFusedChunk = 32 * kBucketWG;
static_assert(kFusedChunk <= 65535, "a chunk fits the 16-bit counters");
template <int MODE, int AMODE, int KPI>
__global__ __launch_bounds__(kBucketWG) void k_compress_bucket(KeySrc k, CompressPlan plan,
                                                               uint64_t *__restrict__ ck,
                                                               uint32_t *__restrict__ rowids,
                                                               BucketArgs ba) {
    extern __shared__ uint32_t s_dyn[];
    bucket_lds_init<AMODE>(ba, s_dyn);
    __syncthreads();
    for (uint64_t c = blockIdx.x; c * kFusedChunk < k.n; c += gridDim.x) {
        const uint64_t i0 = c * kFusedChunk;
        const uint64_t i1 = min<uint64_t>(k.n, i0 + kFusedChunk);
        if (KPI > 1) {
            // kLoad16 keys of at most four chunks, KPI keys per thread per
            // iteration: every key's loads are issued before any of them is
            // compressed, so their latencies overlap (a loop waits on its own
            // stores too, as loads and stores share one in-order counter).
            const uint64_t last = i1 - 1;
            for (uint64_t base = i0 + threadIdx.x; base < i1; base += uint64_t(KPI) * kBucketWG) {
                uint4 kc[KPI][4];
    #pragma unroll
                for (int q = 0; q < KPI; ++q) {
                    const uint64_t r = min<uint64_t>(base + uint64_t(q) * kBucketWG, last);
                    const uint8_t *p = k.bytes + r * k.stride;
    #pragma unroll
                    for (int c = 0; c < 4; ++c)  // unused slots reload chunk 0: in bounds, ignored
                        kc[q][c] = *reinterpret_cast<const uint4 *>(p + 16 * plan.chunk[uint32_t(c) < plan.n_chunks ? c : 0]);
                }
                uint64_t w0[KPI];
    #pragma unroll
                for (int q = 0; q < KPI; ++q) {
                    const uint64_t r = base + uint64_t(q) * kBucketWG;
                    w0[q] = 0;
                    if (r < i1) {
                        w0[q] = compress_key(plan, RegLoader{kc[q]}, ck, k.n, r);
                        if (plan.write_rowids && rowids) rowids[r] = uint32_t(r);
                    }
                }
                if (AMODE == 1 && ba.S == 1) {  // the keys' networks together, searches in LDS
                    uint32_t g[KPI];
                    predict_bucket_n<KPI>(ba.p, w0, ba.B, g);
    #pragma unroll
                    for (int q = 0; q < KPI; ++q) {
                        const uint64_t r = base + uint64_t(q) * kBucketWG;
                        // 2 x 512 buckets around the guess (the trained network's
                        // rank error is a few hundred buckets at 2^14)
                        const uint32_t b = correct_bucket_window<512>(reinterpret_cast<const uint64_t *>(s_dyn), ba.B, w0[q], g[q]);
                        if (r < i1) bucket_record<AMODE>(ba, s_dyn, b, r);
                    }
                } else if (AMODE == 1) {  // the keys' networks together, then T in memory searched from the guesses
                    uint32_t g[KPI], b[KPI];
                    predict_bucket_n<KPI>(ba.p, w0, ba.B, g);
                    correct_bucket_n<KPI>(ba.T, ba.B, w0, g, b);
    #pragma unroll
                    for (int q = 0; q < KPI; ++q) {
                        const uint64_t r = base + uint64_t(q) * kBucketWG;
                        if (r < i1) bucket_record<AMODE>(ba, s_dyn, b[q], r);
                    }
                } else if (AMODE == 0 && ba.S > 1) {  // the keys' sampled searches interleaved
                    uint32_t b[KPI];
                    splitter_search_sampled_n<KPI>(ba, s_dyn, w0, b);
    #pragma unroll
                    for (int q = 0; q < KPI; ++q) {
                        const uint64_t r = base + uint64_t(q) * kBucketWG;
                        if (r < i1) bucket_record<AMODE>(ba, s_dyn, b[q], r);
                    }
                } else {
    #pragma unroll
                    for (int q = 0; q < KPI; ++q) {
                        const uint64_t r = base + uint64_t(q) * kBucketWG;
                        if (r < i1) bucket_assign_one<AMODE>(ba, s_dyn, w0[q], r);
                    }
                }
            }
        } else {
            for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBucketWG) {
                GlobalLoader<MODE> ld{k.bytes + i * k.stride, k.L};
                const uint64_t w0 = compress_key(plan, ld, ck, k.n, i);
                if (plan.write_rowids && rowids) rowids[i] = uint32_t(i);
                bucket_assign_one<AMODE>(ba, s_dyn, w0, i);
            }
        }
        __syncthreads();
        const uint64_t nx = (c + gridDim.x) * kFusedChunk;
        bucket_lds_flush_before<AMODE>(ba, s_dyn, nx < k.n ? uint32_t(min<uint64_t>(kFusedChunk, k.n - nx)) : 0u);
        __syncthreads();  // counters cleared before the next chunk's records
    }
}

}  // namespace

ckey_status compress_bucket_launch(const KeySrc &k, const uint8_t *bm, uint64_t *ck, uint32_t words,
                                   uint32_t *rowids, uint32_t *flags, int amode, const BucketArgs &ba,
                                   hipStream_t st) {
    // Fused only for fixed-width keys whose compression fits one launch.
    const int mode = load_mode(k);
    std::vector<SrcWord> src;
    uint32_t nbits = 0, nch = 0, lc = UINT32_MAX;
    for (uint32_t j = 0; j < (k.L + 3) / 4; ++j) {
        uint32_t m = 0;
        for (uint32_t t = 0; t < 4; ++t) m = (m << 8) | (4 * j + t < k.L ? bm[4 * j + t] : 0u);
        if (!m) continue;
        src.push_back({j, m, nbits});
        nbits += __builtin_popcount(m);
        if (j / 4 != lc) { ++nch; lc = j / 4; }
    }
    const uint32_t w = nbits ? (nbits + 63) / 64 : 1;
    if (k.offsets || nch > uint32_t(kMaxChunks) || words < w) return CKEY_ERR_UNSUPPORTED;
    if (k.n == 0) return CKEY_OK;
    CompressPlan plan{};
    plan.write_rowids = 1;
    plan.word_begin = 0;
    plan.word_end = w;
    plan.zero_end = words;
    plan.kw_init = 0;
    uint32_t cidx = 0;
    lc = UINT32_MAX;
    for (const SrcWord &sw : src) {
        const uint32_t cb = sw.j / 4, q = sw.j % 4;
        if (cb != lc) {
            plan.chunk[cidx++] = cb;
            lc = cb;
        }
        WordOp &op = plan.op[4 * (cidx - 1) + q];
        op.m = sw.m;
        compress_masks(sw.m, op.mv);
        op.pc = __builtin_popcount(sw.m);
        op.off = sw.off;
    }
    plan.n_chunks = cidx;
    const size_t lds = bucket_lds_bytes(ba, amode);
    // One pass of workgroups resident at once (each loads its thresholds once).
    auto grid = [&](const void *fn) {
        return uint32_t(std::min<uint64_t>((k.n + kFusedChunk - 1) / kFusedChunk, resident_grid(fn, kBucketWG, lds)));
    };
    constexpr int kKPI = 4;  // keys per thread per iteration
    const bool multi = mode == kLoad16 && cidx <= 4;
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad16, 0, kKPI>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad16, 1, kKPI>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad16, 0, 1>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad16, 1, 1>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad4, 0, 1>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoad4, 1, 1>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoadBytes, 0, 1>));
    raise_lds_limit(reinterpret_cast<const void *>(k_compress_bucket<kLoadBytes, 1, 1>));
    const int pr_ = prof_begin(st, "compress_bucket");
#define CKEY_LAUNCH_CB(M, KPI)                                                                         \
    if (amode)                                                                                         \
        hipLaunchKernelGGL((k_compress_bucket<M, 1, KPI>),                                             \
                           dim3(grid(reinterpret_cast<const void *>(k_compress_bucket<M, 1, KPI>))),   \
                           dim3(kBucketWG), lds, st, k, plan, ck, rowids, ba);                         \
    else                                                                                               \
        hipLaunchKernelGGL((k_compress_bucket<M, 0, KPI>),                                             \
                           dim3(grid(reinterpret_cast<const void *>(k_compress_bucket<M, 0, KPI>))),   \
                           dim3(kBucketWG), lds, st, k, plan, ck, rowids, ba);
    switch (mode) {
        case kLoad16:
            if (multi) {
                CKEY_LAUNCH_CB(kLoad16, kKPI)
            } else {
                CKEY_LAUNCH_CB(kLoad16, 1)
            }
            break;
        case kLoad4: CKEY_LAUNCH_CB(kLoad4, 1) break;
        default: CKEY_LAUNCH_CB(kLoadBytes, 1) break;
    }
#undef CKEY_LAUNCH_CB
    prof_end(st, pr_);
    (void)flags;
    return launch_status();
}

ckey_status compress_launch(const KeySrc &k, const uint8_t *bm, uint64_t *ck, uint32_t words,
                            uint32_t *rowids, uint32_t *flags, hipStream_t st) {
    // Source words with D bits, in key order, with their offsets in the compressed string.
    std::vector<SrcWord> src;
    uint32_t nbits = 0;
    for (uint32_t j = 0; j < (k.L + 3) / 4; ++j) {
        uint32_t m = 0;
        for (uint32_t t = 0; t < 4; ++t) m = (m << 8) | (4 * j + t < k.L ? bm[4 * j + t] : 0u);
        if (!m) continue;
        src.push_back({j, m, nbits});
        nbits += __builtin_popcount(m);
    }
    const uint32_t w = nbits ? (nbits + 63) / 64 : 1;
    if (words < w) return CKEY_ERR_INVALID;
    if (k.n == 0) return CKEY_OK;
    const int mode = load_mode(k);
    const uint32_t blocks = uint32_t((k.n + kWG - 1) / kWG);

    // Each launch owns a range of output words [wb, we) and takes every source
    // word with a bit in it (at most kMaxChunks chunks); a source word that
    // straddles a range boundary is processed by both launches, each storing
    // only its own words.
    auto overlapping = [&](uint32_t wb, uint32_t we, size_t &a0, size_t &a1) {
        a0 = 0;
        while (a0 < src.size() && src[a0].off + __builtin_popcount(src[a0].m) <= 64 * wb) ++a0;
        a1 = a0;
        while (a1 < src.size() && src[a1].off < 64 * we) ++a1;
    };
    auto chunks_of = [&](size_t a0, size_t a1) {
        uint32_t nc = 0, lc = UINT32_MAX;
        for (size_t r = a0; r < a1; ++r)
            if (src[r].j / 4 != lc) { ++nc; lc = src[r].j / 4; }
        return nc;
    };
    uint32_t wb = 0;
    bool first = true;
    do {
        uint32_t we = wb + 1;
        size_t a0, a1;
        overlapping(wb, we, a0, a1);
        if (chunks_of(a0, a1) > uint32_t(kMaxChunks)) return CKEY_ERR_UNSUPPORTED;
        while (we < w) {
            size_t b0, b1;
            overlapping(wb, we + 1, b0, b1);
            if (chunks_of(b0, b1) > uint32_t(kMaxChunks)) break;
            ++we;
            a0 = b0;
            a1 = b1;
        }
        CompressPlan plan{};
        plan.write_rowids = first ? 1u : 0u;
        plan.word_begin = wb;
        plan.word_end = we;
        plan.zero_end = we == w ? words : 0u;
        plan.kw_init = a0 < a1 ? src[a0].off >> 6 : wb;
        uint32_t cidx = 0, lc = UINT32_MAX;
        for (size_t r = a0; r < a1; ++r) {
            const uint32_t cb = src[r].j / 4, q = src[r].j % 4;
            if (cb != lc) {
                plan.chunk[cidx++] = cb;
                lc = cb;
            }
            WordOp &op = plan.op[4 * (cidx - 1) + q];
            op.m = src[r].m;
            compress_masks(src[r].m, op.mv);
            op.pc = __builtin_popcount(src[r].m);
            op.off = src[r].off;
        }
        plan.n_chunks = cidx;
        {
            const int pr_ = prof_begin(st, "compress");
            switch (mode) {
                case kLoad16:
                    hipLaunchKernelGGL(k_compress<kLoad16>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    break;
                case kLoad4:
                    hipLaunchKernelGGL(k_compress<kLoad4>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    break;
                default:
                    if (k.offsets)
                        hipLaunchKernelGGL(k_compress_var, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    else
                        hipLaunchKernelGGL(k_compress<kLoadBytes>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    break;
            }
            prof_end(st, pr_);
        }
        CKEY_TRY(launch_status());
        first = false;
        wb = we;
    } while (wb < w);
    return CKEY_OK;
}

}  // namespace ckey
