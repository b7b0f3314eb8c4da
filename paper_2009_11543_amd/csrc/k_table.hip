// Rebuild of every index of a table in one persistent kernel launch (Sec. 5
// steps 2-3: extract the compressed keys and sort the (compressed key, row id)
// pairs; Sec. 4.3: refresh the D-bitmap from the sorted keys), radix method.
//
// The workgroups of one launch take work items from a queue (an atomic
// counter).  Queue order is phase by phase, and within a phase index by index:
//   phase 0        compress: kTComp rows -> the index's compressed words
//                  (word-major) and, from the words while they are in
//                  registers, the digit histograms of all its radix passes
//                  (packed 16-bit counters in LDS, then global atomics)
//   phase 1        scan: each pass histogram -> exclusive bucket starts
//   phase 1+p      radix pass p (p = 1..P): one kTTile-row tile of a stable LSD
//                  scatter -- wave64 ballot ranks, the tile's per-digit totals
//                  published for a decoupled look-back over the earlier tiles,
//                  an LDS reorder so each digit's run is written contiguously
//   phase 2+P      refresh: one tile of adjacent sorted pairs -> each pair's
//                  D position (D-offset of the first differing compressed bit,
//                  Sec. 5.3), OR-ed into the new D-bitmap (Sec. 4.3)
//   phase 3+P      finalize: the accumulated bitmap -> bytes
// An item of phase h > 0 starts once every item of phase h-1 of its index has
// finished (a counter per phase); a pass tile also waits on the totals of the
// tiles before it.  Items are handed out in queue order and each wait is on
// earlier items, so the earliest unfinished item can always proceed and the
// launch drains whatever its grid size; every wait is still bounded
// (CKEY_FLAG_SPIN_LIMIT).
//
// Hand-offs between workgroups cross the XCDs' separate L2 caches: each
// thread of a finishing item writes its stores back at agent scope (release)
// before the item's counter is bumped, and a waiting item invalidates its
// caches (acquire) before it reads what earlier items wrote.
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace ckey {

namespace {

constexpr int kTKPT = 16;                    // rows per thread in a pass tile
constexpr uint32_t kTTile = kWG * kTKPT;     // rows per pass / refresh tile
constexpr uint32_t kTComp = 4 * kTTile;      // rows per compress item (< 2^16)
constexpr int kTWaves = kWG / 64;
constexpr uint32_t kTMaxIdx = CKEY_TABLE_MAX_INDEXES;
constexpr uint32_t kTMaxKB = CKEY_TABLE_MAX_KEY_BYTES;
constexpr uint32_t kTMaxPass = CKEY_TABLE_MAX_PASSES;
constexpr uint32_t kTMaxPhase = kTMaxPass + 4;
constexpr uint32_t kTMaxOps = kTMaxKB / 4;   // 32-bit source words
constexpr uint32_t kTMaxWords = kTMaxKB / 8; // compressed words
constexpr uint32_t kTSpin = 1u << 22;
constexpr uint32_t kTAgg = 1u << 30;         // tile total published
constexpr uint32_t kTInc = 2u << 30;         // inclusive prefix published
constexpr uint32_t kTVal = (1u << 30) - 1;

static_assert(kTMaxPass * 256 * 2 <= kTTile * 8, "pass histograms fit the reorder buffer");

// One index as the kernel sees it (a kernel argument).
struct TIdx {
    const uint8_t *bytes;
    const uint64_t *offsets;  // nullptr: fixed width
    uint64_t n;
    uint32_t L, stride;
    uint32_t nbits, words, d, npass;
    uint32_t ncomp, ntiles;   // compress items; pass / refresh tiles
    uint32_t aligned;         // fixed width with 4-byte aligned rows: 32-bit loads
    uint32_t pad;
    uint64_t *ck[2];          // compress writes ck[0]; pass p reads ck[(p-1)&1], writes ck[p&1]
    uint32_t *rid[2];         // pass 1 generates the row ids; rid[P&1] is the permutation
    uint32_t *hist;           // [P][256] pass histograms, then bucket starts
    uint32_t *lookback;       // [2][ntiles][256] published tile totals (pass p: array (p-1)&1)
    uint32_t *done;           // [kTMaxPhase] finished items per phase
    uint32_t *acc;            // (L+3)/4 words: the new D-bitmap, little-endian u32 view
    uint32_t *pair_pos;       // nullptr or [n-1]
    uint8_t *bitmap_out;      // nullptr or [L]
    uint32_t *flags;          // nullptr or device flags word
    uint8_t bm[kTMaxKB];      // bitmap the keys are compressed with
};

struct TArgs {
    uint32_t count, total;
    uint32_t *counter;                      // next item
    uint32_t phase_start[kTMaxPhase + 1];   // first item of each phase
    TIdx ix[kTMaxIdx];
};

__host__ __device__ inline uint32_t t_items(const TIdx &x, uint32_t ph) {
    if (ph == 0) return x.ncomp;
    if (ph == 1) return 1;
    if (ph <= 2 + x.npass) return x.ntiles;  // passes, then the refresh
    if (ph == 3 + x.npass) return 1;
    return 0;
}

struct TOp {        // one 32-bit big-endian source word holding D bits
    uint32_t j;     // word index in the key
    uint32_t m;     // its D bits
    uint32_t mv[5]; // bits moved right by 1, 2, 4, 8, 16 in the log-step compress
    uint32_t pc;    // popcount(m)
    uint32_t off;   // offset of its first selected bit in the compressed string
};

// Move masks of the log-step compress of the bits selected by m (Warren,
// Hacker's Delight, 2nd ed., Sec. 7-4).
__device__ void t_masks(uint32_t m, uint32_t *mv) {
    uint32_t mk = ~m << 1;
    for (int i = 0; i < 5; ++i) {
        uint32_t mp = mk ^ (mk << 1);
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        const uint32_t v = mp & m;
        mv[i] = v;
        m = (m ^ v) | (v >> (1u << i));
        mk &= ~mp;
    }
}

// Radix pass p (0-based) of an index: digits from the least significant
// meaningful bit upward, never straddling a 64-bit word.
struct TPass {
    uint32_t word, shift, bits;
};
__device__ __forceinline__ TPass t_pass(const TIdx &x, uint32_t p) {
    for (int k = int(x.words) - 1; k >= 0; --k) {
        const int have = int(x.nbits) - 64 * k;
        if (have <= 0) continue;
        uint32_t s = 64u - uint32_t(have > 64 ? 64 : have);
        while (s < 64) {
            const uint32_t b = min(x.d, 64u - s);
            if (p == 0) return TPass{uint32_t(k), s, b};
            --p;
            s += b;
        }
    }
    return TPass{0, 0, 1};
}

union TShared {
    struct {
        uint32_t wc[kTWaves][256];  // per-wave digit counts, then offsets
        uint32_t tstart[256];       // tile-local digit starts
        uint32_t gbase[256];        // global index of tile slot 0 of each digit
    } p;
    struct {
        TOp op[kTMaxOps];
        uint32_t nops;
        uint32_t wpass[kTMaxWords]; // first pass of each compressed word
    } c;
    struct {
        uint16_t doff[8 * kTMaxKB]; // D-offset: key position of each compressed bit
        uint32_t bm[kTMaxKB / 4];
    } r;
};

__device__ __forceinline__ void t_wait(uint32_t *cnt, uint32_t target, uint32_t *flags) {
    if (threadIdx.x == 0 && target > 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kTSpin) {
                if (flags) atomicOr(flags, CKEY_FLAG_SPIN_LIMIT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void t_signal(uint32_t *cnt) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Phase 0: compress rows [c*kTComp, ...) into ck[0]; histogram every pass digit.
__device__ __forceinline__ void t_compress(const TIdx &x, uint32_t c, TShared &u, uint32_t *h32) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        uint32_t nops = 0, off = 0;
        for (uint32_t j = 0; 4 * j < x.L; ++j) {
            uint32_t m = 0;
            for (uint32_t t = 0; t < 4; ++t) m = (m << 8) | (4 * j + t < x.L ? uint32_t(x.bm[4 * j + t]) : 0u);
            if (!m) continue;
            TOp &o = u.c.op[nops++];
            o.j = j;
            o.m = m;
            o.pc = uint32_t(__popc(m));
            o.off = off;
            off += o.pc;
            t_masks(m, o.mv);
        }
        u.c.nops = nops;
        uint32_t p = 0;  // passes run word w-1 first
        for (int k = int(x.words) - 1; k >= 0; --k) {
            u.c.wpass[k] = p;
            const int have = int(x.nbits) - 64 * k;
            if (have > 0) {
                const uint32_t bk = uint32_t(have > 64 ? 64 : have);
                p += (bk + x.d - 1) / x.d;
            }
        }
    }
    for (uint32_t t = tid; t < x.npass * 128; t += kWG) h32[t] = 0u;
    __syncthreads();
    const uint64_t r0 = uint64_t(c) * kTComp;
    const uint64_t r1 = min<uint64_t>(x.n, r0 + kTComp);
    const uint32_t nops = u.c.nops;
    bool too_long = false;
    for (uint64_t r = r0 + tid; r < r1; r += kWG) {
        const uint8_t *p;
        uint32_t len;
        if (x.offsets) {
            const uint64_t o0 = x.offsets[r], o1 = x.offsets[r + 1];
            p = x.bytes + o0;
            len = uint32_t(min<uint64_t>(o1 - o0, x.L));
            too_long |= o1 - o0 > x.L;
        } else {
            p = x.bytes + r * x.stride;
            len = x.L;
        }
        // Emit compressed word k of row r: store it and count its pass digits.
        auto emit = [&](uint32_t k, uint64_t v) {
            x.ck[0][uint64_t(k) * x.n + r] = v;
            const int have = int(x.nbits) - 64 * int(k);
            if (have <= 0 || x.npass == 0) return;
            uint32_t s = 64u - uint32_t(have > 64 ? 64 : have), q = u.c.wpass[k];
            while (s < 64) {
                const uint32_t b = min(x.d, 64u - s);
                const uint32_t dg = uint32_t(v >> s) & ((1u << b) - 1u);
                atomicAdd(&h32[(q * 256 + dg) >> 1], 1u << (16 * (dg & 1u)));
                ++q;
                s += b;
            }
        };
        uint64_t acc = 0;
        uint32_t kw = 0;
        for (uint32_t o = 0; o < nops; ++o) {
            const TOp &op = u.c.op[o];
            // word op.j of the key exists: 4*op.j < L, and for fixed width 4*op.j < len = L
            uint32_t v = (x.aligned ? key_word_aligned(p, op.j, len) : key_word_bytes(p, op.j, len)) & op.m;
            if (op.m != 0xFFFFFFFFu) {
#pragma unroll
                for (int s = 0; s < 5; ++s) {
                    const uint32_t t = v & op.mv[s];
                    v = (v ^ t) | (t >> (1u << s));
                }
            }
            const uint32_t o6 = op.off & 63u, end = o6 + op.pc;
            if ((op.off >> 6) != kw) {  // the previous word is complete
                emit(kw, acc);
                acc = 0;
                kw = op.off >> 6;
            }
            if (end <= 64) {
                acc |= uint64_t(v) << (64 - end);
            } else {  // straddles two words
                emit(kw, acc | (uint64_t(v) >> (end - 64)));
                ++kw;
                acc = uint64_t(v) << (128 - end);
            }
        }
        emit(kw, acc);
        for (uint32_t k = kw + 1; k < x.words; ++k) emit(k, 0ull);
    }
    if (too_long && x.flags) atomicOr(x.flags, CKEY_FLAG_KEY_TOO_LONG);
    __syncthreads();
    for (uint32_t t = tid; t < x.npass * 256; t += kWG) {
        const uint32_t v = (h32[t >> 1] >> (16 * (t & 1u))) & 0xFFFFu;
        if (v) atomicAdd(&x.hist[t], v);
    }
}

// Phase 1: exclusive scan of every pass histogram, in place.
__device__ __forceinline__ void t_scan(const TIdx &x, uint32_t *s_tmp) {
    for (uint32_t p = 0; p < x.npass; ++p) {
        uint32_t *h = x.hist + p * 256;
        const uint32_t v = h[threadIdx.x];
        uint32_t all;
        const uint32_t e = block_excl_scan(v, s_tmp, all);
        h[threadIdx.x] = e;
    }
}

// Radix pass p (1-based), tile t.
__device__ __forceinline__ void t_pass_tile(const TIdx &x, uint32_t p, uint32_t t, TShared &u, uint64_t *s_buf,
                            uint32_t *s_tmp) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t sb = (p - 1) & 1u, db = p & 1u;
    const uint64_t n = x.n;
    const uint64_t *src = x.ck[sb];
    const uint32_t *src_rid = p == 1 ? nullptr : x.rid[sb];
    uint64_t *dst = x.ck[db];
    uint32_t *dst_rid = x.rid[db];
    const uint64_t rowlen = uint64_t(x.ntiles) * 256;
    uint32_t *lb = x.lookback + sb * rowlen;
    if (p >= 2)  // pass p-1's look-back row is free again: clear it for pass p+1
        __hip_atomic_store(x.lookback + db * rowlen + uint64_t(t) * 256 + tid, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    const TPass ps = t_pass(x, p - 1);
    const uint32_t dmask = (1u << ps.bits) - 1u;
    const uint64_t base = uint64_t(t) * kTTile;
    const uint32_t cnt = uint32_t(min<uint64_t>(kTTile, n - base));
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    for (int q = tid; q < kTWaves * 256; q += kWG) (&u.p.wc[0][0])[q] = 0u;
    uint64_t xv[kTKPT];
    uint32_t dig[kTKPT], lpos[kTKPT];
    const uint64_t *dsrc = src + uint64_t(ps.word) * n + base;
#pragma unroll
    for (int m = 0; m < kTKPT; ++m) {
        const uint32_t li = uint32_t(wave) * (kTKPT * 64) + uint32_t(m) * 64 + uint32_t(lane);
        xv[m] = li < cnt ? dsrc[li] : 0ull;
        dig[m] = uint32_t(xv[m] >> ps.shift) & dmask;
    }
    __syncthreads();
    // Stable rank within the wave: peers = valid lanes holding the same digit.
#pragma unroll
    for (int m = 0; m < kTKPT; ++m) {
        const uint32_t li = uint32_t(wave) * (kTKPT * 64) + uint32_t(m) * 64 + uint32_t(lane);
        const bool valid = li < cnt;
        uint64_t peers = __ballot(valid);
        for (uint32_t b = 0; b < ps.bits; ++b) {
            const bool bit = (dig[m] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = uint32_t(__popcll(peers & lane_lt));
        uint32_t old = 0;
        if (valid) old = u.p.wc[wave][dig[m]];
        if (valid && below == 0) u.p.wc[wave][dig[m]] = old + uint32_t(__popcll(peers));
        lpos[m] = old + below;
    }
    __syncthreads();
    {  // thread tid owns digit tid
        const uint32_t c0 = u.p.wc[0][tid], c1 = u.p.wc[1][tid], c2 = u.p.wc[2][tid], c3 = u.p.wc[3][tid];
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t *me = lb + uint64_t(t) * 256 + tid;
        __hip_atomic_store(me, (t == 0 ? kTInc : kTAgg) | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u.p.wc[0][tid] = 0;
        u.p.wc[1][tid] = c0;
        u.p.wc[2][tid] = c0 + c1;
        u.p.wc[3][tid] = c0 + c1 + c2;
        uint32_t all;
        const uint32_t tstart = block_excl_scan(tot, s_tmp, all);
        u.p.tstart[tid] = tstart;
        uint32_t excl = 0;
        if (t > 0 && uint32_t(tid) <= dmask) {  // no tile holds a larger digit
            uint32_t j = t - 1, spins = 0;
            for (;;) {
                const uint32_t e = __hip_atomic_load(lb + uint64_t(j) * 256 + tid, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = e & ~kTVal;
                if (f == 0) {
                    if (++spins > kTSpin) {
                        if (x.flags) atomicOr(x.flags, CKEY_FLAG_SPIN_LIMIT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += e & kTVal;
                if (f == kTInc || j == 0) break;
                --j;
            }
            __hip_atomic_store(me, kTInc | (excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        u.p.gbase[tid] = x.hist[(p - 1) * 256 + tid] + excl - tstart;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kTKPT; ++m) lpos[m] += u.p.tstart[dig[m]] + u.p.wc[wave][dig[m]];
    // The digit word first: its reordered values give each slot's digit.
    uint32_t gdst[kTKPT];
#pragma unroll
    for (int m = 0; m < kTKPT; ++m) {
        const uint32_t li = uint32_t(wave) * (kTKPT * 64) + uint32_t(m) * 64 + uint32_t(lane);
        if (li < cnt) s_buf[lpos[m]] = xv[m];
    }
    __syncthreads();
    uint64_t *ddst = dst + uint64_t(ps.word) * n;
#pragma unroll
    for (int m = 0; m < kTKPT; ++m) {
        const uint32_t j = uint32_t(m) * kWG + uint32_t(tid);
        gdst[m] = 0xFFFFFFFFu;
        if (j < cnt) {
            const uint64_t v = s_buf[j];
            gdst[m] = u.p.gbase[uint32_t(v >> ps.shift) & dmask] + j;
            if (gdst[m] < n) ddst[gdst[m]] = v;  // < n unless a look-back gave up
        }
    }
    // The other words, then the row ids, through the same reorder.
    for (uint32_t k = 0; k <= x.words; ++k) {
        if (k == ps.word) continue;
        const bool is_rid = k == x.words;
        const uint64_t *ksrc = src + uint64_t(k) * n + base;
        uint64_t vv[kTKPT];
#pragma unroll
        for (int m = 0; m < kTKPT; ++m) {
            const uint32_t li = uint32_t(wave) * (kTKPT * 64) + uint32_t(m) * 64 + uint32_t(lane);
            vv[m] = 0ull;
            if (li < cnt)
                vv[m] = !is_rid ? ksrc[li] : src_rid ? uint64_t(src_rid[base + li]) : base + li;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kTKPT; ++m) {
            const uint32_t li = uint32_t(wave) * (kTKPT * 64) + uint32_t(m) * 64 + uint32_t(lane);
            if (li < cnt) s_buf[lpos[m]] = vv[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kTKPT; ++m) {
            const uint32_t j = uint32_t(m) * kWG + uint32_t(tid);
            if (j < cnt && gdst[m] < n) {
                if (is_rid) dst_rid[gdst[m]] = uint32_t(s_buf[j]);
                else dst[uint64_t(k) * n + gdst[m]] = s_buf[j];
            }
        }
    }
}

// Refresh tile t: pairs (i-1, i) for i in the tile; the permutation when
// there were no passes.
__device__ __forceinline__ void t_refine(const TIdx &x, uint32_t t, TShared &u, uint32_t *s_tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t f = x.npass & 1u;
    const uint64_t *ck = x.ck[f];
    const uint64_t n = x.n;
    {  // D-offset: thread tid owns bitmap byte tid
        const uint32_t byte = tid < x.L ? uint32_t(x.bm[tid]) : 0u;
        uint32_t all;
        uint32_t c = block_excl_scan(uint32_t(__popc(byte)), s_tmp, all);
        for (uint32_t b = 0; b < 8; ++b)
            if ((byte >> (7 - b)) & 1u) u.r.doff[c++] = uint16_t(8 * tid + b);
        if (tid < kTMaxKB / 4) u.r.bm[tid] = 0u;
    }
    __syncthreads();
    const uint64_t i0 = uint64_t(t) * kTTile, i1 = min<uint64_t>(n, i0 + kTTile);
    for (uint64_t i = i0 + tid; i < i1; i += kWG) {
        if (x.npass == 0) x.rid[0][i] = uint32_t(i);
        if (i == 0) continue;
        uint32_t pos = 0xFFFFFFFFu;
        for (uint32_t k = 0; k < x.words; ++k) {
            const uint64_t a = ck[uint64_t(k) * n + i - 1], b = ck[uint64_t(k) * n + i];
            if (a != b) {
                const uint32_t ci = 64 * k + uint32_t(__clzll(a ^ b));
                if (ci < x.nbits) {
                    pos = u.r.doff[ci];
                    atomicOr(&u.r.bm[pos >> 5], bitmap_word_bit(pos));
                }
                break;
            }
        }
        if (x.pair_pos) x.pair_pos[i - 1] = pos;
    }
    __syncthreads();
    if (tid < (x.L + 3) / 4 && u.r.bm[tid]) atomicOr(&x.acc[tid], u.r.bm[tid]);
}

__global__ __launch_bounds__(kWG) void k_table(TArgs a) {
    __shared__ uint64_t s_buf[kTTile];  // pass reorder; packed compress histograms
    __shared__ TShared u;
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_item[4];
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t q = atomicAdd(a.counter, 1u);
            uint32_t ph = 0, i = 0, r = 0;
            if (q < a.total) {
                while (q >= a.phase_start[ph + 1]) ++ph;
                r = q - a.phase_start[ph];
                for (;; ++i) {
                    const uint32_t c = t_items(a.ix[i], ph);
                    if (r < c) break;
                    r -= c;
                }
            }
            s_item[0] = q;
            s_item[1] = ph;
            s_item[2] = i;
            s_item[3] = r;
        }
        __syncthreads();
        const uint32_t q = __builtin_amdgcn_readfirstlane(s_item[0]);
        if (q >= a.total) break;
        const uint32_t ph = __builtin_amdgcn_readfirstlane(s_item[1]);
        const uint32_t i = __builtin_amdgcn_readfirstlane(s_item[2]);
        const uint32_t r = __builtin_amdgcn_readfirstlane(s_item[3]);
        const TIdx &x = a.ix[i];
        if (ph > 0) t_wait(x.done + ph - 1, t_items(x, ph - 1), x.flags);
        if (ph == 0)
            t_compress(x, r, u, reinterpret_cast<uint32_t *>(s_buf));
        else if (ph == 1)
            t_scan(x, s_tmp);
        else if (ph <= 1 + x.npass)
            t_pass_tile(x, ph - 1, r, u, s_buf, s_tmp);
        else if (ph == 2 + x.npass)
            t_refine(x, r, u, s_tmp);
        else if (x.bitmap_out)
            for (uint32_t j = threadIdx.x; j < x.L; j += kWG)
                x.bitmap_out[j] = uint8_t(x.acc[j >> 2] >> (8 * (j & 3)));
        t_signal(x.done + ph);  // its barrier also keeps s_item until every thread has read it
    }
}

uint32_t t_npass(uint32_t words, uint32_t nbits, uint32_t d) {
    uint32_t p = 0;
    for (uint32_t k = 0; k < words; ++k) {
        const int have = int(nbits) - 64 * int(k);
        if (have > 0) p += (uint32_t(have > 64 ? 64 : have) + d - 1) / d;
    }
    return p;
}

struct TLayout {
    size_t ctrl;                  // bytes of the cleared control block (at offset 0)
    size_t done[kTMaxIdx], hist[kTMaxIdx], acc[kTMaxIdx], lookback[kTMaxIdx];
    size_t ckf[kTMaxIdx], cko[kTMaxIdx], rid[kTMaxIdx];
    size_t total;
};

}  // namespace

ckey_status table_fused_plan(const TableIndex *ti, uint32_t count, void *ws, size_t *need,
                             hipStream_t st) {
    if (count == 0) return CKEY_ERR_INVALID;
    if (count > kTMaxIdx) return CKEY_ERR_UNSUPPORTED;
    TArgs a{};
    TLayout l{};
    size_t off = 256;  // the item counter
    a.count = count;
    for (uint32_t i = 0; i < count; ++i) {
        const TableIndex &t = ti[i];
        TIdx &x = a.ix[i];
        if (t.keys.L > kTMaxKB) return CKEY_ERR_UNSUPPORTED;
        if (t.keys.n >= (1ull << 30)) return CKEY_ERR_UNSUPPORTED;
        x.bytes = t.keys.bytes;
        x.offsets = t.keys.offsets;
        x.n = t.keys.n;
        x.L = t.keys.L;
        x.stride = t.keys.stride;
        for (uint32_t j = 0; j < kTMaxKB; ++j) x.bm[j] = j < x.L ? t.bitmap[j] : 0;
        x.nbits = 0;
        for (uint32_t j = 0; j < x.L; ++j) x.nbits += uint32_t(__builtin_popcount(x.bm[j]));
        x.words = x.nbits ? (x.nbits + 63) / 64 : 1;
        x.d = t.digit_bits;
        x.npass = x.n < 2 ? 0 : t_npass(x.words, x.nbits, x.d);
        if (x.npass > kTMaxPass) return CKEY_ERR_UNSUPPORTED;
        x.ncomp = uint32_t((x.n + kTComp - 1) / kTComp);
        x.ntiles = uint32_t((x.n + kTTile - 1) / kTTile);
        x.aligned = (!x.offsets && x.stride % 4 == 0 && reinterpret_cast<uintptr_t>(x.bytes) % 4 == 0) ? 1u : 0u;
        l.done[i] = off;     off += align256(kTMaxPhase * 4);
        l.hist[i] = off;     off += align256(size_t(x.npass) * 256 * 4);
        l.acc[i] = off;      off += align256(kTMaxKB);
        l.lookback[i] = off; off += align256(size_t(x.npass ? 2 : 0) * x.ntiles * 256 * 4);
    }
    l.ctrl = off;
    for (uint32_t i = 0; i < count; ++i) {
        const TIdx &x = a.ix[i];
        l.ckf[i] = l.cko[i] = l.rid[i] = SIZE_MAX;
        if (!ti[i].ckeys_out) { l.ckf[i] = off; off += align256(size_t(x.words) * x.n * 8); }
        if (x.npass >= 1) { l.cko[i] = off; off += align256(size_t(x.words) * x.n * 8); }
        if (x.npass >= 2) { l.rid[i] = off; off += align256(size_t(x.n) * 4); }
    }
    l.total = off;
    if (!ws) {
        *need = l.total;
        return CKEY_OK;
    }
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    // Phase starts: phase by phase, index by index.
    uint32_t nphase = 0;
    for (uint32_t i = 0; i < count; ++i) nphase = std::max(nphase, 4 + a.ix[i].npass);
    uint64_t q = 0;
    for (uint32_t ph = 0; ph <= kTMaxPhase; ++ph) {
        a.phase_start[ph] = uint32_t(q);
        if (ph < nphase)
            for (uint32_t i = 0; i < count; ++i) q += t_items(a.ix[i], ph);
    }
    if (q >= (1ull << 31)) return CKEY_ERR_UNSUPPORTED;
    a.total = uint32_t(q);
    a.counter = reinterpret_cast<uint32_t *>(w8);
    for (uint32_t i = 0; i < count; ++i) {
        TIdx &x = a.ix[i];
        const TableIndex &t = ti[i];
        const uint32_t f = x.npass & 1u;
        uint64_t *ckf = t.ckeys_out ? t.ckeys_out : reinterpret_cast<uint64_t *>(w8 + l.ckf[i]);
        x.ck[f] = ckf;
        x.ck[f ^ 1u] = x.npass >= 1 ? reinterpret_cast<uint64_t *>(w8 + l.cko[i]) : nullptr;
        x.rid[f] = t.perm;
        x.rid[f ^ 1u] = x.npass >= 2 ? reinterpret_cast<uint32_t *>(w8 + l.rid[i]) : nullptr;
        x.hist = reinterpret_cast<uint32_t *>(w8 + l.hist[i]);
        x.lookback = reinterpret_cast<uint32_t *>(w8 + l.lookback[i]);
        x.done = reinterpret_cast<uint32_t *>(w8 + l.done[i]);
        x.acc = reinterpret_cast<uint32_t *>(w8 + l.acc[i]);
        x.pair_pos = x.n > 1 ? t.pair_pos : nullptr;
        x.bitmap_out = t.bitmap_out;
        x.flags = t.flags;
        if (x.n > 0 && !x.rid[f]) return CKEY_ERR_INVALID;
    }
    CKEY_TRY(fill_u32(reinterpret_cast<uint32_t *>(w8), l.ctrl / 4, 0u, st));
    // As many workgroups as fit the GPU at once (any count drains the queue).
    int dev = 0, cus = 0, per_cu = 0;
    CKEY_HIP_TRY(hipGetDevice(&dev));
    CKEY_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CKEY_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_table, kWG, 0));
    uint32_t grid = uint32_t(cus > 0 ? cus : 1) * uint32_t(per_cu > 0 ? per_cu : 1);
    if (grid > a.total) grid = a.total ? a.total : 1;
    const int pr_ = prof_begin(st, "table_fused");
    hipLaunchKernelGGL(k_table, dim3(grid), dim3(kWG), 0, st, a);
    prof_end(st, pr_);
    return launch_status();
}

}  // namespace ckey
