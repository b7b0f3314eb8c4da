// Stable LSD radix sort of (compressed key, row id) pairs (Sec. 3.2; the
// paper sorts with a comparison sort, Appendix A -- on the GPU a radix sort
// over the few meaningful bits moves far fewer bytes).
//
// Keys are `words` 64-bit words stored word-major; only the top `nbits` bits
// of the word string order the rows.  Digits are taken from the least
// significant meaningful bit upward, never straddling a word.
//
//   k_hist      one read of every key word: histograms of every digit pass.
//   k_scan      exclusive scan of each pass histogram -> global bucket starts.
//   k_onesweep  one pass per digit: a workgroup takes the next tile (atomic
//               tile counter), ranks keys stably with wave64 ballots,
//               publishes its per-bucket counts, looks back over the
//               predecessor tiles' published counts (decoupled look-back), and
//               scatters every word and the row id through an LDS reorder
//               buffer so each bucket's run is written contiguously.
//               Keys of 1..8 words take k_onesweep_pre (1024 threads, every
//               array loaded before any work, 4096..12288-key tiles: longer
//               runs per bucket and tile); wider keys take 4096-key tiles.
//
// The grouping by a 16-bit aux key (the bucket ids of the bucketing sort,
// aux_sort) uses the same pass kernels, but takes each tile's starts from a
// table instead of the look-back: k_tile_counts counts the pass digit per
// tile from the 2-byte aux key and k_tile_scan scans each digit's counts over
// the tiles; k_aux_hist derives both passes' starts from the full bucket
// histogram.
//
// The look-back waits only on tiles whose workgroups started earlier (tile
// numbers are handed out in start order), so every wait ends; a spin bound
// still guarantees termination and raises CKEY_FLAG_SPIN_LIMIT.
#include <vector>

#include "internal.h"

namespace ckey {

namespace {

constexpr int kRadixMax = 256;
constexpr int kKPT = 16;                  // keys per thread
constexpr int kTile = kWG * kKPT;         // 4096 keys per tile
constexpr int kWaves = kWG / 64;
constexpr uint32_t kFlagAgg = 1u << 30;   // tile aggregate published
constexpr uint32_t kFlagInc = 2u << 30;   // inclusive prefix published
constexpr uint32_t kValMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

constexpr uint32_t kRidWord = 0xFFFFu;  // Pass::word for a digit of the row id
constexpr uint32_t kAuxWord = 0xFFFEu;  // Pass::word for a digit of the 16-bit aux key

struct Pass {
    uint32_t word, shift, bits;  // digit = (word[i] >> shift) & (2^bits - 1)
};

// Buffers of one pass: word k of row i at base + k*ld + i.
struct Bufs {
    const uint64_t *src;
    const uint32_t *src_rid;
    uint64_t *dst;
    uint32_t *dst_rid;
    uint64_t src_ld, dst_ld;
    const uint16_t *src_aux;  // aux key: read by aux-digit passes,
    uint16_t *dst_aux;        // and moved along when dst_aux != nullptr
    const uint32_t *gate;     // nullptr, or a device word: 0 = the sort does nothing
};

struct HistArgs {
    uint32_t npass;
    uint32_t shift[8];
    uint32_t bits[8];
    uint32_t out[8];  // pass index of each digit
    const uint32_t *gate;
};

// A gated sort (the fallback of a captured bucketing sort) runs only when the
// device word says so: every kernel of it returns at once on a closed gate.
__device__ __forceinline__ bool gate_closed(const uint32_t *gate) { return gate && *gate == 0u; }

// Histograms of up to 8 digit passes of one key word: eight words per thread
// per round, all loaded before any is counted (eight loads in flight per
// thread instead of one), counted with LDS atomics, then added to `hist`.
template <typename T>
__global__ __launch_bounds__(kWG) void k_hist(const T *__restrict__ word, uint64_t n, HistArgs ha,
                                              uint32_t *__restrict__ hist) {
    constexpr int U = 8;
    __shared__ uint32_t s_h[8][kRadixMax];
    if (gate_closed(ha.gate)) return;
    for (int t = threadIdx.x; t < 8 * kRadixMax; t += kWG) (&s_h[0][0])[t] = 0;
    __syncthreads();
    const uint64_t step = uint64_t(gridDim.x) * kWG * U;
    for (uint64_t i0 = uint64_t(blockIdx.x) * kWG * U + threadIdx.x; i0 < n; i0 += step) {
        uint64_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + uint64_t(u) * kWG;
            x[u] = i < n ? uint64_t(word[i]) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + uint64_t(u) * kWG >= n) break;
            for (uint32_t p = 0; p < ha.npass; ++p) {
                const uint32_t d = uint32_t(x[u] >> ha.shift[p]) & ((1u << ha.bits[p]) - 1u);
                atomicAdd(&s_h[p][d], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < ha.npass * kRadixMax; t += kWG) {
        const uint32_t p = t / kRadixMax, d = t % kRadixMax;
        if (s_h[p][d]) atomicAdd(&hist[ha.out[p] * kRadixMax + d], s_h[p][d]);
    }
}

// One workgroup per pass: hist[p][*] -> exclusive prefix in place.
__global__ __launch_bounds__(kWG) void k_scan(uint32_t *__restrict__ hist, const uint32_t *gate) {
    __shared__ uint32_t s_tmp[4];
    if (gate_closed(gate)) return;
    uint32_t *h = hist + blockIdx.x * kRadixMax;
    const uint32_t v = h[threadIdx.x];
    uint32_t total;
    const uint32_t e = block_excl_scan(v, s_tmp, total);
    h[threadIdx.x] = e;
}

// Pass over keys wider than 8 words.  WC: a fixed word count to unroll, or 0
// (runtime `words`).
template <int WC>
__global__ __launch_bounds__(kWG) void k_onesweep(
    Bufs bf, uint64_t n, uint32_t words_rt, Pass ps, const uint32_t *__restrict__ bstart, uint32_t *lookback, uint32_t *tile_counter,
    uint32_t *flags) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wc[kWaves][kRadixMax];  // per-wave bucket counts, then offsets
    __shared__ uint32_t s_tstart[kRadixMax];      // tile-local bucket starts
    __shared__ uint32_t s_gbase[kRadixMax];       // global index of tile-local slot 0 per bucket
    __shared__ uint32_t s_tmp[4];
    __shared__ uint64_t s_buf[kTile];

    if (gate_closed(bf.gate)) return;
    const uint32_t words = WC > 0 ? uint32_t(WC) : words_rt;
    const uint64_t *__restrict__ src = bf.src;
    const uint32_t *__restrict__ src_rid = bf.src_rid;
    uint64_t *__restrict__ dst = bf.dst;
    uint32_t *__restrict__ dst_rid = bf.dst_rid;
    const bool rid_pass = ps.word == kRidWord;
    const bool aux_pass = ps.word == kAuxWord;
    const bool word_pass = !rid_pass && !aux_pass;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int t = tid; t < kWaves * kRadixMax; t += kWG) (&s_wc[0][0])[t] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = uint64_t(tile) * kTile;
    const uint32_t cnt = uint32_t(min<uint64_t>(kTile, n - base));
    const uint32_t dmask = (1u << ps.bits) - 1u;
    const uint64_t *dsrc = src + uint64_t(word_pass ? ps.word : 0) * bf.src_ld + base;
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    const uint32_t gstart = bstart[tid];  // read early: its latency overlaps the tile's loads

    uint64_t xv[kKPT];
    uint32_t dig[kKPT];
    uint32_t lpos[kKPT];
#pragma unroll
    for (int m = 0; m < kKPT; ++m) {
        const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
        xv[m] = li < cnt ? (word_pass ? dsrc[li]
                            : rid_pass ? uint64_t(src_rid ? src_rid[base + li] : uint32_t(base + li))
                                       : uint64_t(bf.src_aux[base + li]))
                         : 0ull;
        dig[m] = uint32_t(xv[m] >> ps.shift) & dmask;
    }

    // Stable rank within the wave: peers = lanes holding the same digit.
#pragma unroll
    for (int m = 0; m < kKPT; ++m) {
        const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
        const bool valid = li < cnt;
        uint64_t peers = __ballot(valid);
        for (uint32_t b = 0; b < ps.bits; ++b) {
            const bool bit = (dig[m] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = __popcll(peers & lane_lt);
        const uint32_t tot = __popcll(peers);
        uint32_t old = 0;
        if (valid) old = s_wc[wave][dig[m]];
        if (valid && below == 0) s_wc[wave][dig[m]] = old + tot;
        lpos[m] = old + below;
    }
    __syncthreads();

    // Thread `tid` owns bucket `tid`.
    {
        const uint32_t c0 = s_wc[0][tid], c1 = s_wc[1][tid], c2 = s_wc[2][tid], c3 = s_wc[3][tid];
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t *lb = lookback + uint64_t(tile) * kRadixMax + tid;
        __hip_atomic_store(lb, (tile == 0 ? kFlagInc : kFlagAgg) | tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        s_wc[0][tid] = 0;
        s_wc[1][tid] = c0;
        s_wc[2][tid] = c0 + c1;
        s_wc[3][tid] = c0 + c1 + c2;
        uint32_t all;
        const uint32_t tstart = block_excl_scan(tot, s_tmp, all);
        s_tstart[tid] = tstart;
        uint32_t excl = 0;
        if (tile > 0) {
            uint32_t j = tile - 1, spins = 0;
            for (;;) {
                const uint32_t e = __hip_atomic_load(lookback + uint64_t(j) * kRadixMax + tid,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = e & ~kValMask;
                if (f == 0) {
                    if (++spins > kSpinLimit) {
                        if (flags) atomicOr(flags, CKEY_FLAG_SPIN_LIMIT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += e & kValMask;
                if (f == kFlagInc || j == 0) break;
                --j;
            }
            __hip_atomic_store(lb, kFlagInc | (excl + tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_gbase[tid] = gstart + excl - tstart;
    }
    __syncthreads();

#pragma unroll
    for (int m = 0; m < kKPT; ++m) lpos[m] += s_tstart[dig[m]] + s_wc[wave][dig[m]];

    // Reorder and write: the digit word first (it yields each slot's bucket).
    uint32_t gdst[kKPT];
#pragma unroll
    for (int m = 0; m < kKPT; ++m) {
        const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
        if (li < cnt) s_buf[lpos[m]] = xv[m];
    }
    __syncthreads();
    uint64_t *ddst = dst + uint64_t(word_pass ? ps.word : 0) * bf.dst_ld;
#pragma unroll
    for (int m = 0; m < kKPT; ++m) {
        const uint32_t j = m * kWG + tid;
        gdst[m] = 0xFFFFFFFFu;
        if (j < cnt) {
            const uint64_t v = s_buf[j];
            gdst[m] = s_gbase[uint32_t(v >> ps.shift) & dmask] + j;
            // every index is < n unless a look-back gave up (CKEY_FLAG_SPIN_LIMIT)
            if (gdst[m] < n) {
                if (word_pass) ddst[gdst[m]] = v;
                else if (rid_pass) dst_rid[gdst[m]] = uint32_t(v);
                else if (bf.dst_aux) bf.dst_aux[gdst[m]] = uint16_t(v);
            }
        }
    }
    for (uint32_t k = 0; k < words; ++k) {
        if (word_pass && k == ps.word) continue;
        const uint64_t *ksrc = src + uint64_t(k) * bf.src_ld + base;
        uint64_t vv[kKPT];
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
            vv[m] = li < cnt ? ksrc[li] : 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
            if (li < cnt) s_buf[lpos[m]] = vv[m];
        }
        __syncthreads();
        uint64_t *kdst = dst + uint64_t(k) * bf.dst_ld;
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t j = m * kWG + tid;
            if (j < cnt && gdst[m] < n) kdst[gdst[m]] = s_buf[j];
        }
    }
    if (!rid_pass) {
        uint32_t rv[kKPT];
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
            rv[m] = li < cnt ? (src_rid ? src_rid[base + li] : uint32_t(base + li)) : 0u;
        }
        uint32_t *s_buf32 = reinterpret_cast<uint32_t *>(s_buf);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t li = wave * (kKPT * 64) + m * 64 + lane;
            if (li < cnt) s_buf32[lpos[m]] = rv[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kKPT; ++m) {
            const uint32_t j = m * kWG + tid;
            if (j < cnt && gdst[m] < n) dst_rid[gdst[m]] = s_buf32[j];
        }
    }
}

// The same pass for WC = 1..8 words with every array of the tile loaded into
// registers before any work: one memory round trip per tile instead of one per
// array, so the loads of all arrays overlap.  KPT keys per thread (fewer for
// more words, to fit the registers); each slot's digit is kept in LDS to find
// its destination.  NT threads: larger tiles make each bucket's run per tile
// longer, so the scattered writes come in longer pieces.
//
// offs (optional): each tile's global start per digit, offs[d * ntiles + tile],
// from k_tile_counts + k_tile_scan; the tile then needs no look-back.
// AUX: the pass digit is a digit of the 16-bit aux key (a bucket-id pass).
template <int WC, int KPT, int NT, bool AUX>
__global__ __launch_bounds__(NT) void k_onesweep_pre(
    Bufs bf, uint64_t n, Pass ps, const uint32_t *__restrict__ bstart, uint32_t *lookback,
    uint32_t *tile_counter, uint32_t *flags, const uint32_t *__restrict__ offs, uint32_t ntiles) {
    constexpr int TILE = NT * KPT;
    constexpr int NW = NT / 64;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wc[NW][kRadixMax];      // per-wave bucket counts, then offsets
    __shared__ uint32_t s_tstart[kRadixMax];      // tile-local bucket starts
    __shared__ uint32_t s_gbase[kRadixMax];       // global index of tile-local slot 0 per bucket
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint64_t s_buf[TILE];
    __shared__ uint8_t s_dig[TILE];               // digit of each slot, in slot order

    if (gate_closed(bf.gate)) return;
    const bool rid_pass = ps.word == kRidWord;
    const bool aux_pass = AUX;  // ps.word == kAuxWord
    const uint32_t rot = (AUX || rid_pass) ? 0u : ps.word;  // word held in register row 0
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int t = tid; t < NW * kRadixMax; t += NT) (&s_wc[0][0])[t] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = uint64_t(tile) * TILE;
    const uint32_t cnt = uint32_t(min<uint64_t>(TILE, n - base));
    const uint32_t dmask = (1u << ps.bits) - 1u;
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    // The bucket's global start (this tile's from offs, else the pass's) is
    // read before the tile, so that its latency overlaps the tile's loads.
    uint32_t gstart = 0;
    if (tid <= int(dmask)) gstart = offs ? offs[uint64_t(tid) * ntiles + tile] : bstart[tid];

    uint64_t wv[WC][KPT];
    uint32_t rv[KPT], av[KPT], dig[KPT], lpos[KPT];
    if constexpr (AUX) {
        // Every load of the tile is issued before any work, unconditionally:
        // slots past the end of the last tile read its last row (their
        // values are never used).  A select between a loaded value and a
        // constant would make each round of loads wait for the previous ones.
        // The bucket ids go first and the digits come from them alone: loads
        // retire in order, so the ranking waits for those loads only while
        // the other arrays' loads stay in flight.
        const uint32_t last = cnt - 1;
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t li = min(wave * (KPT * 64) + m * 64 + lane, last);
            av[m] = uint32_t(bf.src_aux[base + li]);
        }
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t li = min(wave * (KPT * 64) + m * 64 + lane, last);
#pragma unroll
            for (int k = 0; k < WC; ++k) wv[k][m] = bf.src[uint64_t(k) * bf.src_ld + base + li];
        }
#pragma unroll
        for (int m = 0; m < KPT; ++m) rv[m] = uint32_t(base) + wave * (KPT * 64) + m * 64 + lane;
        if (bf.src_rid) {  // else the pass generates the row ids
#pragma unroll
            for (int m = 0; m < KPT; ++m) {
                const uint32_t li = min(wave * (KPT * 64) + m * 64 + lane, last);
                rv[m] = bf.src_rid[base + li];
            }
        }
#pragma unroll
        for (int m = 0; m < KPT; ++m) dig[m] = (av[m] >> ps.shift) & dmask;
    } else {
        // The digit comes from a key word (or the row id).  Register row k
        // holds word (k + rot) mod WC, so the digit's word is row 0: its loads
        // go first and the digits come from it alone, the ranking waiting
        // for those loads only.  Every load is unconditional, as above.
        const uint32_t last = cnt - 1;
#pragma unroll
        for (int k = 0; k < WC; ++k) {
            const uint32_t kw = uint32_t(k) + rot < uint32_t(WC) ? uint32_t(k) + rot : uint32_t(k) + rot - WC;
#pragma unroll
            for (int m = 0; m < KPT; ++m) {
                const uint32_t li = min(wave * (KPT * 64) + m * 64 + lane, last);
                wv[k][m] = bf.src[uint64_t(kw) * bf.src_ld + base + li];
            }
        }
#pragma unroll
        for (int m = 0; m < KPT; ++m) rv[m] = uint32_t(base) + wave * (KPT * 64) + m * 64 + lane;
        if (bf.src_rid) {  // else the pass generates the row ids
#pragma unroll
            for (int m = 0; m < KPT; ++m) {
                const uint32_t li = min(wave * (KPT * 64) + m * 64 + lane, last);
                rv[m] = bf.src_rid[base + li];
            }
        }
#pragma unroll
        for (int m = 0; m < KPT; ++m) av[m] = 0u;
        if (rid_pass) {
#pragma unroll
            for (int m = 0; m < KPT; ++m) dig[m] = (rv[m] >> ps.shift) & dmask;
        } else {
#pragma unroll
            for (int m = 0; m < KPT; ++m) dig[m] = uint32_t(wv[0][m] >> ps.shift) & dmask;
        }
    }

    // Stable rank within the wave: peers = lanes holding the same digit.
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
        const uint32_t li = wave * (KPT * 64) + m * 64 + lane;
        const bool valid = li < cnt;
        uint64_t peers = __ballot(valid);
        for (uint32_t b = 0; b < ps.bits; ++b) {
            const bool bit = (dig[m] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = __popcll(peers & lane_lt);
        const uint32_t tot = __popcll(peers);
        uint32_t old = 0;
        if (valid) old = s_wc[wave][dig[m]];
        if (valid && below == 0) s_wc[wave][dig[m]] = old + tot;
        lpos[m] = old + below;
    }
    __syncthreads();

    // Thread `tid` < 256 owns bucket `tid`: publish, look back, global base.
    {
        uint32_t tot = 0;
        if (tid < kRadixMax) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = s_wc[w][tid];
                s_wc[w][tid] = tot;  // the wave's offset inside the tile's bucket run
                tot += c;
            }
        }
        uint32_t all;
        const uint32_t tstart = block_excl_scan_n<NT>(tot, s_tmp, all);
        if (tid < kRadixMax && offs) {
            s_tstart[tid] = tstart;
            s_gbase[tid] = gstart - tstart;
        } else if (tid < kRadixMax) {
            s_tstart[tid] = tstart;
            uint32_t *lb = lookback + uint64_t(tile) * kRadixMax + tid;
            __hip_atomic_store(lb, (tile == 0 ? kFlagInc : kFlagAgg) | tot, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            uint32_t excl = 0;
            if (tile > 0) {
                uint32_t j = tile - 1, spins = 0;
                for (;;) {
                    const uint32_t e = __hip_atomic_load(lookback + uint64_t(j) * kRadixMax + tid,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t f = e & ~kValMask;
                    if (f == 0) {
                        if (++spins > kSpinLimit) {
                            if (flags) atomicOr(flags, CKEY_FLAG_SPIN_LIMIT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    excl += e & kValMask;
                    if (f == kFlagInc || j == 0) break;
                    --j;
                }
                __hip_atomic_store(lb, kFlagInc | (excl + tot), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            s_gbase[tid] = gstart + excl - tstart;
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
        const uint32_t li = wave * (KPT * 64) + m * 64 + lane;
        lpos[m] += s_tstart[dig[m]] + s_wc[wave][dig[m]];
        if (li < cnt) s_dig[lpos[m]] = uint8_t(dig[m]);
    }
    __syncthreads();
    uint32_t gdst[KPT];
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
        const uint32_t j = m * NT + tid;
        // every index is < n unless a look-back gave up (CKEY_FLAG_SPIN_LIMIT)
        gdst[m] = j < cnt ? s_gbase[s_dig[j]] + j : 0xFFFFFFFFu;
    }
    // Reorder each array through LDS and write it in slot order.
#pragma unroll
    for (int k = 0; k < WC; ++k) {
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t li = wave * (KPT * 64) + m * 64 + lane;
            if (li < cnt) s_buf[lpos[m]] = wv[k][m];
        }
        __syncthreads();
        const uint32_t kw = uint32_t(k) + rot < uint32_t(WC) ? uint32_t(k) + rot : uint32_t(k) + rot - WC;
        uint64_t *kdst = bf.dst + uint64_t(kw) * bf.dst_ld;
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t j = m * NT + tid;
            if (j < cnt && gdst[m] < n) kdst[gdst[m]] = s_buf[j];
        }
        __syncthreads();
    }
    uint32_t *s_buf32 = reinterpret_cast<uint32_t *>(s_buf);
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
        const uint32_t li = wave * (KPT * 64) + m * 64 + lane;
        if (li < cnt) s_buf32[lpos[m]] = rv[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
        const uint32_t j = m * NT + tid;
        if (j < cnt && gdst[m] < n) bf.dst_rid[gdst[m]] = s_buf32[j];
    }
    if (aux_pass && bf.dst_aux) {
        uint16_t *s_buf16 = reinterpret_cast<uint16_t *>(s_buf32 + TILE);  // past the row ids
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t li = wave * (KPT * 64) + m * 64 + lane;
            if (li < cnt) s_buf16[lpos[m]] = uint16_t(av[m]);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < KPT; ++m) {
            const uint32_t j = m * NT + tid;
            if (j < cnt && gdst[m] < n) bf.dst_aux[gdst[m]] = s_buf16[j];
        }
    }
}

// Per-tile digit counts of a 16-bit aux key for one pass (cnt[d * ntiles + t]):
// one workgroup per tile, 8 keys per thread per load.
__global__ __launch_bounds__(1024) void k_tile_counts(const uint16_t *__restrict__ aux, uint64_t n,
                                                      uint32_t tile_keys, Pass ps, uint32_t ntiles,
                                                      uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_c[kRadixMax];
    const uint32_t t = blockIdx.x;
    for (int i = threadIdx.x; i < kRadixMax; i += 1024) s_c[i] = 0u;
    __syncthreads();
    const uint64_t base = uint64_t(t) * tile_keys;
    const uint32_t m = uint32_t(min<uint64_t>(tile_keys, n - base));
    const uint32_t mask = (1u << ps.bits) - 1u;
    for (uint32_t i = 8 * threadIdx.x; i < m; i += 8 * 1024) {
        if (i + 8 <= m) {  // base is a multiple of 1024: 16-byte aligned
            const uint4 v = *reinterpret_cast<const uint4 *>(aux + base + i);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                atomicAdd(&s_c[((w[k] & 0xFFFFu) >> ps.shift) & mask], 1u);
                atomicAdd(&s_c[((w[k] >> 16) >> ps.shift) & mask], 1u);
            }
        } else {
            for (uint32_t k = i; k < m; ++k) atomicAdd(&s_c[(uint32_t(aux[base + k]) >> ps.shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d <= mask; d += 1024) cnt[uint64_t(d) * ntiles + t] = s_c[d];
}

// Each digit's per-tile counts -> the tiles' global starts (exclusive scan
// over the tiles plus the digit's start), in place; one workgroup per digit.
__global__ __launch_bounds__(1024) void k_tile_scan(uint32_t *__restrict__ cnt, uint32_t ntiles,
                                                    const uint32_t *__restrict__ bstart) {
    __shared__ uint32_t s_tmp[16];
    const uint32_t d = blockIdx.x;
    uint32_t *row = cnt + uint64_t(d) * ntiles;
    const uint32_t per = (ntiles + 1023) / 1024;
    const uint32_t t0 = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (t0 + q < ntiles) sum += row[t0 + q];
    uint32_t tot;
    uint32_t run = block_excl_scan_n<1024>(sum, s_tmp, tot) + bstart[d];
    for (uint32_t q = 0; q < per; ++q)
        if (t0 + q < ntiles) {
            const uint32_t c = row[t0 + q];
            row[t0 + q] = run;
            run += c;
        }
}

// Keys per thread of the load-first pass kernel for a word count, and the
// tile each pass kernel uses (the load-first kernel moves the bucket-id
// passes; the radix passes keep the 4096-key tiles, measured faster there).
inline int pre_kpt(uint32_t words) {
    return words == 1 ? 12 : words == 2 ? 10 : words == 3 ? 8 : words <= 5 ? 6 : words == 6 ? 5 : 4;
}
constexpr int kPreNT = 1024;  // threads of the load-first kernel
// Passes over 1..8 words take the load-first kernel, wider keys the 256-thread one.
inline bool use_pre(uint32_t words) { return words >= 1 && words <= 8; }
// half: the half tile (512 threads, the same rows per thread) -- half the
// LDS, so two workgroups share a CU; an autotuning choice.
inline uint64_t pass_tile(uint32_t words, bool half = false) {
    return use_pre(words) ? uint64_t(half ? kPreNT / 2 : kPreNT) * pre_kpt(words) : uint64_t(kTile);
}

template <int NT, bool AUX>
void launch_pre(uint32_t words, dim3 g, hipStream_t st, const Bufs &bf, uint64_t n, const Pass &ps,
                const uint32_t *bstart, uint32_t *lookback, uint32_t *counter, uint32_t *flags,
                const uint32_t *offs, uint32_t nt) {
    const dim3 b(NT);
    switch (words) {
        case 1: hipLaunchKernelGGL((k_onesweep_pre<1, 12, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 2: hipLaunchKernelGGL((k_onesweep_pre<2, 10, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 3: hipLaunchKernelGGL((k_onesweep_pre<3, 8, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 4: hipLaunchKernelGGL((k_onesweep_pre<4, 6, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 5: hipLaunchKernelGGL((k_onesweep_pre<5, 6, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 6: hipLaunchKernelGGL((k_onesweep_pre<6, 5, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        case 7: hipLaunchKernelGGL((k_onesweep_pre<7, 4, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
        default: hipLaunchKernelGGL((k_onesweep_pre<8, 4, NT, AUX>), g, b, 0, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt); break;
    }
}

void launch_pass(uint32_t words, uint64_t tiles, const Bufs &bf, uint64_t n, const Pass &ps,
                 const uint32_t *bstart, uint32_t *lookback, uint32_t *counter, uint32_t *flags,
                 hipStream_t st, const uint32_t *offs = nullptr, bool half = false) {
    const uint32_t nt = uint32_t(tiles);
    const dim3 g = dim3(uint32_t(tiles));
    if (!use_pre(words)) {
        hipLaunchKernelGGL(k_onesweep<0>, g, dim3(kWG), 0, st, bf, n, words, ps, bstart, lookback, counter, flags);
        return;
    }
    if (ps.word == kAuxWord && !half)
        launch_pre<kPreNT, true>(words, g, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt);
    else if (ps.word == kAuxWord)
        launch_pre<kPreNT / 2, true>(words, g, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt);
    else if (half)
        launch_pre<kPreNT / 2, false>(words, g, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt);
    else
        launch_pre<kPreNT, false>(words, g, st, bf, n, ps, bstart, lookback, counter, flags, offs, nt);
}

__global__ void k_copy_back(Bufs bf, uint64_t n, uint32_t words) {
    if (gate_closed(bf.gate)) return;
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
        for (uint32_t k = 0; k < words; ++k)
            bf.dst[uint64_t(k) * bf.dst_ld + i] = bf.src[uint64_t(k) * bf.src_ld + i];
        bf.dst_rid[i] = bf.src_rid[i];
    }
}

// The passes of one sort: held inline (no heap allocation) up to
// kRadixInlinePasses, on the heap beyond.
class PassList {
  public:
    void clear() {
        n_ = 0;
        heap_.clear();
    }
    void push_back(const Pass &p) {
        if (n_ < kRadixInlinePasses) inl_[n_] = p;
        else heap_.push_back(p);
        ++n_;
    }
    size_t size() const { return n_; }
    const Pass &operator[](size_t i) const { return i < kRadixInlinePasses ? inl_[i] : heap_[i - kRadixInlinePasses]; }

  private:
    Pass inl_[kRadixInlinePasses];
    std::vector<Pass> heap_;
    size_t n_ = 0;
};

void make_passes(uint32_t words, uint32_t nbits, uint32_t d, uint32_t rid_bits, PassList &ps) {
    ps.clear();
    for (uint32_t s = 0; s < rid_bits;) {  // row-id digits are the least significant
        const uint32_t b = std::min<uint32_t>(d, rid_bits - s);
        ps.push_back({kRidWord, s, b});
        s += b;
    }
    for (int k = int(words) - 1; k >= 0; --k) {
        const int64_t have = int64_t(nbits) - 64 * int64_t(k);
        if (have <= 0) continue;
        const uint32_t bits_k = uint32_t(have > 64 ? 64 : have);
        uint32_t s = 64 - bits_k;
        while (s < 64) {
            const uint32_t b = std::min<uint32_t>(d, 64 - s);
            ps.push_back({uint32_t(k), s, b});
            s += b;
        }
    }
}

struct Layout {
    size_t alt_keys, alt_rid, hist, lookback, counters, total;
    uint64_t tiles;
    uint32_t npass;
};

Layout layout(uint32_t words, uint32_t nbits, uint64_t n, uint32_t d, uint32_t rid_bits, bool half) {
    PassList ps;
    make_passes(words, nbits, d, rid_bits, ps);
    Layout l{};
    l.npass = uint32_t(ps.size());
    l.tiles = (n + pass_tile(words, half) - 1) / pass_tile(words, half);
    size_t off = 0;
    l.alt_keys = off; off += align256(size_t(words) * n * 8);
    l.alt_rid = off;  off += align256(size_t(n) * 4);
    l.hist = off;     off += align256(size_t(l.npass) * kRadixMax * 4);
    l.lookback = off; off += align256(size_t(l.tiles) * kRadixMax * 4);
    l.counters = off; off += align256(size_t(l.npass) * 4);
    l.total = off;
    return l;
}

struct AuxLayout {
    size_t alt_keys, alt_rid, alt_aux, hist, lookback, counters, total;
    uint64_t tiles;
};

AuxLayout aux_layout(uint32_t words, uint64_t n) {
    AuxLayout l{};
    l.tiles = (n + pass_tile(words) - 1) / pass_tile(words);
    size_t off = 0;
    l.alt_keys = off; off += align256(size_t(words) * n * 8);
    l.alt_rid = off;  off += align256(size_t(n) * 4);
    l.alt_aux = off;  off += align256(size_t(n) * 2);
    l.hist = off;     off += align256(2 * kRadixMax * 4);
    l.lookback = off; off += align256(size_t(l.tiles) * kRadixMax * 4);
    l.counters = off; off += align256(2 * 4);
    l.total = off;
    return l;
}

}  // namespace

size_t aux_sort_workspace(uint32_t words, uint64_t n) { return aux_layout(words, n).total; }

// Pass starts of the two aux digits from a histogram over all 2^aux_bits aux
// values: thread d sums digit value d of the low pass and thread 256 + d of
// the high one, then each pass's 256 sums are scanned (exclusive) in place of
// a separate histogram + scan; the passes' tile counters are cleared too.
// LDS: the histogram is staged in LDS first (16-byte loads; 2^aux_bits <=
// 2^15), else the sums read it from global memory.
template <bool LDS>
__global__ __launch_bounds__(1024) void k_aux_hist(const uint32_t *__restrict__ full, uint32_t aux_bits,
                                                   uint32_t lo, uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ counters) {
    extern __shared__ uint32_t s_full[];
    __shared__ uint32_t s_tot[8];
    const uint32_t tid = threadIdx.x, hi = aux_bits - lo, m = 1u << aux_bits;
    const uint32_t *src = full;
    if (LDS) {
        for (uint32_t i = 4 * tid; i < m; i += 4 * 1024) {
            if (i + 4 <= m) {
                *reinterpret_cast<uint4 *>(s_full + i) = *reinterpret_cast<const uint4 *>(full + i);
            } else {
                for (uint32_t k = i; k < m; ++k) s_full[k] = full[k];
            }
        }
        __syncthreads();
        src = s_full;
    }
    const uint32_t pass = tid >> 8, d = tid & 255u;  // pass 0: low digit, 1: high digit
    uint32_t v = 0;
    if (pass == 0 && lo && d < (1u << lo))
        for (uint32_t h = 0; h < (1u << hi); ++h) v += src[(h << lo) | d];
    if (pass == 1 && d < (1u << hi))
        for (uint32_t l = 0; l < (1u << lo); ++l) v += src[(d << lo) | l];
    const uint32_t incl = wave_incl_scan(v);
    const uint32_t wave = tid >> 6, lane = tid & 63u;
    if (lane == 63 && wave < 8) s_tot[wave] = incl;
    __syncthreads();
    if (pass < 2) {
        uint32_t off = 0;
        for (uint32_t w = 4 * pass; w < wave; ++w) off += s_tot[w];
        const uint32_t ex = off + incl - v;
        if (lo)
            hist[pass * kRadixMax + d] = ex;
        else if (pass == 1)
            hist[d] = ex;
    }
    if (tid < 2) counters[tid] = 0u;
}

ckey_status aux_sort(uint64_t *ck, uint32_t *rid, bool rid_identity, const uint16_t *aux, uint64_t n,
                     uint32_t words, uint32_t aux_bits, const uint32_t *aux_full_hist, uint32_t *flags,
                     void *ws, hipStream_t st) {
    if (n < 2 || aux_bits == 0) return CKEY_OK;
    const AuxLayout l = aux_layout(words, n);
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    uint64_t *alt = reinterpret_cast<uint64_t *>(w8 + l.alt_keys);
    uint32_t *alt_rid = reinterpret_cast<uint32_t *>(w8 + l.alt_rid);
    uint16_t *alt_aux = reinterpret_cast<uint16_t *>(w8 + l.alt_aux);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w8 + l.hist);
    uint32_t *lookback = reinterpret_cast<uint32_t *>(w8 + l.lookback);
    uint32_t *counters = reinterpret_cast<uint32_t *>(w8 + l.counters);
    const uint32_t lo = aux_bits / 2, hi = aux_bits - lo;
    std::vector<Pass> ps;
    if (lo) ps.push_back({kAuxWord, 0, lo});
    ps.push_back({kAuxWord, lo, hi});
    HistArgs ha{};
    for (size_t p = 0; p < ps.size(); ++p) {
        ha.shift[p] = ps[p].shift;
        ha.bits[p] = ps[p].bits;
        ha.out[p] = uint32_t(p);
    }
    ha.npass = uint32_t(ps.size());
    if (aux_full_hist) {  // pass starts and cleared counters in one launch
        if (aux_bits <= 15) {
            raise_lds_limit(reinterpret_cast<const void *>(k_aux_hist<true>));
            hipLaunchKernelGGL(k_aux_hist<true>, dim3(1), dim3(1024), size_t(4) << aux_bits, st, aux_full_hist,
                               aux_bits, lo, hist, counters);
        } else {
            hipLaunchKernelGGL(k_aux_hist<false>, dim3(1), dim3(1024), 0, st, aux_full_hist, aux_bits, lo, hist,
                               counters);
        }
        CKEY_TRY(launch_status());
    } else {
        CKEY_TRY(fill_u32(hist, 2 * kRadixMax, 0, st));
        CKEY_TRY(fill_u32(counters, 2, 0, st));
        uint64_t hblocks = (n + kWG * 16 - 1) / (kWG * 16);
        if (hblocks > 2048) hblocks = 2048;
        const int pr_ = prof_begin(st, "hist");
        hipLaunchKernelGGL(k_hist<uint16_t>, dim3(uint32_t(hblocks)), dim3(kWG), 0, st, aux, n, ha, hist);
        prof_end(st, pr_);
        CKEY_TRY(launch_status());
        hipLaunchKernelGGL(k_scan, dim3(ha.npass), dim3(kWG), 0, st, hist, static_cast<const uint32_t *>(nullptr));
        CKEY_TRY(launch_status());
    }
    // With two passes: caller -> workspace (moving aux) -> caller.
    Bufs first{ck, rid_identity ? nullptr : rid, alt, alt_rid, n, n, aux, ps.size() == 2 ? alt_aux : nullptr};
    Bufs second{alt, alt_rid, ck, rid, n, n, alt_aux, nullptr};
    for (size_t p = 0; p < ps.size(); ++p) {
        const Bufs &bf = p == 0 ? first : second;
        const uint32_t *offs = nullptr;
        if (use_pre(words)) {
            // Tile starts from per-tile counts of the pass's digit (a read of
            // the 2-byte aux key) instead of a look-back chain across tiles.
            const int pc_ = prof_begin(st, "tile_counts");
            hipLaunchKernelGGL(k_tile_counts, dim3(uint32_t(l.tiles)), dim3(1024), 0, st, bf.src_aux, n,
                               uint32_t(pass_tile(words)), ps[p], uint32_t(l.tiles), lookback);
            hipLaunchKernelGGL(k_tile_scan, dim3(1u << ps[p].bits), dim3(1024), 0, st, lookback,
                               uint32_t(l.tiles), hist + p * kRadixMax);
            prof_end(st, pc_);
            offs = lookback;
        } else {
            CKEY_TRY(fill_u32(lookback, size_t(l.tiles) * kRadixMax, 0, st));
        }
        CKEY_TRY(launch_status());
        const int pr_ = prof_begin(st, "bucket_pass");
        launch_pass(words, l.tiles, bf, n, ps[p], hist + p * kRadixMax, lookback, counters + p, flags, st,
                    offs);
        prof_end(st, pr_);
        CKEY_TRY(launch_status());
    }
    if (ps.size() == 1) {  // one pass wrote the workspace: copy back
        Bufs back{alt, alt_rid, ck, rid, n, n, nullptr, nullptr};
        uint64_t blocks = (n + kWG - 1) / kWG;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_copy_back, dim3(uint32_t(blocks)), dim3(kWG), 0, st, back, n, words);
        CKEY_TRY(launch_status());
    }
    return CKEY_OK;
}

size_t radix_workspace(uint32_t words, uint32_t nbits, uint64_t n, uint32_t d, uint32_t rid_bits,
                       bool half_tile) {
    return layout(words, nbits, n, d, rid_bits, half_tile).total;
}

uint32_t radix_pass_count(uint32_t words, uint32_t nbits, uint32_t d) {
    uint32_t p = 0;
    for (uint32_t k = 0; k < words; ++k) {
        const int64_t have = int64_t(nbits) - 64 * int64_t(k);
        if (have > 0) p += (uint32_t(have > 64 ? 64 : have) + d - 1) / d;
    }
    return p;
}

ckey_status radix_sort(uint64_t *ck, uint64_t ld, uint32_t words, uint32_t nbits, uint32_t *rid,
                       uint64_t n, uint32_t d, uint32_t rid_bits, uint32_t *flags, void *ws,
                       hipStream_t st, bool skip_trivial, const uint32_t *gate, bool half_tile) {
    if (n < 2 || (nbits == 0 && rid_bits == 0)) return CKEY_OK;
    PassList ps;
    make_passes(words, nbits, d, rid_bits, ps);
    const Layout l = layout(words, nbits, n, d, rid_bits, half_tile);
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    uint64_t *alt = reinterpret_cast<uint64_t *>(w8 + l.alt_keys);
    uint32_t *alt_rid = reinterpret_cast<uint32_t *>(w8 + l.alt_rid);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w8 + l.hist);
    uint32_t *lookback = reinterpret_cast<uint32_t *>(w8 + l.lookback);
    uint32_t *counters = reinterpret_cast<uint32_t *>(w8 + l.counters);

    CKEY_TRY(fill_u32(hist, size_t(l.npass) * kRadixMax, 0, st, gate));
    CKEY_TRY(fill_u32(counters, l.npass, 0, st, gate));
    // Upfront histograms, grouped by source array, at most 8 digits per launch.
    uint64_t hblocks = (n + kWG * 16 - 1) / (kWG * 16);
    if (hblocks > 2048) hblocks = 2048;
    for (size_t p0 = 0; p0 < ps.size();) {
        HistArgs ha{};
        ha.gate = gate;
        const uint32_t wk = ps[p0].word;
        size_t p = p0;
        while (p < ps.size() && ps[p].word == wk && ha.npass < 8) {
            ha.shift[ha.npass] = ps[p].shift;
            ha.bits[ha.npass] = ps[p].bits;
            ha.out[ha.npass] = uint32_t(p);
            ++ha.npass;
            ++p;
        }
        {
            const int pr_ = prof_begin(st, "hist");
            if (wk == kRidWord)
                hipLaunchKernelGGL(k_hist<uint32_t>, dim3(uint32_t(hblocks)), dim3(kWG), 0, st, rid,
                                   n, ha, hist);
            else
                hipLaunchKernelGGL(k_hist<uint64_t>, dim3(uint32_t(hblocks)), dim3(kWG), 0, st,
                                   ck + uint64_t(wk) * ld, n, ha, hist);
            prof_end(st, pr_);
        }
        CKEY_TRY(launch_status());
        p0 = p;
    }
    std::vector<uint8_t> trivial;  // skip_trivial only: passes that leave the order as it is
    if (skip_trivial) {
        // A pass whose digit is the same for every row leaves the order as it is.
        std::vector<uint32_t> h(size_t(l.npass) * kRadixMax);
        CKEY_HIP_TRY(hipMemcpyAsync(h.data(), hist, h.size() * 4, hipMemcpyDeviceToHost, st));
        CKEY_HIP_TRY(hipStreamSynchronize(st));
        trivial.assign(ps.size(), 0);
        for (size_t p = 0; p < ps.size(); ++p)
            for (int b = 0; b < kRadixMax; ++b) trivial[p] |= h[p * kRadixMax + b] == n;
    }
    hipLaunchKernelGGL(k_scan, dim3(l.npass), dim3(kWG), 0, st, hist, gate);
    CKEY_TRY(launch_status());

    // Ping-pong between the caller's arrays (leading dimension ld) and the
    // workspace copy (leading dimension n).
    Bufs cur{ck, rid, alt, alt_rid, ld, n, nullptr, nullptr, gate};
    for (size_t p = 0; p < ps.size(); ++p) {
        if (!trivial.empty() && trivial[p]) continue;
        CKEY_TRY(fill_u32(lookback, size_t(l.tiles) * kRadixMax, 0, st, gate));
        {
            const int pr_ = prof_begin(st, "onesweep");
            launch_pass(words, l.tiles, cur, n, ps[p], hist + p * kRadixMax, lookback, counters + p,
                        flags, st, nullptr, half_tile);
            prof_end(st, pr_);
        }
        CKEY_TRY(launch_status());
        cur = Bufs{cur.dst, cur.dst_rid, const_cast<uint64_t *>(cur.src),
                   const_cast<uint32_t *>(cur.src_rid), cur.dst_ld, cur.src_ld, nullptr, nullptr, gate};
    }
    if (cur.src != ck) {
        uint64_t blocks = (n + kWG - 1) / kWG;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_copy_back, dim3(uint32_t(blocks)), dim3(kWG), 0, st, cur, n, words);
        CKEY_TRY(launch_status());
    }
    return CKEY_OK;
}

}  // namespace ckey
