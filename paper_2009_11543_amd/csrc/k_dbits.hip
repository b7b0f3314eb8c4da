// Distinction bits of adjacent sorted keys (Sec. 3.1, Theorem 1).
//
// One thread per adjacent pair (i-1, i): the keys are compared as big-endian
// 32-bit words (read 16 bytes at a time when rows are 16-byte aligned); the
// first differing word gives the pair's D-bit as
// 32*j + clz(x xor y).  Keys of at most 64 bytes: each thread ORs its pairs'
// positions into a bitmap held in registers (16 u32), the wave OR-reduces it
// by lane shuffles, and one lane per wave ORs it into the workgroup's bitmap in
// LDS; longer keys OR each position into the LDS bitmap directly.  Each
// workgroup ORs its non-zero words into the global accumulator once.  A pair
// whose earlier key has a 1 at its D-bit is descending and raises
// CKEY_FLAG_DESCENDING.
#include "internal.h"

namespace ckey {

template <int MODE>
__device__ __forceinline__ uint32_t load_key_word(const KeySrc &k, uint64_t row, uint32_t j,
                                                  const uint8_t *&p, uint32_t &len) {
    return MODE == kLoadBytes ? key_word_bytes(p, j, len) : key_word_aligned(p, j, len);
}

// Word j of a key at any byte offset o of a 4-byte aligned buffer of `total`
// bytes: the two aligned 32-bit words around it, funnel-shifted, when both lie
// inside the buffer (else byte by byte); bytes at or past len read as zero.
__device__ __forceinline__ uint32_t key_word_unaligned(const uint8_t *bytes, uint64_t total, uint64_t o,
                                                       uint32_t j, uint32_t len) {
    const int32_t have = int32_t(len) - int32_t(4 * j);
    if (have <= 0) return 0u;
    const uint64_t b = o + 4 * uint64_t(j);
    const uint64_t wa = b >> 2;
    if (4 * (wa + 2) > total) return key_word_bytes(bytes + o, j, len);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(bytes);
    const uint32_t lo = w[wa], hi = w[wa + 1];
    const uint32_t sh = 8 * uint32_t(b & 3);
    uint32_t v = __builtin_bswap32(sh ? (lo >> sh) | (hi << (32 - sh)) : lo);
    if (have < 4) v &= ~(0xFFFFFFFFu >> (8 * have));
    return v;
}

constexpr uint32_t kDbitsRegWords = 16;  // register bitmap: keys of at most 64 bytes

// RB: words of the per-thread register bitmap (kDbitsRegWords, L <= 64), or 0.
template <int MODE, int RB>
__global__ __launch_bounds__(kWG) void k_dbits(KeySrc k, const uint32_t *__restrict__ order,
                                               uint32_t *__restrict__ acc,
                                               uint32_t *__restrict__ flags) {
    extern __shared__ uint32_t s_bm[];
    const uint32_t nw = (k.L + 3) / 4;
    for (uint32_t t = threadIdx.x; t < nw; t += kWG) s_bm[t] = 0;
    __syncthreads();
    uint32_t rb[RB > 0 ? RB : 1];
#pragma unroll
    for (int q = 0; q < (RB > 0 ? RB : 1); ++q) rb[q] = 0u;
    auto mark = [&](uint32_t p) {  // D-bit p of a pair
        const uint32_t bit = bitmap_word_bit(p);
        if constexpr (RB > 0) {
#pragma unroll
            for (int q = 0; q < RB; ++q) rb[q] |= (p >> 5) == uint32_t(q) ? bit : 0u;
        } else {
            atomicOr(&s_bm[p >> 5], bit);
        }
    };

    bool desc = false;
    bool too_long = false;
    const uint64_t step = uint64_t(gridDim.x) * kWG;
    // byte-addressed keys in a 4-byte aligned buffer: word reads (else 0: bytes)
    const uint64_t total = (MODE == kLoadBytes && (reinterpret_cast<uintptr_t>(k.bytes) & 3u) == 0)
                               ? (k.offsets ? k.offsets[k.n] : k.n * uint64_t(k.stride))
                               : 0;
    for (uint64_t i = 1 + uint64_t(blockIdx.x) * kWG + threadIdx.x; i < k.n; i += step) {
        const uint64_t ra = order ? order[i - 1] : i - 1;
        const uint64_t rb = order ? order[i] : i;
        const uint8_t *pa, *pb;
        uint32_t la, lb;
        if (k.offsets) {
            uint64_t a0 = k.offsets[ra], a1 = k.offsets[ra + 1];
            uint64_t b0 = k.offsets[rb], b1 = k.offsets[rb + 1];
            pa = k.bytes + a0;
            pb = k.bytes + b0;
            la = uint32_t(min<uint64_t>(a1 - a0, k.L));
            lb = uint32_t(min<uint64_t>(b1 - b0, k.L));
            too_long |= (a1 - a0 > k.L) | (b1 - b0 > k.L);
        } else {
            pa = k.bytes + ra * k.stride;
            pb = k.bytes + rb * k.stride;
            la = lb = k.L;
        }
        if (MODE == kLoad16) {
            // 16 bytes of both keys per step (rows are 16-byte aligned and
            // the stride a multiple of 16, so a chunk starting inside the key
            // stays inside the row); bytes at or past L read as zero.  The
            // first key's first chunk is the second key's of the pair one lane
            // down (pairs are consecutive across lanes), so each row's first
            // 16 bytes are read once; lane 0 reads its own.
            const uint4 vb0 = *reinterpret_cast<const uint4 *>(pb);
            uint4 va0;
            va0.x = __shfl_up(vb0.x, 1, 64);
            va0.y = __shfl_up(vb0.y, 1, 64);
            va0.z = __shfl_up(vb0.z, 1, 64);
            va0.w = __shfl_up(vb0.w, 1, 64);
            if ((threadIdx.x & 63) == 0) va0 = *reinterpret_cast<const uint4 *>(pa);
            for (uint32_t c = 0; 16 * c < k.L; ++c) {
                const uint4 va = c == 0 ? va0 : *reinterpret_cast<const uint4 *>(pa + 16 * c);
                const uint4 vb = c == 0 ? vb0 : *reinterpret_cast<const uint4 *>(pb + 16 * c);
                const uint32_t xa[4] = {va.x, va.y, va.z, va.w}, xb[4] = {vb.x, vb.y, vb.z, vb.w};
                bool done = false;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t j = 4 * c + uint32_t(q);
                    if (done || j >= nw) continue;
                    uint32_t x = __builtin_bswap32(xa[q]), y = __builtin_bswap32(xb[q]);
                    const uint32_t have = k.L - 4 * j;
                    if (have < 4) {
                        const uint32_t m = ~(0xFFFFFFFFu >> (8 * have));
                        x &= m;
                        y &= m;
                    }
                    if (x != y) {
                        const uint32_t lz = __clz(x ^ y);
                        const uint32_t p = 32 * j + lz;
                        desc |= ((x >> (31 - lz)) & 1u) != 0;
                        mark(p);
                        done = true;
                    }
                }
                if (done) break;
            }
            continue;
        }
        uint32_t j = 0;
        if (MODE == kLoadBytes && total) {
            // 16 key bytes of both keys per step: the five aligned words around
            // each key's next four are loaded together (while inside the
            // buffer), then funnel-shifted; the word-by-word loop below
            // finishes what is left.
            const uint32_t *w = reinterpret_cast<const uint32_t *>(k.bytes);
            const uint64_t oa = uint64_t(pa - k.bytes), ob = uint64_t(pb - k.bytes);
            const uint32_t sha = 8 * uint32_t(oa & 3), shb = 8 * uint32_t(ob & 3);
            bool done = false;
            for (; j + 4 <= nw; j += 4) {
                const uint64_t wa = (oa >> 2) + j, wb = (ob >> 2) + j;
                if (4 * (wa + 5) > total || 4 * (wb + 5) > total) break;
                uint32_t ua[5], ub[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    ua[q] = w[wa + q];
                    ub[q] = w[wb + q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t jq = j + uint32_t(q);
                    uint32_t x = __builtin_bswap32(sha ? (ua[q] >> sha) | (ua[q + 1] << (32 - sha)) : ua[q]);
                    uint32_t y = __builtin_bswap32(shb ? (ub[q] >> shb) | (ub[q + 1] << (32 - shb)) : ub[q]);
                    const int32_t ha = int32_t(la) - int32_t(4 * jq), hb = int32_t(lb) - int32_t(4 * jq);
                    x = ha <= 0 ? 0u : ha < 4 ? x & ~(0xFFFFFFFFu >> (8 * ha)) : x;
                    y = hb <= 0 ? 0u : hb < 4 ? y & ~(0xFFFFFFFFu >> (8 * hb)) : y;
                    if (!done && x != y) {
                        const uint32_t lz = __clz(x ^ y);
                        desc |= ((x >> (31 - lz)) & 1u) != 0;
                        mark(32 * jq + lz);
                        done = true;
                    }
                }
                if (done) break;
            }
            if (done) continue;
        }
        for (; j < nw; ++j) {
            uint32_t x, y;
            if (MODE == kLoadBytes && total) {
                x = key_word_unaligned(k.bytes, total, uint64_t(pa - k.bytes), j, la);
                y = key_word_unaligned(k.bytes, total, uint64_t(pb - k.bytes), j, lb);
            } else {
                x = load_key_word<MODE>(k, ra, j, pa, la);
                y = load_key_word<MODE>(k, rb, j, pb, lb);
            }
            if (x != y) {
                uint32_t lz = __clz(x ^ y);
                uint32_t p = 32 * j + lz;
                desc |= ((x >> (31 - lz)) & 1u) != 0;
                mark(p);
                break;
            }
        }
    }
    if (flags && (desc || too_long))
        atomicOr(flags, (desc ? CKEY_FLAG_DESCENDING : 0u) | (too_long ? CKEY_FLAG_KEY_TOO_LONG : 0u));
    if constexpr (RB > 0) {  // OR across the wave, then one lane per wave into LDS
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            uint32_t v = rb[q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v |= uint32_t(__shfl_xor(int(v), off, 64));
            rb[q] = v;
        }
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (rb[q]) atomicOr(&s_bm[q], rb[q]);  // rb[q] != 0 only for q < nw
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nw; t += kWG)
        if (s_bm[t]) atomicOr(&acc[t], s_bm[t]);
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v, const uint32_t *gate) {
    if (gate && *gate == 0u) return;
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

__global__ void k_bitmap_finalize(const uint32_t *acc, uint8_t *bitmap, uint32_t L) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < L; j += gridDim.x * blockDim.x)
        bitmap[j] = uint8_t(acc[j >> 2] >> (8 * (j & 3)));
}

__global__ void k_flag_or(uint32_t *f, uint32_t v) { atomicOr(f, v); }

ckey_status fill_flag_or(uint32_t *flags, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_flag_or, dim3(1), dim3(1), 0, st, flags, v);
    return launch_status();
}

ckey_status fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st, const uint32_t *gate) {
    if (n == 0) return CKEY_OK;
    uint64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(uint32_t(blocks)), dim3(kWG), 0, st, p, n, v, gate);
    return launch_status();
}

ckey_status bitmap_finalize(const uint32_t *acc, uint8_t *bitmap, uint32_t L, hipStream_t st) {
    uint32_t blocks = (L + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_bitmap_finalize, dim3(blocks), dim3(kWG), 0, st, acc, bitmap, L);
    return launch_status();
}

ckey_status dbits_launch(const KeySrc &k, const uint32_t *order, uint32_t *acc, uint32_t *flags,
                         hipStream_t st) {
    if (k.n < 2) return CKEY_OK;
    const uint32_t nw = (k.L + 3) / 4;
    uint64_t blocks = (k.n - 1 + kWG - 1) / kWG;
    if (blocks > 2048) blocks = 2048;
    const size_t lds = nw * sizeof(uint32_t);
    const bool reg = nw <= kDbitsRegWords;
#define CKEY_LAUNCH_DB(M)                                                                              \
    if (reg)                                                                                           \
        hipLaunchKernelGGL((k_dbits<M, kDbitsRegWords>), dim3(uint32_t(blocks)), dim3(kWG), lds, st, k, \
                           order, acc, flags);                                                         \
    else                                                                                               \
        hipLaunchKernelGGL((k_dbits<M, 0>), dim3(uint32_t(blocks)), dim3(kWG), lds, st, k, order, acc,  \
                           flags);
    const int pr_ = prof_begin(st, "dbits");
    switch (load_mode(k)) {
        case kLoadBytes: CKEY_LAUNCH_DB(kLoadBytes) break;
        case kLoad16: CKEY_LAUNCH_DB(kLoad16) break;
        default: CKEY_LAUNCH_DB(kLoad4) break;
    }
#undef CKEY_LAUNCH_DB
    prof_end(st, pr_);
    return launch_status();
}

}  // namespace ckey
