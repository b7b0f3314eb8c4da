// D-bitmap refresh at index rebuild (Sec. 4.3) and per-pair distinction
// positions (Sec. 5.3).
//
// After the sort, the distinction position of adjacent compressed keys is
// c = 64*k + clz64(a_k xor b_k) for the first differing word k; D-offset[c]
// (the position of the (c+1)-st 1 of the input bitmap) maps it back to a
// full-key position.  Each workgroup rebuilds D-offset in LDS from the input
// bitmap (passed by value), then handles pairs in a grid-stride loop, four
// pairs per thread at a time; keys of at most 64 bytes collect their D-bits
// in a register bitmap per thread, OR-reduced across the wave.
#include <algorithm>

#include "internal.h"

namespace ckey {

namespace {

struct alignas(8) BitmapArg {
    uint8_t b[CKEY_MAX_KEY_BYTES];
};

constexpr uint32_t kRefineRegWords = 16;  // register bitmap: keys of at most 64 bytes

// RB: words of the per-thread register bitmap (kRefineRegWords when L <= 64),
// or 0: each D position ORed into the workgroup's LDS bitmap directly.
template <int RB>
__global__ __launch_bounds__(kWG) void k_refine(const uint64_t *__restrict__ ck, uint32_t words,
                                                uint64_t n, BitmapArg bm, uint32_t L, uint32_t nbits,
                                                uint32_t *__restrict__ acc,
                                                uint32_t *__restrict__ pair_pos) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint32_t s_tmp[4];
    const uint32_t nw = (L + 3) / 4;
    uint32_t *s_bm = s_dyn;                                   // nw words
    uint16_t *s_doff = reinterpret_cast<uint16_t *>(s_dyn + nw);  // nbits entries

    // D-offset table: thread t owns bitmap bytes [8t, 8t+8), read with one
    // 8-byte load (bytes at or past L are zero in the argument).
    static_assert(CKEY_MAX_KEY_BYTES == 8 * kWG, "one 8-byte group of the bitmap per thread");
    const uint32_t tid = threadIdx.x;
    const uint64_t b8 = *reinterpret_cast<const uint64_t *>(&bm.b[8 * tid]);
    uint32_t total;
    uint32_t c = block_excl_scan(uint32_t(__popcll(b8)), s_tmp, total);
    for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t j = 8 * tid + q;
        if (j >= L) break;
        const uint32_t byte = uint32_t(b8 >> (8 * q)) & 0xFFu;
        for (uint32_t t = 0; t < 8; ++t)
            if ((byte >> (7 - t)) & 1u) s_doff[c++] = uint16_t(8 * j + t);
    }
    for (uint32_t t = tid; t < nw; t += kWG) s_bm[t] = 0;
    __syncthreads();
    // With few bitmap words every pair's LDS OR would hit the same handful of
    // addresses: each thread ORs its pairs' bits into registers instead, and
    // the wave OR-reduces them before one LDS OR per word.
    uint32_t rb[RB > 0 ? RB : 1];
#pragma unroll
    for (int q = 0; q < (RB > 0 ? RB : 1); ++q) rb[q] = 0u;

    // Four pairs per thread at a time: their first words' loads are issued
    // together (unconditionally: a pair past the end rereads the last pair;
    // it is not used), later words only where the first words are equal.
    constexpr int kPairs = 4;
    const uint64_t step = uint64_t(gridDim.x) * kWG;
    for (uint64_t i0 = 1 + uint64_t(blockIdx.x) * kWG + tid; i0 < n; i0 += kPairs * step) {
        uint64_t a[kPairs], b[kPairs];
#pragma unroll
        for (int q = 0; q < kPairs; ++q) {
            const uint64_t i = min<uint64_t>(i0 + q * step, n - 1);
            a[q] = ck[i - 1];
            b[q] = ck[i];
        }
#pragma unroll
        for (int q = 0; q < kPairs; ++q) {
            const uint64_t i = i0 + q * step;
            if (i >= n) break;
            uint64_t x = a[q], y = b[q];
            uint32_t k = 0;
            while (x == y && ++k < words) {
                x = ck[uint64_t(k) * n + i - 1];
                y = ck[uint64_t(k) * n + i];
            }
            uint32_t pos = 0xFFFFFFFFu;
            if (x != y) {
                const uint32_t ci = 64 * k + uint32_t(__clzll(x ^ y));
                if (ci < nbits) {
                    pos = s_doff[ci];
                    const uint32_t bit = bitmap_word_bit(pos);
                    if constexpr (RB > 0) {
#pragma unroll
                        for (int w = 0; w < RB; ++w) rb[w] |= (pos >> 5) == uint32_t(w) ? bit : 0u;
                    } else {
                        atomicOr(&s_bm[pos >> 5], bit);
                    }
                }
            }
            if (pair_pos) pair_pos[i - 1] = pos;
        }
    }
    if constexpr (RB > 0) {
#pragma unroll
        for (int w = 0; w < RB; ++w) {
            uint32_t x = rb[w];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) x |= __shfl_xor(x, off, 64);
            if ((tid & 63) == 0 && x) atomicOr(&s_bm[w], x);
        }
    }
    __syncthreads();
    for (uint32_t t = tid; t < nw; t += kWG)
        if (s_bm[t]) atomicOr(&acc[t], s_bm[t]);
}

}  // namespace

ckey_status refine_launch(const uint64_t *ck, uint32_t words, uint64_t n, const uint8_t *bm_host,
                          uint32_t L, uint32_t *acc, uint32_t *pair_pos, uint32_t *flags,
                          hipStream_t st) {
    (void)flags;
    if (n < 2) return CKEY_OK;
    BitmapArg bm;
    uint32_t nbits = 0;
    for (uint32_t j = 0; j < CKEY_MAX_KEY_BYTES; ++j) {
        bm.b[j] = j < L ? bm_host[j] : 0;
        nbits += __builtin_popcount(bm.b[j]);
    }
    const uint32_t nw = (L + 3) / 4;
    const size_t lds = nw * sizeof(uint32_t) + ((nbits + 1) / 2) * sizeof(uint32_t);
    // The grid-stride loop runs on the workgroups resident at once.
    uint64_t blocks = (n - 1 + kWG - 1) / kWG;
    const bool reg = nw <= kRefineRegWords;
    const void *fn = reg ? reinterpret_cast<const void *>(k_refine<kRefineRegWords>)
                         : reinterpret_cast<const void *>(k_refine<0>);
    blocks = std::min<uint64_t>(blocks, resident_grid(fn, kWG, lds));
    {
        const int pr_ = prof_begin(st, "refine");
        if (reg)
            hipLaunchKernelGGL(k_refine<kRefineRegWords>, dim3(uint32_t(blocks)), dim3(kWG), lds, st, ck, words, n,
                               bm, L, nbits, acc, pair_pos);
        else
            hipLaunchKernelGGL(k_refine<0>, dim3(uint32_t(blocks)), dim3(kWG), lds, st, ck, words, n, bm, L, nbits,
                               acc, pair_pos);
        prof_end(st, pr_);
    }
    return launch_status();
}

}  // namespace ckey
