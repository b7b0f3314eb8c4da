// D-bitmap refresh at index rebuild (Sec. 4.3) and per-pair distinction
// positions (Sec. 5.3).
//
// After the sort, the distinction position of adjacent compressed keys is
// c = 64*k + clz64(a_k xor b_k) for the first differing word k; D-offset[c]
// (the position of the (c+1)-st 1 of the input bitmap) maps it back to a
// full-key position.  Each workgroup rebuilds D-offset in LDS from the input
// bitmap (passed by value), then handles pairs in a grid-stride loop.
#include "internal.h"

namespace ckey {

namespace {

struct BitmapArg {
    uint8_t b[CKEY_MAX_KEY_BYTES];
};

__global__ __launch_bounds__(kWG) void k_refine(const uint64_t *__restrict__ ck, uint32_t words,
                                                uint64_t n, BitmapArg bm, uint32_t L, uint32_t nbits,
                                                uint32_t *__restrict__ acc,
                                                uint32_t *__restrict__ pair_pos) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint32_t s_tmp[4];
    const uint32_t nw = (L + 3) / 4;
    uint32_t *s_bm = s_dyn;                                   // nw words
    uint16_t *s_doff = reinterpret_cast<uint16_t *>(s_dyn + nw);  // nbits entries

    // D-offset table: thread t owns bitmap bytes [8t, 8t+8).
    const uint32_t tid = threadIdx.x;
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t j = 8 * tid + q;
        if (j < L) cnt += __popc(uint32_t(bm.b[j]));
    }
    uint32_t total;
    uint32_t c = block_excl_scan(cnt, s_tmp, total);
    for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t j = 8 * tid + q;
        if (j >= L) break;
        const uint32_t byte = bm.b[j];
        for (uint32_t t = 0; t < 8; ++t)
            if ((byte >> (7 - t)) & 1u) s_doff[c++] = uint16_t(8 * j + t);
    }
    for (uint32_t t = tid; t < nw; t += kWG) s_bm[t] = 0;
    __syncthreads();

    const uint64_t step = uint64_t(gridDim.x) * kWG;
    for (uint64_t i = 1 + uint64_t(blockIdx.x) * kWG + tid; i < n; i += step) {
        uint32_t pos = 0xFFFFFFFFu;
        for (uint32_t k = 0; k < words; ++k) {
            const uint64_t a = ck[uint64_t(k) * n + i - 1], b = ck[uint64_t(k) * n + i];
            if (a != b) {
                const uint32_t ci = 64 * k + uint32_t(__clzll(a ^ b));
                if (ci < nbits) {
                    pos = s_doff[ci];
                    atomicOr(&s_bm[pos >> 5], bitmap_word_bit(pos));
                }
                break;
            }
        }
        if (pair_pos) pair_pos[i - 1] = pos;
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
    uint64_t blocks = (n - 1 + kWG - 1) / kWG;
    if (blocks > 4096) blocks = 4096;
    {
        const int pr_ = prof_begin(st, "refine");
        hipLaunchKernelGGL(k_refine, dim3(uint32_t(blocks)), dim3(kWG), lds, st, ck, words, n, bm, L,
                           nbits, acc, pair_pos);
        prof_end(st, pr_);
    }
    return launch_status();
}

}  // namespace ckey
