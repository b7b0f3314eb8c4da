// Wave and workgroup scans by DPP moves (device code, included by the
// library's translation units through internal.h).  Kept in a header of its
// own so that a host build of a kernel can include the same code.
#pragma once

#include <stdint.h>

namespace ckey {

// Inclusive scan across a wave64 by DPP moves (no LDS, no lane addresses):
// shifts right by 1, 2, 4, 8 lanes within each 16-lane row (lanes shifted in
// from outside the row read 0), then lane 15's total is added to row 1 and
// row 3 (row_bcast:15) and lane 31's to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xF, 0xF, true));  // row_shr:1
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xF, 0xF, true));  // row_shr:2
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xF, 0xF, true));  // row_shr:4
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xF, 0xF, true));  // row_shr:8
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xA, 0xF, false)); // row_bcast:15
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xC, 0xF, false)); // row_bcast:31
    return v;
}

// Exclusive scan over the NT threads of a workgroup; all threads must call.
// s_tmp: NT/64 words of LDS.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_n(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
    const uint32_t incl = wave_incl_scan(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) s_tmp[wave] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const uint32_t t = s_tmp[w];
        off += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

// Exclusive scan over the 256 threads of a workgroup; all threads must call.
// s_tmp: 4 words of LDS.  Returns the exclusive prefix; `total` gets the sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
    return block_excl_scan_n<256>(v, s_tmp, total);
}

}  // namespace ckey
