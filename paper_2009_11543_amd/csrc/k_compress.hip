// Key compression (Sec. 3.2; extraction procedure of Sec. 5.1).
//
// The paper cuts the D-bitmap into 8-byte masks and applies x86 PEXT to each
// 8-byte slice of the key, joining the pieces with shift and OR.  gfx950 has
// no PEXT, but the masks are the same for every key, so the host turns them
// into a wave-uniform program once per call: every maximal run of 1-bits of
// the bitmap, cut at 32-bit source-word and 32-bit destination-half
// boundaries, becomes one (bit-field extract, shift, OR) step.  The program
// lives in the kernel argument segment and is read with scalar loads; each key
// costs one 128-bit load per 16 key bytes that hold D bits, one v_bfe_u32 and
// one shift-or per run, and one coalesced 64-bit store per output word.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace ckey {

namespace {

constexpr int kMaxRuns = 512;
constexpr int kMaxChunks = 64;

// Run encoding (one u32 per run).
constexpr uint32_t kRunLenShift = 5;     // bits 5..10: length 1..32
constexpr uint32_t kRunDstShift = 11;    // bits 11..15: destination shift inside the 32-bit half
constexpr uint32_t kRunHi = 1u << 16;    // destination is the high half of the 64-bit word
constexpr uint32_t kRunFlush = 1u << 17; // this run completes the output word
constexpr uint32_t kRunWhole = 1u << 18; // the run is the whole 32-bit source word

struct CompressPlan {
    uint32_t n_chunks;
    uint32_t word_begin;     // first output word this launch writes
    uint32_t zero_end;       // after the runs, zero-fill output words up to this one
    uint32_t write_rowids;
    uint16_t chunk[kMaxChunks];             // 16-byte source chunk index
    uint16_t run_begin[kMaxChunks * 4 + 1]; // runs of chunk c, word q: [run_begin[4c+q], run_begin[4c+q+1])
    uint32_t runs[kMaxRuns];
};

struct Run {
    uint32_t src_word;  // 32-bit source word index
    uint32_t code;
    uint32_t out_word;  // 64-bit output word index
};

// Decompose the bitmap into runs in output order.
void bitmap_runs(const uint8_t *bm, uint32_t L, std::vector<Run> &runs, uint32_t &nbits) {
    runs.clear();
    uint32_t c = 0;  // output bit index
    const uint32_t nw = (L + 3) / 4;
    for (uint32_t j = 0; j < nw; ++j) {
        uint32_t m = 0;
        for (uint32_t t = 0; t < 4; ++t) m = (m << 8) | (4 * j + t < L ? bm[4 * j + t] : 0u);
        uint32_t a = 0;  // MSB-based index inside the source word
        while (a < 32) {
            if (!((m >> (31 - a)) & 1u)) { ++a; continue; }
            uint32_t len = 0;
            while (a + len < 32 && ((m >> (31 - a - len)) & 1u)) ++len;
            // source bits [a, a+len) -> output bits [c, c+len), split at 32-bit output halves
            uint32_t done = 0;
            while (done < len) {
                uint32_t o = (c + done) & 63;
                uint32_t room = 32 - (o & 31);
                uint32_t part = std::min(len - done, room);
                uint32_t rshift = 32 - (a + done) - part;
                uint32_t dshift = 32 - (o & 31) - part;
                uint32_t code = rshift | (part << kRunLenShift) | (dshift << kRunDstShift) |
                                (o < 32 ? kRunHi : 0u) | (part == 32 ? kRunWhole : 0u);
                if (((c + done + part) & 63) == 0) code |= kRunFlush;
                runs.push_back({j, code, (c + done) >> 6});
                done += part;
            }
            c += len;
            a += len;
        }
    }
    nbits = c;
    if (!runs.empty()) runs.back().code |= kRunFlush;  // the last (possibly partial) word
}

template <int MODE>
__global__ __launch_bounds__(kWG) void k_compress(KeySrc k, CompressPlan plan,
                                                  uint64_t *__restrict__ ck,
                                                  uint32_t *__restrict__ rowids,
                                                  uint32_t *__restrict__ flags) {
    const uint64_t i = uint64_t(blockIdx.x) * kWG + threadIdx.x;
    if (i >= k.n) return;
    const uint8_t *p;
    uint32_t len = k.L;
    if (MODE == kLoadBytes && k.offsets) {
        const uint64_t o0 = k.offsets[i], o1 = k.offsets[i + 1];
        p = k.bytes + o0;
        if (o1 - o0 > k.L) {
            if (flags) atomicOr(flags, CKEY_FLAG_KEY_TOO_LONG);
        } else {
            len = uint32_t(o1 - o0);
        }
    } else {
        p = k.bytes + i * k.stride;
    }
    uint32_t lo = 0, hi = 0, kw = plan.word_begin;
    // Chunks are taken four at a time: all loads of a group are issued before
    // any of its output stores, so they overlap.
    for (uint32_t c0 = 0; c0 < plan.n_chunks; c0 += 4) {
        uint32_t x[4][4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t c = c0 + g;
#pragma unroll
            for (int q = 0; q < 4; ++q) x[g][q] = 0;
            if (c >= plan.n_chunks) continue;
            const uint32_t cb = plan.chunk[c];
            if (MODE == kLoad16) {
                const uint4 v = *reinterpret_cast<const uint4 *>(p + 16 * cb);
                x[g][0] = __builtin_bswap32(v.x);
                x[g][1] = __builtin_bswap32(v.y);
                x[g][2] = __builtin_bswap32(v.z);
                x[g][3] = __builtin_bswap32(v.w);
            } else if (MODE == kLoad4) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (plan.run_begin[4 * c + q] != plan.run_begin[4 * c + q + 1])
                        x[g][q] = __builtin_bswap32(*reinterpret_cast<const uint32_t *>(p + 16 * cb + 4 * q));
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (plan.run_begin[4 * c + q] != plan.run_begin[4 * c + q + 1])
                        x[g][q] = key_word_bytes(p, 4 * cb + q, len);
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t c = c0 + g;
            if (c >= plan.n_chunks) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t r1 = plan.run_begin[4 * c + q + 1];
                for (uint32_t r = plan.run_begin[4 * c + q]; r < r1; ++r) {
                    const uint32_t R = plan.runs[r];
                    uint32_t f = (R & kRunWhole) ? x[g][q]
                                                 : __builtin_amdgcn_ubfe(x[g][q], R & 31u, (R >> kRunLenShift) & 63u);
                    f <<= (R >> kRunDstShift) & 31u;
                    if (R & kRunHi) hi |= f; else lo |= f;
                    if (R & kRunFlush) {
                        ck[uint64_t(kw) * k.n + i] = (uint64_t(hi) << 32) | lo;
                        ++kw;
                        lo = hi = 0;
                    }
                }
            }
        }
    }
    for (; kw < plan.zero_end; ++kw) ck[uint64_t(kw) * k.n + i] = 0;
    if (plan.write_rowids && rowids) rowids[i] = uint32_t(i);
}

}  // namespace

ckey_status compress_launch(const KeySrc &k, const uint8_t *bm, uint64_t *ck, uint32_t words,
                            uint32_t *rowids, uint32_t *flags, hipStream_t st) {
    std::vector<Run> runs;
    uint32_t nbits = 0;
    bitmap_runs(bm, k.L, runs, nbits);
    const uint32_t w = nbits ? (nbits + 63) / 64 : 1;
    if (words < w) return CKEY_ERR_INVALID;
    if (k.n == 0) return CKEY_OK;
    const int mode = load_mode(k);
    const uint32_t blocks = uint32_t((k.n + kWG - 1) / kWG);

    // Greedily pack whole output words into launches that fit the argument block.
    size_t r0 = 0;
    bool first = true;
    do {
        CompressPlan plan{};
        plan.write_rowids = first ? 1u : 0u;
        plan.word_begin = runs.empty() ? 0u : runs[r0].out_word;
        size_t r1 = r0;
        // extend by whole output words while the limits hold
        while (r1 < runs.size()) {
            size_t e = r1;
            const uint32_t ow = runs[r1].out_word;
            while (e < runs.size() && runs[e].out_word == ow) ++e;
            // count chunks for [r0, e)
            uint32_t chunks = 0, last = UINT32_MAX;
            for (size_t r = r0; r < e; ++r) {
                uint32_t cb = runs[r].src_word / 4;
                if (cb != last) { ++chunks; last = cb; }
            }
            if ((e - r0) > size_t(kMaxRuns) || chunks > uint32_t(kMaxChunks)) {
                if (r1 == r0) return CKEY_ERR_UNSUPPORTED;  // one output word too large
                break;
            }
            r1 = e;
        }
        // fill the plan with runs [r0, r1)
        uint32_t nc = 0, last = UINT32_MAX;
        for (size_t r = r0; r < r1; ++r) {
            const uint32_t cb = runs[r].src_word / 4, q = runs[r].src_word % 4;
            if (cb != last) {
                plan.chunk[nc] = uint16_t(cb);
                for (int t = 0; t <= 4; ++t) plan.run_begin[4 * nc + t] = uint16_t(r - r0);
                ++nc;
                last = cb;
            }
            plan.runs[r - r0] = runs[r].code;
            // run r belongs to (chunk nc-1, word q): bump the ends of words q..3 of this chunk
            for (uint32_t t = q + 1; t <= 4; ++t) plan.run_begin[4 * (nc - 1) + t] = uint16_t(r - r0 + 1);
        }
        plan.n_chunks = nc;
        const bool last_launch = (r1 == runs.size());
        plan.zero_end = last_launch ? words : 0u;
        if (runs.empty()) plan.word_begin = 0;
        switch (mode) {
            case kLoad16:
                {
                    const int pr_ = prof_begin(st, "compress");
                    hipLaunchKernelGGL(k_compress<kLoad16>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    prof_end(st, pr_);
                }
                break;
            case kLoad4:
                {
                    const int pr_ = prof_begin(st, "compress");
                    hipLaunchKernelGGL(k_compress<kLoad4>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    prof_end(st, pr_);
                }
                break;
            default:
                {
                    const int pr_ = prof_begin(st, "compress");
                    hipLaunchKernelGGL(k_compress<kLoadBytes>, dim3(blocks), dim3(kWG), 0, st, k, plan, ck, rowids, flags);
                    prof_end(st, pr_);
                }
                break;
        }
        CKEY_TRY(launch_status());
        first = false;
        r0 = r1;
    } while (r0 < runs.size());
    return CKEY_OK;
}

}  // namespace ckey
