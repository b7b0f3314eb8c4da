// DS-metadata maintenance (Sec. 4.3).
//
// Variant bitmap: the OR over all keys of (key xor reference key).  Each
// thread ORs its keys' words into registers, a group of kVG words at a time;
// the wave reduces them with shuffles and one lane ORs the result into a
// workgroup bitmap in LDS, which is OR-ed into the global accumulator once.
//
// Batched insert: inserting K between its neighbours A and B sets
// max(D-bit(A, K), D-bit(K, B)); the smaller one is D-bit(A, B) (Lemma 1),
// already in the bitmap.  For a whole batch, taken in key order, the bits
// added are those of the adjacent pairs of the merged order that contain a
// batch key: each batch key finds its place in the index by binary search
// (pos = number of index keys below it); its predecessor is the previous batch
// key when no index key lies between the two, else index key pos-1; when the
// next batch key does not share its place, index key pos is its successor.
// Deletes leave both bitmaps unchanged (Sec. 4.3): they need no kernel.
#include <algorithm>

#include "internal.h"

namespace ckey {

namespace {

constexpr uint32_t kVG = 16;  // words per register group of the variant kernel

struct KeyView {
    const uint8_t *p;
    uint32_t len;  // stored bytes (<= L); bytes past it read as zero
};

__device__ __forceinline__ KeyView key_view(const KeySrc &k, uint64_t r, bool &too_long) {
    if (k.offsets) {
        const uint64_t a = k.offsets[r], b = k.offsets[r + 1];
        too_long |= b - a > k.L;
        return KeyView{k.bytes + a, uint32_t(min<uint64_t>(b - a, k.L))};
    }
    return KeyView{k.bytes + r * k.stride, k.L};
}

// Big-endian word j of a key (zero past its length).  MODE kLoadBytes reads
// bytes; otherwise the key is 4-byte aligned and read by words.
template <int MODE>
__device__ __forceinline__ uint32_t view_word(const KeyView &v, uint32_t j) {
    if (4 * j >= v.len) return 0u;
    return MODE == kLoadBytes ? key_word_bytes(v.p, j, v.len) : key_word_aligned(v.p, j, v.len);
}

template <int MA, int MB>
__device__ __forceinline__ int64_t view_dbit(const KeyView &a, const KeyView &b, uint32_t nw) {
    for (uint32_t j = 0; j < nw; ++j) {
        const uint32_t x = view_word<MA>(a, j), y = view_word<MB>(b, j);
        if (x != y) return int64_t(32 * j + __clz(x ^ y));
    }
    return -1;
}

template <int MA, int MB>
__device__ __forceinline__ bool view_less(const KeyView &a, const KeyView &b, uint32_t nw) {
    for (uint32_t j = 0; j < nw; ++j) {
        const uint32_t x = view_word<MA>(a, j), y = view_word<MB>(b, j);
        if (x != y) return x < y;
    }
    return false;
}

template <int MODE>
__global__ __launch_bounds__(kWG) void k_variant(KeySrc k, const uint8_t *__restrict__ ref,
                                                 uint32_t *__restrict__ acc,
                                                 uint32_t *__restrict__ flags) {
    extern __shared__ uint32_t s_acc[];
    const uint32_t nw = (k.L + 3) / 4;
    for (uint32_t t = threadIdx.x; t < nw; t += kWG) s_acc[t] = 0;
    __syncthreads();
    bool too_long = false;
    const KeyView rv = ref ? KeyView{ref, k.L} : key_view(k, 0, too_long);
    const int lane = threadIdx.x & 63;
    // Byte-addressed keys in a 4-byte aligned buffer of `total` bytes: a
    // group's words come from the aligned words around them (else 0: bytes).
    const uint64_t total = (MODE == kLoadBytes && (reinterpret_cast<uintptr_t>(k.bytes) & 3u) == 0)
                               ? (k.offsets ? k.offsets[k.n] : k.n * uint64_t(k.stride))
                               : 0;
    const uint64_t step = uint64_t(gridDim.x) * kWG;
    for (uint32_t j0 = 0; j0 < nw; j0 += kVG) {
        uint32_t rw[kVG], a[kVG];
#pragma unroll
        for (uint32_t t = 0; t < kVG; ++t) {
            a[t] = 0;
            rw[t] = 0;
            if (j0 + t < nw)
                rw[t] = ref ? key_word_bytes(ref, j0 + t, k.L)
                            : view_word<MODE == kLoadBytes ? kLoadBytes : kLoad4>(rv, j0 + t);
            rw[t] = __builtin_amdgcn_readfirstlane(rw[t]);  // the same for every lane: scalar registers
        }
        for (uint64_t i = uint64_t(blockIdx.x) * kWG + threadIdx.x; i < k.n; i += step) {
            const KeyView v = key_view(k, i, too_long);
            if (MODE == kLoad16 && j0 + kVG <= nw) {
                // 16-byte aligned rows, the whole group inside the key: its
                // 128-bit loads are issued together, then combined.
                uint4 u[kVG / 4];
#pragma unroll
                for (uint32_t c = 0; c < kVG / 4; ++c)
                    u[c] = *reinterpret_cast<const uint4 *>(v.p + 4 * (j0 + 4 * c));
#pragma unroll
                for (uint32_t c = 0; c < kVG / 4; ++c) {
                    const uint32_t j = j0 + 4 * c;
                    const uint32_t w4[4] = {u[c].x, u[c].y, u[c].z, u[c].w};
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        const int32_t have = int32_t(v.len) - int32_t(4 * (j + q));
                        uint32_t x = have > 0 ? __builtin_bswap32(w4[q]) : 0u;
                        if (have > 0 && have < 4) x &= ~(0xFFFFFFFFu >> (8 * have));
                        a[4 * c + q] |= x ^ rw[4 * c + q];
                    }
                }
            } else if (MODE == kLoad16) {  // 16-byte aligned rows: 128-bit loads
#pragma unroll
                for (uint32_t c = 0; c < kVG / 4; ++c) {
                    const uint32_t j = j0 + 4 * c;
                    if (j >= nw) break;
                    const uint4 u = *reinterpret_cast<const uint4 *>(v.p + 4 * j);
                    const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        const int32_t have = int32_t(v.len) - int32_t(4 * (j + q));
                        uint32_t x = have > 0 ? __builtin_bswap32(w4[q]) : 0u;
                        if (have > 0 && have < 4) x &= ~(0xFFFFFFFFu >> (8 * have));
                        a[4 * c + q] |= x ^ rw[4 * c + q];
                    }
                }
            } else if (MODE == kLoadBytes && total && j0 < (v.len + 3) / 4 &&
                       4 * ((uint64_t(v.p - k.bytes) >> 2) + j0 + kVG + 1) <= total) {
                // The kVG + 1 aligned words around the group, loaded together,
                // then funnel-shifted into the key's big-endian words.
                const uint64_t o = uint64_t(v.p - k.bytes);
                const uint32_t *w = reinterpret_cast<const uint32_t *>(k.bytes) + (o >> 2) + j0;
                const uint32_t sh = 8 * uint32_t(o & 3);
                uint32_t u[kVG + 1];
#pragma unroll
                for (uint32_t t = 0; t <= kVG; ++t) u[t] = w[t];
#pragma unroll
                for (uint32_t t = 0; t < kVG; ++t) {
                    const int32_t have = int32_t(v.len) - int32_t(4 * (j0 + t));
                    uint32_t x = __builtin_bswap32(sh ? (u[t] >> sh) | (u[t + 1] << (32 - sh)) : u[t]);
                    x = have <= 0 ? 0u : have < 4 ? x & ~(0xFFFFFFFFu >> (8 * have)) : x;
                    if (j0 + t < nw) a[t] |= x ^ rw[t];
                }
            } else {
#pragma unroll
                for (uint32_t t = 0; t < kVG; ++t)
                    if (j0 + t < nw) a[t] |= view_word<MODE>(v, j0 + t) ^ rw[t];
            }
        }
#pragma unroll
        for (uint32_t t = 0; t < kVG; ++t) {
            uint32_t x = a[t];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) x |= __shfl_xor(x, off, 64);
            // the accumulator is the little-endian u32 view of the byte bitmap
            if (lane == 0 && x && j0 + t < nw) atomicOr(&s_acc[j0 + t], __builtin_bswap32(x));
        }
    }
    if (flags && too_long) atomicOr(flags, CKEY_FLAG_KEY_TOO_LONG);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nw; t += kWG)
        if (s_acc[t]) atomicOr(&acc[t], s_acc[t]);
}

__global__ void k_ref_copy(KeySrc k, uint8_t *__restrict__ out) {
    bool too_long = false;
    const KeyView v = k.n ? key_view(k, 0, too_long) : KeyView{nullptr, 0};
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k.L; j += gridDim.x * blockDim.x)
        out[j] = j < v.len ? v.p[j] : uint8_t(0);
}

__global__ void k_bitmap_or_finalize(const uint32_t *__restrict__ acc, uint8_t *__restrict__ bitmap,
                                     uint32_t L) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < L; j += gridDim.x * blockDim.x)
        bitmap[j] |= uint8_t(acc[j >> 2] >> (8 * (j & 3)));
}

template <int MI, int MB>
__global__ __launch_bounds__(kWG) void k_insert_pos(KeySrc ix, const uint32_t *__restrict__ ix_order,
                                                    KeySrc bt, const uint32_t *__restrict__ bt_order,
                                                    uint32_t *__restrict__ pos,
                                                    uint32_t *__restrict__ flags) {
    const uint64_t j = uint64_t(blockIdx.x) * kWG + threadIdx.x;
    if (j >= bt.n) return;
    bool too_long = false;
    const KeyView K = key_view(bt, bt_order ? bt_order[j] : j, too_long);
    const uint32_t nw = (bt.L + 3) / 4;
    uint64_t lo = 0, hi = ix.n;  // index keys [0, lo) are below K, [hi, n) are not
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        const KeyView A = key_view(ix, ix_order ? ix_order[mid] : mid, too_long);
        if (view_less<MI, MB>(A, K, nw)) lo = mid + 1; else hi = mid;
    }
    pos[j] = uint32_t(lo);
    if (flags && too_long) atomicOr(flags, CKEY_FLAG_KEY_TOO_LONG);
}

template <int MI, int MB>
__global__ __launch_bounds__(kWG) void k_insert_dbits(KeySrc ix, const uint32_t *__restrict__ ix_order,
                                                      KeySrc bt, const uint32_t *__restrict__ bt_order,
                                                      const uint32_t *__restrict__ pos,
                                                      uint32_t *__restrict__ acc) {
    extern __shared__ uint32_t s_bm[];
    const uint32_t nw = (bt.L + 3) / 4;
    for (uint32_t t = threadIdx.x; t < nw; t += kWG) s_bm[t] = 0;
    __syncthreads();
    bool too_long = false;
    const uint64_t step = uint64_t(gridDim.x) * kWG;
    for (uint64_t j = uint64_t(blockIdx.x) * kWG + threadIdx.x; j < bt.n; j += step) {
        const uint32_t p = pos[j];
        const KeyView K = key_view(bt, bt_order ? bt_order[j] : j, too_long);
        int64_t d = -1;
        if (j > 0 && pos[j - 1] == p) {  // no index key between the two batch keys
            const KeyView P = key_view(bt, bt_order ? bt_order[j - 1] : j - 1, too_long);
            d = view_dbit<MB, MB>(P, K, nw);
        } else if (p > 0) {
            const KeyView P = key_view(ix, ix_order ? ix_order[p - 1] : p - 1, too_long);
            d = view_dbit<MI, MB>(P, K, nw);
        }
        if (d >= 0) atomicOr(&s_bm[uint32_t(d) >> 5], bitmap_word_bit(uint32_t(d)));
        if (p < ix.n && (j + 1 == bt.n || pos[j + 1] > p)) {  // successor is index key p
            const KeyView S = key_view(ix, ix_order ? ix_order[p] : p, too_long);
            d = view_dbit<MB, MI>(K, S, nw);
            if (d >= 0) atomicOr(&s_bm[uint32_t(d) >> 5], bitmap_word_bit(uint32_t(d)));
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nw; t += kWG)
        if (s_bm[t]) atomicOr(&acc[t], s_bm[t]);
}

// kLoad16 and kLoad4 key sets are both read by aligned words here.
int word_mode(const KeySrc &k) { return load_mode(k) == kLoadBytes ? kLoadBytes : kLoad4; }

}  // namespace

ckey_status variant_launch(const KeySrc &k, const uint8_t *ref, uint32_t *acc, uint32_t *flags,
                           hipStream_t st) {
    if (k.n == 0) return CKEY_OK;
    const uint32_t nw = (k.L + 3) / 4;
    const size_t lds = nw * sizeof(uint32_t);
    // The grid-stride loop runs on the workgroups resident at once (a second
    // round of workgroups would start late and leave the tail uneven).
    const int mode = load_mode(k);
    const void *fn = mode == kLoad16 ? reinterpret_cast<const void *>(k_variant<kLoad16>)
                   : mode == kLoad4  ? reinterpret_cast<const void *>(k_variant<kLoad4>)
                                     : reinterpret_cast<const void *>(k_variant<kLoadBytes>);
    uint64_t blocks = (k.n + kWG - 1) / kWG;
    blocks = std::min<uint64_t>(blocks, resident_grid(fn, kWG, lds));
    const int pr = prof_begin(st, "variant");
    switch (mode) {
        case kLoad16:
            hipLaunchKernelGGL(k_variant<kLoad16>, dim3(uint32_t(blocks)), dim3(kWG), lds, st, k, ref, acc, flags);
            break;
        case kLoad4:
            hipLaunchKernelGGL(k_variant<kLoad4>, dim3(uint32_t(blocks)), dim3(kWG), lds, st, k, ref, acc, flags);
            break;
        default:
            hipLaunchKernelGGL(k_variant<kLoadBytes>, dim3(uint32_t(blocks)), dim3(kWG), lds, st, k, ref, acc, flags);
            break;
    }
    prof_end(st, pr);
    return launch_status();
}

ckey_status ref_copy_launch(const KeySrc &k, uint8_t *out, hipStream_t st) {
    hipLaunchKernelGGL(k_ref_copy, dim3((k.L + kWG - 1) / kWG), dim3(kWG), 0, st, k, out);
    return launch_status();
}

ckey_status bitmap_or_finalize(const uint32_t *acc, uint8_t *bitmap, uint32_t L, hipStream_t st) {
    hipLaunchKernelGGL(k_bitmap_or_finalize, dim3((L + kWG - 1) / kWG), dim3(kWG), 0, st, acc, bitmap, L);
    return launch_status();
}

ckey_status insert_launch(const KeySrc &ix, const uint32_t *ix_order, const KeySrc &bt,
                          const uint32_t *bt_order, uint32_t *pos, uint32_t *acc, uint32_t *flags,
                          hipStream_t st) {
    if (bt.n == 0) return CKEY_OK;
    const uint32_t nw = (bt.L + 3) / 4;
    const uint32_t pblocks = uint32_t((bt.n + kWG - 1) / kWG);
    uint64_t dblocks = (bt.n + kWG - 1) / kWG;
    if (dblocks > 2048) dblocks = 2048;
    const size_t lds = nw * sizeof(uint32_t);
    const int mi = word_mode(ix), mb = word_mode(bt);
#define CKEY_INSERT(MI, MB)                                                                             \
    {                                                                                                   \
        const int pr = prof_begin(st, "insert_pos");                                                    \
        hipLaunchKernelGGL((k_insert_pos<MI, MB>), dim3(pblocks), dim3(kWG), 0, st, ix, ix_order, bt,   \
                           bt_order, pos, flags);                                                       \
        prof_end(st, pr);                                                                               \
        const int pr2 = prof_begin(st, "insert_dbits");                                                 \
        hipLaunchKernelGGL((k_insert_dbits<MI, MB>), dim3(uint32_t(dblocks)), dim3(kWG), lds, st, ix,   \
                           ix_order, bt, bt_order, pos, acc);                                           \
        prof_end(st, pr2);                                                                              \
    }
    if (mi == kLoad4 && mb == kLoad4) CKEY_INSERT(kLoad4, kLoad4)
    else if (mi == kLoad4) CKEY_INSERT(kLoad4, kLoadBytes)
    else if (mb == kLoad4) CKEY_INSERT(kLoadBytes, kLoad4)
    else CKEY_INSERT(kLoadBytes, kLoadBytes)
#undef CKEY_INSERT
    return launch_status();
}

}  // namespace ckey
