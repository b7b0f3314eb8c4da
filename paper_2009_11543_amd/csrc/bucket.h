// Bucket assignment of a first compressed word x: the b with
// T[b] <= x < T[b+1] for a sorted threshold table T (T[0] = 0).  Used by the
// stand-alone assignment kernel and by compression fused with assignment.
//   splitter: binary search of a 1-in-S sample of T held in LDS, then of T;
//   learned:  a 4 -> 64 -> 1 ReLU MLP guesses b, then an exponential-then-
//             binary search of T from the guess finds it exactly (fused with
//             compression: a fixed-depth search of the buckets around the
//             guess, or of all of T when x lies outside them).
// Up to 2^14 buckets (S == 1) all of T is held in LDS for both methods.
#pragma once

#include "internal.h"

namespace ckey {

constexpr int kH = 64;                         // hidden units
constexpr int kBucketWG = 1024;                // threads per assigning workgroup
constexpr uint32_t kBucketKeysPerWG = 65535;   // keeps packed 16-bit LDS counters exact

struct BucketArgs {
    const float *p;        // MLP parameters (learned)
    const uint64_t *T;     // thresholds
    uint32_t B, S;         // bucket count, splitter sample stride
    uint16_t *bid;         // bucket ids (u16) or null
    uint32_t *bid32;       // bucket ids (u32) or null
    uint32_t *pred;        // network guesses or null (learned)
    uint32_t *hist;        // global bucket histogram (added to; 8-byte aligned) or null
};

// T[g] and T[g + 1] (g + 1 < B) in one 16-byte load: the pair lies in one
// 128-byte cache line unless T[g] is a line's last word (1 in 16), so a
// random pair costs one memory request instead of two.  The load needs only
// the 8-byte alignment of T.
struct alignas(8) TPair {
    uint64_t lo, hi;
};
__device__ __forceinline__ TPair load_tpair(const uint64_t *__restrict__ T, uint32_t g) {
    return *reinterpret_cast<const TPair *>(T + g);
}

// Splitter sample stride.  S == 1 means every threshold is held in LDS
// (B <= 2^14: 128 KB) and the search runs in LDS alone.
inline uint32_t splitter_stride(uint32_t B) {
    if (B <= (1u << 14)) return 1;
    return B / 16 > 2048 ? B / 2048 : 16;
}

// LDS layout: (splitter) the threshold sample, then (if a.hist) B/2 packed
// 16-bit counters.
inline size_t bucket_sample_words(const BucketArgs &a, int amode) {
    if (amode != 0) return a.S == 1 ? size_t(a.B) * 2 : 0;  // learned: all of T, or none
    return a.S == 1 ? size_t(a.B) * 2 : size_t(a.B / a.S) * 2;
}

inline size_t bucket_lds_bytes(const BucketArgs &a, int amode) {
    return bucket_sample_words(a, amode) * 4 + (a.hist ? size_t(a.B / 2) * 4 : 0);
}

__device__ __forceinline__ void mlp_features(uint64_t x, float f[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) f[j] = float(uint32_t(x >> (48 - 16 * j)) & 0xFFFFu) * (1.0f / 65536.0f);
}

__device__ __forceinline__ float mlp_eval(const float *__restrict__ p, const float f[4]) {
    float y = p[6 * kH];
#pragma unroll 16
    for (int k = 0; k < kH; ++k) {
        float a = p[4 * kH + k];
        a = fmaf(p[4 * k + 0], f[0], a);
        a = fmaf(p[4 * k + 1], f[1], a);
        a = fmaf(p[4 * k + 2], f[2], a);
        a = fmaf(p[4 * k + 3], f[3], a);
        y = fmaf(p[5 * kH + k], fmaxf(a, 0.0f), y);
    }
    return y;
}

__device__ __forceinline__ uint32_t predict_bucket(const float *__restrict__ p, uint64_t x, uint32_t B) {
    float f[4];
    mlp_features(x, f);
    const float y = mlp_eval(p, f) * float(B);
    if (!(y > 0.0f)) return 0;  // also maps NaN to 0
    if (y >= float(B)) return B - 1;
    return uint32_t(y);
}

// The network's guesses for N keys at once: each parameter is read once for
// all N keys; every key's arithmetic is in the same order as mlp_eval's, so
// the guesses equal predict_bucket's.
template <int N>
__device__ __forceinline__ void predict_bucket_n(const float *__restrict__ p, const uint64_t *x, uint32_t B,
                                                 uint32_t *guess) {
    float f[N][4], y[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        mlp_features(x[q], f[q]);
        y[q] = p[6 * kH];
    }
#pragma unroll 8
    for (int k = 0; k < kH; ++k) {
        const float w0 = p[4 * k + 0], w1 = p[4 * k + 1], w2 = p[4 * k + 2], w3 = p[4 * k + 3];
        const float b1 = p[4 * kH + k], v = p[5 * kH + k];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            float a = b1;
            a = fmaf(w0, f[q][0], a);
            a = fmaf(w1, f[q][1], a);
            a = fmaf(w2, f[q][2], a);
            a = fmaf(w3, f[q][3], a);
            y[q] = fmaf(v, fmaxf(a, 0.0f), y[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const float t = y[q] * float(B);
        guess[q] = !(t > 0.0f) ? 0u : t >= float(B) ? B - 1 : uint32_t(t);
    }
}

// Exact bucket from a start guess: exponential search outward, then binary.
__device__ __forceinline__ uint32_t correct_bucket(const uint64_t *__restrict__ T, uint32_t B,
                                                   uint64_t x, uint32_t pb, uint32_t &probes) {
    uint32_t lo, hi;  // T[lo] <= x and (hi == B or T[hi] > x)
    ++probes;
    if (T[pb] <= x) {
        lo = pb;
        hi = B;
        for (uint32_t step = 1;; step <<= 1) {
            const uint32_t j = lo + step;
            if (j >= B) break;
            ++probes;
            if (T[j] > x) { hi = j; break; }
            lo = j;
        }
    } else {
        hi = pb;
        lo = 0;  // T[0] = 0 <= x
        for (uint32_t step = 1;; step <<= 1) {
            if (hi <= step) break;
            const uint32_t j = hi - step;
            ++probes;
            if (T[j] <= x) { lo = j; break; }
            hi = j;
        }
    }
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        ++probes;
        if (T[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Exact buckets of N keys from guesses g, T in global memory (the learned
// method beyond 2^14 buckets): the guess and its right neighbour are read
// together; a miss gallops outward from the guess with doubling steps until
// the answer is bracketed, then halves the bracket.  Each round issues every
// key's read before any is used, so the reads overlap.  b[q] = the largest b
// with T[b] <= x[q] (T sorted, T[0] = 0), as correct_bucket returns.
template <int N>
__device__ __forceinline__ void correct_bucket_n(const uint64_t *__restrict__ T, uint32_t B, const uint64_t *x,
                                                 const uint32_t *g, uint32_t *b) {
    uint32_t lo[N], hi[N], step[N];  // T[lo] <= x; hi == B or T[hi] > x once bracketed
    int dir[N];                      // +1 galloping up, -1 down, 0 bracketed
    uint64_t t0[N], t1[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        if (g[q] + 1 < B) {
            const TPair t = load_tpair(T, g[q]);
            t0[q] = t.lo;
            t1[q] = t.hi;
        } else {
            t0[q] = T[g[q]];
            t1[q] = ~0ull;
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        step[q] = 1;
        if (t0[q] <= x[q]) {
            lo[q] = g[q];
            if (g[q] + 1 >= B || t1[q] > x[q]) {
                hi[q] = g[q] + 1;
                dir[q] = 0;
            } else {
                lo[q] = g[q] + 1;
                hi[q] = B;
                dir[q] = 1;
            }
        } else {
            lo[q] = 0;
            hi[q] = g[q];
            dir[q] = -1;
        }
    }
    for (;;) {  // gallop
        bool more = false;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            if (dir[q] > 0) {
                const uint32_t j = lo[q] + step[q];
                if (j >= B) {
                    dir[q] = 0;
                } else if (T[j] > x[q]) {
                    hi[q] = j;
                    dir[q] = 0;
                } else {
                    lo[q] = j;
                    step[q] <<= 1;
                }
            } else if (dir[q] < 0) {
                if (hi[q] <= step[q]) {
                    dir[q] = 0;  // lo stays 0: T[0] = 0 <= x
                } else {
                    const uint32_t j = hi[q] - step[q];
                    if (T[j] <= x[q]) {
                        lo[q] = j;
                        dir[q] = 0;
                    } else {
                        hi[q] = j;
                        step[q] <<= 1;
                    }
                }
            }
            more |= dir[q] != 0;
        }
        if (!more) break;
    }
    for (;;) {  // halve the brackets
        bool more = false;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            if (hi[q] - lo[q] > 1) {
                const uint32_t mid = lo[q] + (hi[q] - lo[q]) / 2;
                if (T[mid] <= x[q]) lo[q] = mid;
                else hi[q] = mid;
                more = true;
            }
        }
        if (!more) break;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] = lo[q];
}

// Exact bucket from a guess g without per-lane loops of varying length (so a
// wave never waits on its slowest lane): the 2W buckets around g are searched
// to a fixed depth when they hold x (checked with one read at each end), else
// all B are (B a power of two, T sorted, T[0] = 0).  Returns the largest b
// with T[b] <= x, as correct_bucket does.
template <uint32_t W>
__device__ __forceinline__ uint32_t correct_bucket_window(const uint64_t *__restrict__ T, uint32_t B, uint64_t x,
                                                          uint32_t g) {
    uint32_t lo = 0, span = B;
    if (B > 2 * W) {
        lo = g > W ? g - W : 0;
        if (lo + 2 * W > B) lo = B - 2 * W;
        if (T[lo] <= x && (lo + 2 * W == B || T[lo + 2 * W] > x)) span = 2 * W;
        else lo = 0;
    }
    uint32_t b = lo;  // T[b] <= x throughout
    for (uint32_t step = span >> 1; step >= 1; step >>= 1)
        if (b + step < B && T[b + step] <= x) b += step;
    return b;
}

template <int AMODE>
__device__ __forceinline__ uint32_t *bucket_counters(const BucketArgs &a, uint32_t *s) {
    return s + (a.S == 1 ? 2 * a.B : AMODE == 0 ? (a.B / a.S) * 2 : 0);
}

template <int AMODE>
__device__ __forceinline__ void bucket_lds_init(const BucketArgs &a, uint32_t *s) {
    if (a.hist) {
        uint32_t *h = bucket_counters<AMODE>(a, s);
        for (uint32_t t = threadIdx.x; t < a.B / 2; t += blockDim.x) h[t] = 0;
    }
    if (a.S == 1 && AMODE == 0) {
        // Splitter: T[1..B) in breadth-first (Eytzinger) order, e[i] for node
        // i of the perfect search tree of depth log2(B) -- node i at level k,
        // position p in its level, holds T[(2p + 1) << (log2(B) - 1 - k)].
        // The search's early levels then read neighbouring words (distinct
        // LDS banks) instead of words a power of two apart (one bank).
        uint64_t *e = reinterpret_cast<uint64_t *>(s);
        const uint32_t d = 31u - uint32_t(__clz(a.B));
        for (uint32_t i = threadIdx.x; i < a.B; i += blockDim.x) {
            if (i == 0) {
                e[0] = 0;
                continue;
            }
            const uint32_t k = 31u - uint32_t(__clz(i)), p = i - (1u << k);
            e[i] = a.T[(2 * p + 1) << (d - 1 - k)];
        }
    } else if (a.S == 1) {  // learned: T in sorted order (searched outward from a guess)
        uint64_t *th = reinterpret_cast<uint64_t *>(s);
        for (uint32_t t = threadIdx.x; t < a.B; t += blockDim.x) th[t] = a.T[t];
    } else if (AMODE == 0) {
        // The splitter's 1-in-S sample ts[j] = T[j S], j < m = B/S, in the
        // same breadth-first order as the full table: node i holds
        // ts[(2p + 1) << (log2(m) - 1 - k)].
        uint64_t *e = reinterpret_cast<uint64_t *>(s);
        const uint32_t m = a.B / a.S, d = 31u - uint32_t(__clz(m));
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            if (i == 0) {
                e[0] = 0;
                continue;
            }
            const uint32_t k = 31u - uint32_t(__clz(i)), p = i - (1u << k);
            e[i] = a.T[uint64_t(a.S) * ((2 * p + 1) << (d - 1 - k))];
        }
    }
}

// Sorted element j (1 <= j < m) of a breadth-first image e of m sorted
// values: j = (2p + 1) << (log2(m) - 1 - k) sits at node 2^k + p, so k and p
// follow from the trailing zeros of j.
__device__ __forceinline__ uint64_t bfs_sorted(const uint64_t *e, uint32_t m, uint32_t j) {
    const uint32_t d = 31u - uint32_t(__clz(m)), tz = uint32_t(__ffs(j)) - 1u;
    return e[(1u << (d - 1u - tz)) + (j >> (tz + 1u))];
}

template <int AMODE>
__device__ __forceinline__ uint32_t bucket_of(const BucketArgs &a, const uint32_t *s, uint64_t x,
                                              uint32_t &probes, uint32_t &guess) {
    if (AMODE == 1) {
        guess = predict_bucket(a.p, x, a.B);
        if (a.S == 1) return correct_bucket(reinterpret_cast<const uint64_t *>(s), a.B, x, guess, probes);
        return correct_bucket(a.T, a.B, x, guess, probes);
    }
    if (a.S == 1) {  // every threshold in LDS, breadth-first: descend log2(B) levels
        const uint64_t *e = reinterpret_cast<const uint64_t *>(s);
        uint32_t i = 1;
        while (i < a.B) i = 2 * i + (e[i] <= x ? 1u : 0u);
        guess = i - a.B;  // the number of T[1..B) at most x
        return guess;
    }
    const uint64_t *e = reinterpret_cast<const uint64_t *>(s);  // the sample, breadth-first
    const uint32_t m = a.B / a.S;
    uint32_t i = 1;
    while (i < m) i = 2 * i + (e[i] <= x ? 1u : 0u);
    const uint32_t lo = i - m;  // ts[lo] <= x < ts[lo + 1]
    uint32_t l2 = lo * a.S, h2 = min(a.B, (lo + 1) * a.S);
    while (h2 - l2 > 1) {
        const uint32_t mid = (l2 + h2) >> 1;
        ++probes;
        if (a.T[mid] <= x) l2 = mid; else h2 = mid;
    }
    guess = l2;
    return l2;
}

// Splitter search of several keys at once (every threshold in LDS in
// breadth-first order, S == 1, B a power of two): log2(B) levels per key, the
// keys' steps interleaved so their LDS reads overlap.  b[q] = the largest b
// with T[b] <= x[q] (T[0] = 0), i.e. the number of T[1..B) at most x[q].
template <int N>
__device__ __forceinline__ void splitter_search_n(const BucketArgs &a, const uint32_t *s,
                                                  const uint64_t *x, uint32_t *b) {
    const uint64_t *e = reinterpret_cast<const uint64_t *>(s);
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] = 1;
    for (uint32_t lv = a.B >> 1; lv >= 1; lv >>= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) b[q] = 2 * b[q] + (e[b[q]] <= x[q] ? 1u : 0u);
    }
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] -= a.B;
}

// The same for a 1-in-S sample of T in LDS (S > 1, breadth-first order): a
// fixed-depth descent of the sample finds the run of S thresholds of T that
// holds the answer; a linear interpolation between the two samples around
// the key guesses the bucket, one 16-byte read of T (global memory) tests
// the guess and its right neighbour, and a binary search finishes
// whatever is left of the run.  Exact whatever the data; for smooth data the
// guess is right or one off, so most keys read T in one round instead of
// log2(S) dependent ones.
template <int N>
__device__ __forceinline__ void splitter_search_sampled_n(const BucketArgs &a, const uint32_t *s,
                                                          const uint64_t *x, uint32_t *b) {
    const uint64_t *e = reinterpret_cast<const uint64_t *>(s);  // the sample, breadth-first
    const uint32_t m = a.B / a.S;  // sample size; ts[0] = T[0] = 0
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] = 1;
    for (uint32_t step = m >> 1; step >= 1; step >>= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) b[q] = 2 * b[q] + (e[b[q]] <= x[q] ? 1u : 0u);
    }
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] -= m;  // ts[b] <= x < ts[b + 1]
    // The answer lies in [lo, hi): T[lo] = ts[i] <= x, and T[hi] > x (hi =
    // (i + 1) S is the next sample, or hi = B).
    uint32_t lo[N], hi[N], g[N];
    uint64_t tg[N], tn[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const uint32_t i = b[q];
        const uint64_t t0 = i ? bfs_sorted(e, m, i) : 0ull, t1 = i + 1 < m ? bfs_sorted(e, m, i + 1) : ~0ull;
        lo[q] = i * a.S;
        hi[q] = lo[q] + a.S;
        const uint64_t span = t1 - t0;  // > 0 unless the run ends at the top of the range
        const uint32_t k = span ? uint32_t(float(x[q] - t0) / float(span) * float(a.S)) : 0u;
        g[q] = lo[q] + min(k, a.S - 1u);
        if (g[q] + 1 < a.B) {  // the neighbour only counts inside the run
            const TPair t = load_tpair(a.T, g[q]);
            tg[q] = t.lo;
            tn[q] = g[q] + 1 < hi[q] ? t.hi : ~0ull;
        } else {
            tg[q] = a.T[g[q]];
            tn[q] = ~0ull;
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        if (tg[q] <= x[q]) {
            lo[q] = g[q];
            if (g[q] + 1 < hi[q]) {
                if (tn[q] <= x[q]) lo[q] = g[q] + 1;
                else hi[q] = g[q] + 1;
            }
        } else {
            hi[q] = g[q];  // g > lo here, as T[lo] <= x
        }
    }
    for (;;) {
        bool more = false;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            if (hi[q] - lo[q] > 1) {
                const uint32_t mid = (lo[q] + hi[q]) >> 1;
                if (a.T[mid] <= x[q]) lo[q] = mid;
                else hi[q] = mid;
                more = true;
            }
        }
        if (!more) break;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] = lo[q];
}

template <int AMODE>
__device__ __forceinline__ void bucket_record(const BucketArgs &a, uint32_t *s, uint32_t b, uint64_t i) {
    if (a.bid) a.bid[i] = uint16_t(b);
    if (a.bid32) a.bid32[i] = b;
    if (a.hist) atomicAdd(&bucket_counters<AMODE>(a, s)[b >> 1], 1u << (16 * (b & 1)));
}

template <int AMODE>
__device__ __forceinline__ uint32_t bucket_assign_one(const BucketArgs &a, uint32_t *s, uint64_t x,
                                                      uint64_t i, uint32_t &probes, uint32_t &err) {
    uint32_t guess;
    const uint32_t b = bucket_of<AMODE>(a, s, x, probes, guess);
    err += b > guess ? b - guess : guess - b;
    if (a.bid) a.bid[i] = uint16_t(b);
    if (a.bid32) a.bid32[i] = b;
    if (AMODE == 1 && a.pred) a.pred[i] = guess;
    if (a.hist) atomicAdd(&bucket_counters<AMODE>(a, s)[b >> 1], 1u << (16 * (b & 1)));
    return b;
}

template <int AMODE>
__device__ __forceinline__ void bucket_assign_one(const BucketArgs &a, uint32_t *s, uint64_t x, uint64_t i) {
    uint32_t probes = 0, err = 0;
    (void)bucket_assign_one<AMODE>(a, s, x, i, probes, err);
}

// Before a workgroup records `next` more keys (0: it records no more): adds
// to the global histogram and clears each pair of packed counters in which a
// count could otherwise pass 65535, or every pair when next == 0.  Each thread
// decides for the words it owns; call between barriers.
template <int AMODE>
__device__ __forceinline__ void bucket_lds_flush_before(const BucketArgs &a, uint32_t *s, uint32_t next) {
    if (!a.hist) return;
    uint32_t *h = bucket_counters<AMODE>(a, s);
    const uint32_t lim = 65535u - next;  // next <= 65535
    for (uint32_t t = threadIdx.x; t < a.B / 2; t += blockDim.x) {
        const uint32_t v = h[t];
        if (next != 0u && (v & 0xFFFFu) <= lim && (v >> 16) <= lim) continue;
        h[t] = 0u;
        // Buckets 2t and 2t+1 in one 64-bit add (hist is 8-byte aligned): the
        // low count cannot carry into the high one, as every count is < 2^32.
        if (v)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.hist + 2 * t),
                      (static_cast<unsigned long long>(v >> 16) << 32) | (v & 0xFFFFu));
    }
}

// Compression fused with bucket assignment (k_compress.hip; amode 1 learned,
// 0 splitter).  Fixed-width keys whose compression fits one launch only (else
// CKEY_ERR_UNSUPPORTED).
ckey_status compress_bucket_launch(const KeySrc &k, const uint8_t *bitmap_host, uint64_t *ckeys,
                                   uint32_t words, uint32_t *rowids, uint32_t *flags, int amode,
                                   const BucketArgs &ba, hipStream_t st);

}  // namespace ckey
