// Learned bucketing sort of compressed keys (an extension of the paper's
// compressed key sort; the paper itself sorts by comparison, Appendix A).
//
// Model (device memory owned by the caller, layout below): a threshold table
// T[0..B) of 64-bit key prefixes (T[0] = 0; T[b] = the prefix of rank b*m/B
// in a sorted training set) and a 4 -> 64 -> 1 ReLU MLP predicting the
// normalised rank of a prefix from its four 16-bit chunks.
//
// bucket(x) = the b with T[b] <= prefix(x) < T[b+1].  It is non-decreasing in
// key order, so concatenating the buckets, each sorted, sorts everything.
// The MLP only predicts where to start looking: an exponential-then-binary
// search from the prediction always lands on the exact bucket, so exactness
// never depends on the network (the splitter method instead searches a
// 1-in-S sample of T held in LDS, then T itself).
//
// Sort: assign buckets (+ histogram) -> scan -> group rows by bucket (a
// stable sort on the bucket id: two one-sweep passes) -> one workgroup per
// bucket sorts it in place in LDS by the bits of the first word below the
// bucket's common prefix (stable 8-bit LSD passes with wave ballots, skipping
// digits constant in the bucket), then orders runs of equal first words by the
// remaining words and the row id.  Buckets larger than the LDS capacity, or
// with a run of equal first words longer than kRunCap, are left in place and
// finished by the radix sort (row-id digits first, so ties still end in row-id
// order).
#include <math.h>

#include <vector>

#include "bucket.h"
#include "internal.h"

namespace ckey {

namespace {

constexpr int kNP = 6 * kH + 1;  // parameters
constexpr int kNPad = 392;       // parameters + loss slot, padded
constexpr int kLoss = kNP;       // index of the loss in a partial-sum row
constexpr size_t kOffParams = 0, kOffM = 2048, kOffV = 4096, kOffT = 8192;
constexpr int kCapLarge = 5120;  // max bucket size sorted in LDS (large-bucket kernel)
constexpr int kCapSmall = 2560;  // (small-bucket kernel, for <= 1600 rows per bucket on average)
constexpr int kRunCap = 32;      // max run of equal first words sorted in place
constexpr int kAssignWG = 1024;
constexpr uint32_t kKeysPerAssignWG = 65535;  // keeps the packed 16-bit LDS counters exact

inline float *params_of(void *model) { return reinterpret_cast<float *>(static_cast<uint8_t *>(model) + kOffParams); }
inline const float *params_of(const void *model) {
    return reinterpret_cast<const float *>(static_cast<const uint8_t *>(model) + kOffParams);
}
inline const uint64_t *thresholds_of(const void *model) {
    return reinterpret_cast<const uint64_t *>(static_cast<const uint8_t *>(model) + kOffT);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea, Flood 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------ model --

__global__ void k_model_init(float *p, float *m, float *v, uint64_t seed) {
    const int t = threadIdx.x;
    if (t >= kNPad) return;
    const float noise = float(int64_t(mix64(seed + 0x9E3779B97F4A7C15ull * (t + 1)) >> 40) - (1 << 23)) *
                        (1.0f / float(1 << 23)) * 1e-3f;
    float val = 0.0f;
    if (t < 4 * kH) {
        val = (t % 4 == 0) ? 1.0f + noise : noise;   // W1: unit k watches the top chunk
    } else if (t < 5 * kH) {
        val = -float(t - 4 * kH) / float(kH);        // b1: kinks spread over [0, 1)
    } else if (t < 6 * kH) {
        val = (t == 5 * kH ? 1.0f : 0.0f) + noise;   // w2: start from the uniform CDF
    }
    p[t] = t < kNP ? val : 0.0f;
    m[t] = 0.0f;
    v[t] = 0.0f;
}

__global__ void k_thresholds(const uint64_t *__restrict__ sorted, uint64_t m, uint64_t *__restrict__ T,
                             uint32_t B) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    T[b] = b == 0 ? 0ull : sorted[(uint64_t(b) * m) / B];
}

// Forward + backward on M samples; per-block partial sums (fixed order).
// target == nullptr: sample i = hash(seed, step, j) mod m, target (i+0.5)/m.
__global__ __launch_bounds__(kWG) void k_mlp_grad(const float *__restrict__ p,
                                                  const uint64_t *__restrict__ prefix,
                                                  const float *__restrict__ target, uint64_t m,
                                                  uint32_t M, uint64_t seed, uint32_t step,
                                                  float *__restrict__ partial) {
    __shared__ float s_acc[kWG / 64][kNPad];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int t = tid; t < (kWG / 64) * kNPad; t += kWG) (&s_acc[0][0])[t] = 0.0f;
    __syncthreads();
    const float invM = 1.0f / float(M);
    for (uint64_t base = uint64_t(blockIdx.x) * kWG + wave * 64; base < M;
         base += uint64_t(gridDim.x) * kWG) {
        const uint64_t j = base + lane;
        const bool valid = j < M;
        uint64_t i = j;
        if (!target)
            i = mix64(seed + 0x9E3779B97F4A7C15ull * ((uint64_t(step) << 32) + j + 1)) % m;
        const uint64_t x = valid ? prefix[i] : 0ull;
        const float t = valid ? (target ? target[i] : (float(i) + 0.5f) / float(m)) : 0.0f;
        float f[4];
        mlp_features(x, f);
        float h[kH];
        float y = p[6 * kH];
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            float a = p[4 * kH + k];
            a = fmaf(p[4 * k + 0], f[0], a);
            a = fmaf(p[4 * k + 1], f[1], a);
            a = fmaf(p[4 * k + 2], f[2], a);
            a = fmaf(p[4 * k + 3], f[3], a);
            h[k] = fmaxf(a, 0.0f);
            y = fmaf(p[5 * kH + k], h[k], y);
        }
        const float e = valid ? y - t : 0.0f;
        const float dy = 2.0f * e * invM;
        const float db2 = wave_sum(dy);
        const float ls = wave_sum(e * e * invM);
        if (lane == 0) {
            s_acc[wave][6 * kH] += db2;
            s_acc[wave][kLoss] += ls;
        }
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            const float g = h[k] > 0.0f ? dy * p[5 * kH + k] : 0.0f;
            const float c_w2 = wave_sum(dy * h[k]);
            const float c_b1 = wave_sum(g);
            const float c0 = wave_sum(g * f[0]);
            const float c1 = wave_sum(g * f[1]);
            const float c2 = wave_sum(g * f[2]);
            const float c3 = wave_sum(g * f[3]);
            if (lane == 0) {
                s_acc[wave][5 * kH + k] += c_w2;
                s_acc[wave][4 * kH + k] += c_b1;
                s_acc[wave][4 * k + 0] += c0;
                s_acc[wave][4 * k + 1] += c1;
                s_acc[wave][4 * k + 2] += c2;
                s_acc[wave][4 * k + 3] += c3;
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < kNPad; t += kWG) {
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kWG / 64; ++w) s += s_acc[w][t];
        partial[uint64_t(blockIdx.x) * kNPad + t] = s;
    }
}

// Sum G partial rows in order; then either write grad/loss or take an Adam step.
__global__ __launch_bounds__(512) void k_mlp_reduce(const float *__restrict__ partial, uint32_t G,
                                                    float *__restrict__ grad_out,
                                                    float *__restrict__ loss_out, float *p, float *m,
                                                    float *v, float lr, float b1, float b2, float eps,
                                                    uint32_t t) {
    const int i = threadIdx.x;
    if (i > kLoss) return;
    float s = 0.0f;
    for (uint32_t g = 0; g < G; ++g) s += partial[uint64_t(g) * kNPad + i];
    if (i == kLoss) {
        if (loss_out) *loss_out = s;
        return;
    }
    if (grad_out) grad_out[i] = s;
    if (p) {  // Adam (Kingma & Ba), bias-corrected
        const float mi = b1 * m[i] + (1.0f - b1) * s;
        const float vi = b2 * v[i] + (1.0f - b2) * s * s;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / (1.0f - powf(b1, float(t)));
        const float vh = vi / (1.0f - powf(b2, float(t)));
        p[i] -= lr * mh / (sqrtf(vh) + eps);
    }
}

// ------------------------------------------------------- bucket assignment --

// Stand-alone assignment of first words w0[0..n) (MODE 0: splitter, 1: learned).
template <int MODE>
__global__ __launch_bounds__(kBucketWG) void k_bucket_assign(const uint64_t *__restrict__ w0,
                                                             uint64_t n, BucketArgs ba,
                                                             unsigned long long *__restrict__ stats) {
    extern __shared__ uint32_t s_dyn[];
    bucket_lds_init<MODE>(ba, s_dyn);
    __syncthreads();
    const uint64_t i0 = uint64_t(blockIdx.x) * kBucketKeysPerWG;
    const uint64_t i1 = min<uint64_t>(n, i0 + kBucketKeysPerWG);
    uint32_t probes = 0, err = 0;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBucketWG)
        (void)bucket_assign_one<MODE>(ba, s_dyn, w0[i], i, probes, err);
    __syncthreads();
    bucket_lds_flush<MODE>(ba, s_dyn);
    if (stats) {
        unsigned long long a = probes, e = err;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            e += __shfl_xor(e, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&stats[0], a);
            atomicAdd(&stats[1], e);
        }
    }
}

// Exclusive scan of B counters by one 1024-thread workgroup -> starts[0..B], cursors.
__global__ __launch_bounds__(1024) void k_bucket_scan(const uint32_t *__restrict__ hist, uint32_t B,
                                                      uint32_t *__restrict__ starts,
                                                      uint32_t *__restrict__ cursor) {
    __shared__ uint32_t s_w[16];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t per = (B + 1023) / 1024;
    const uint32_t b0 = tid * per;
    uint32_t sum = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (b0 + q < B) sum += hist[b0 + q];
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        off += w < wave ? s_w[w] : 0u;
        tot += s_w[w];
    }
    uint32_t run = off + incl - sum;
    for (uint32_t q = 0; q < per; ++q)
        if (b0 + q < B) {
            starts[b0 + q] = run;
            cursor[b0 + q] = run;
            run += hist[b0 + q];
        }
    if (tid == 0) starts[B] = tot;
}


// Runs over positions [0, cnt) held thread-contiguously: thread t owns
// positions [P*t, P*t + P), and bit u of `starts` says that owned position u
// begins a run (position 0 always does).  Block-wide prefix max of run starts
// and suffix min of the next run starts (wave shuffles, one LDS exchange) give
// the thread the start of the run that its first position belongs to (*cs)
// and the first run start after its positions (*ce, cnt if none).  Every
// thread of the workgroup calls it; s_x holds 2 * NT/64 ints.
template <int P, int NT>
__device__ __forceinline__ void run_carries(uint32_t cnt, uint32_t starts, uint32_t *cs, uint32_t *ce,
                                            int32_t *s_x) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int32_t j0 = P * tid, kNone = 0x7FFFFFFF;
    int32_t pm = starts ? j0 + 31 - int32_t(__clz(starts)) : -1;  // last start here
    int32_t sm = starts ? j0 + int32_t(__ffs(starts)) - 1 : kNone;  // first start here
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t a = __shfl_up(pm, off, 64), b = __shfl_down(sm, off, 64);
        if (lane >= off) pm = max(pm, a);
        if (lane + off < 64) sm = min(sm, b);
    }
    int32_t pex = __shfl_up(pm, 1, 64), sex = __shfl_down(sm, 1, 64);
    if (lane == 0) pex = -1;
    if (lane == 63) sex = kNone;
    if (lane == 63) s_x[wave] = pm;
    if (lane == 0) s_x[NW + wave] = sm;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave) pex = max(pex, s_x[w]);
        if (w > wave) sex = min(sex, s_x[NW + w]);
    }
    __syncthreads();  // s_x may be reused
    *cs = uint32_t(pex < 0 ? 0 : pex);
    *ce = sex == kNone ? cnt : uint32_t(sex);
}

// One workgroup per bucket, in place on rows [starts[b], starts[b+1]) of ck/rid
// (the rows are already grouped by bucket).  Every first word x in bucket b
// lies in [T[b], T[b+1]), so all share the common prefix (cp bits) of that
// range; the LDS sort key is x << cp, whose equal values are equal first words.
//
// 1. Order by the local key: LSD over its top three varying 8-bit digits (the
//    first pass unstable, by LDS atomics -- the starting order is arbitrary;
//    later passes stable, ranked with wave ballots), then every run of equal
//    top digits is ranked in parallel by the whole local key.  A run longer
//    than kTieCap instead redoes the LSD over every varying digit.
// 2. Runs of equal local keys (equal first words) are ordered by the remaining
//    words and the row id: each array is staged in LDS and the members of
//    every run are ranked by it in parallel, stably (an LSD within the runs,
//    row ids first, then words w-1 .. 1).
// 3. The first words are written from LDS; the other arrays are staged in LDS
//    (coalesced load) and written back in sorted order (coalesced store).
template <int WC, int kCap, int kSortWG>
__global__ __launch_bounds__(kSortWG, 8) void k_bucket_sort(uint64_t *__restrict__ ck,
                                                         uint32_t *__restrict__ rid, uint64_t n,
                                                         uint32_t words_rt,
                                                         const uint32_t *__restrict__ starts,
                                                         const uint64_t *__restrict__ T, uint32_t B,
                                                         uint32_t *__restrict__ ovf) {
    constexpr int NW = kSortWG / 64;
    constexpr int PER = (kCap + kSortWG - 1) / kSortWG;
    constexpr uint32_t kTieCap = 64;
    static_assert(kCap <= 8192 && ((kCap + kSortWG - 1) / kSortWG) * 64 <= 512,
                  "packed ids and ranks need 13 and 9 bits");
    __shared__ uint32_t s_k[2][kCap];    // [0]: high, [1]: low half of the local key;
                                         // afterwards 8-byte staging of the other arrays
    __shared__ uint16_t s_idx[2][kCap];  // element order, ping-pong
    __shared__ uint16_t s_run[kCap];     // start of the run of equal local keys at each position
    __shared__ uint16_t s_wc[NW][256];   // per-wave digit counts, then offsets (< kCap)
    __shared__ uint32_t s_red[NW][4];
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint32_t s_flag[2];       // [0]: some run needs ordering / redo, [1]: run too long
    __shared__ int32_t s_rb[2 * NW];     // run_bounds exchange
    const uint32_t words = WC > 0 ? uint32_t(WC) : words_rt;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t b = blockIdx.x;
    const uint32_t start = starts[b];
    const uint32_t cnt = starts[b + 1] - start;
    if (cnt < 2) return;
    if (cnt > uint32_t(kCap)) {
        if (tid == 0) {
            const uint32_t slot = atomicAdd(&ovf[0], 1u);
            ovf[1 + 2 * slot] = start;
            ovf[2 + 2 * slot] = cnt;
        }
        return;
    }
    const uint64_t lo = T[b], hi = (b + 1 < B) ? T[b + 1] - 1 : ~0ull;
    const uint32_t cp = lo == hi ? 64u : uint32_t(__clzll(lo ^ hi));
    const uint64_t pre = cp == 0 ? 0ull : cp >= 64 ? lo : (lo & ~(~0ull >> cp));  // shared prefix
    uint32_t a_and[2] = {~0u, ~0u}, a_or[2] = {0u, 0u};
    {
        uint64_t xs[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {  // all loads first: PER in flight per thread
            const uint32_t j = tid + u * kSortWG;
            xs[u] = j < cnt ? ck[start + j] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            if (j < cnt) {
                const uint64_t l64 = cp < 64 ? xs[u] << cp : 0ull;
                const uint32_t h32 = uint32_t(l64 >> 32), l32 = uint32_t(l64);
                s_k[0][j] = h32;
                s_k[1][j] = l32;
                s_idx[0][j] = uint16_t(j);
                a_and[0] &= h32;
                a_or[0] |= h32;
                a_and[1] &= l32;
                a_or[1] |= l32;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a_and[0] &= __shfl_xor(a_and[0], off, 64);
        a_and[1] &= __shfl_xor(a_and[1], off, 64);
        a_or[0] |= __shfl_xor(a_or[0], off, 64);
        a_or[1] |= __shfl_xor(a_or[1], off, 64);
    }
    if (lane == 0) {
        s_red[wave][0] = a_and[0];
        s_red[wave][1] = a_and[1];
        s_red[wave][2] = a_or[0];
        s_red[wave][3] = a_or[1];
    }
    if (tid < 2) s_flag[tid] = 0u;
    __syncthreads();
    uint32_t vary[2] = {0u, 0u};
    {
        uint32_t g_and[2] = {~0u, ~0u}, g_or[2] = {0u, 0u};
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            g_and[0] &= s_red[w][0];
            g_and[1] &= s_red[w][1];
            g_or[0] |= s_red[w][2];
            g_or[1] |= s_red[w][3];
        }
        vary[0] = g_and[0] ^ g_or[0];
        vary[1] = g_and[1] ^ g_or[1];
    }
    auto lkey = [&](uint32_t id) { return (uint64_t(s_k[0][id]) << 32) | s_k[1][id]; };
    // Digits of the 64-bit local key, 0 = least significant; d < 4 is in the low half.
    auto digit_varies = [&](int d) { return ((vary[d < 4 ? 1 : 0] >> (8 * (d & 3))) & 0xFFu) != 0; };
    int dmin = 8, nvar = 0, nall = 0;
    for (int d = 7; d >= 0; --d)
        if (digit_varies(d)) {
            ++nall;
            if (nvar < 3) { dmin = d; ++nvar; }
        }
    int cur = 0;
    // Each wave ranks a contiguous slice of Q elements (Q a multiple of 64) in
    // order, at most kRounds rounds of 64.
    constexpr int kRounds = (kCap + kSortWG - 1) / kSortWG;
    const uint32_t Q = ((cnt + NW * 64 - 1) / (NW * 64)) * 64;
    const uint32_t e0 = wave * Q, e1 = min(cnt, e0 + Q);
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    uint32_t *cnt32 = reinterpret_cast<uint32_t *>(&s_wc[0][0]);  // 256 counters (unstable pass)
    for (int attempt = 0; attempt < 2; ++attempt) {
        const int dlo = attempt == 0 ? dmin : 0;
        bool first = true;
        for (int d = dlo; d < 8; ++d) {  // LSD over the chosen digits
            if (!digit_varies(d)) continue;
            const uint32_t *key = s_k[d < 4 ? 1 : 0];
            const uint32_t shift = 8 * (d & 3);
            if (first) {
                // Unstable counting pass straight from the load order.
                first = false;
                if (tid < 256) cnt32[tid] = 0u;
                __syncthreads();
                for (uint32_t j = tid; j < cnt; j += kSortWG) atomicAdd(&cnt32[(key[j] >> shift) & 0xFFu], 1u);
                __syncthreads();
                const uint32_t c = tid < 256 ? cnt32[tid] : 0u;
                uint32_t all;
                const uint32_t ex = block_excl_scan_n<kSortWG>(c, s_tmp, all);
                if (tid < 256) cnt32[tid] = ex;
                __syncthreads();
                for (uint32_t j = tid; j < cnt; j += kSortWG) {
                    const uint32_t pos = atomicAdd(&cnt32[(key[j] >> shift) & 0xFFu], 1u);
                    s_idx[1][pos] = uint16_t(j);
                }
                __syncthreads();
                cur = 1;
                continue;
            }
            for (int t = tid; t < NW * 256; t += kSortWG) (&s_wc[0][0])[t] = 0;
            __syncthreads();
            // per element: id (13 bits) << 17 | digit << 9 | rank within the wave's slice (< 512)
            uint32_t pk[kRounds];
#pragma unroll
            for (int u = 0; u < kRounds; ++u) {
                const uint32_t e = e0 + 64 * u + lane;
                const bool valid = e < e1;
                const uint32_t id = valid ? s_idx[cur][e] : 0u;
                const uint32_t dig = valid ? (key[id] >> shift) & 0xFFu : 0u;
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int bit = 0; bit < 8; ++bit) {
                    const bool on = (dig >> bit) & 1u;
                    const uint64_t bal = __ballot(on);
                    peers &= on ? bal : ~bal;
                }
                const uint32_t below = __popcll(peers & lane_lt);
                uint32_t old = 0;
                if (valid) old = s_wc[wave][dig];
                if (valid && below == 0) s_wc[wave][dig] = uint16_t(old + uint32_t(__popcll(peers)));
                pk[u] = (id << 17) | (dig << 9) | (old + below);
            }
            __syncthreads();
            {
                uint32_t tot = 0;
                if (tid < 256)
#pragma unroll
                    for (int w = 0; w < NW; ++w) tot += s_wc[w][tid];
                uint32_t all;
                uint32_t ds = block_excl_scan_n<kSortWG>(tot, s_tmp, all);
                if (tid < 256) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const uint32_t c = s_wc[w][tid];
                        s_wc[w][tid] = uint16_t(ds);
                        ds += c;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kRounds; ++u) {
                const uint32_t e = e0 + 64 * u + lane;
                if (e < e1) s_idx[cur ^ 1][s_wc[wave][(pk[u] >> 9) & 0xFFu] + (pk[u] & 0x1FFu)] = uint16_t(pk[u] >> 17);
            }
            __syncthreads();
            cur ^= 1;
        }
        if (attempt == 1 || nall <= 3) break;  // every varying digit is sorted
        // Runs of equal top digits: rank each member by the whole local key.
        // Each thread takes PER consecutive positions; run bounds come from
        // block scans, so a long run costs its members one pass over it.
        const uint32_t sh = 8 * uint32_t(dmin);  // bits below the sorted digits
        const uint16_t *ordr = s_idx[cur];
        uint16_t *dst = s_idx[cur ^ 1];
        {
            const uint32_t j0 = PER * uint32_t(tid);
            uint32_t starts = 0;
            uint64_t prevt = (j0 > 0 && j0 - 1 < cnt) ? lkey(ordr[j0 - 1]) >> sh : 0ull;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = j0 + u;
                if (j < cnt) {
                    const uint64_t t = lkey(ordr[j]) >> sh;
                    if (j == 0 || t != prevt) starts |= 1u << u;
                    prevt = t;
                }
            }
            uint32_t cs, ce;
            run_carries<PER, kSortWG>(cnt, starts, &cs, &ce, s_rb);
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = j0 + u;
                if (j >= cnt) break;
                if ((starts >> u) & 1u) cs = j;
                const uint32_t later = starts >> (u + 1);
                const uint32_t re = later ? j + uint32_t(__ffs(later)) : ce;
                const uint32_t len = re - cs;
                const uint16_t id = ordr[j];
                if (len > kTieCap) {  // redo with every digit (dst is discarded)
                    s_flag[0] = 1u;
                    continue;
                }
                if (len == 1) {
                    dst[j] = id;
                    continue;
                }
                const uint64_t kv = lkey(id);
                uint32_t r = 0;
                for (uint32_t q = cs; q < re; ++q) {
                    const uint64_t kq = lkey(ordr[q]);
                    r += (kq < kv || (kq == kv && q < j)) ? 1u : 0u;
                }
                dst[cs + r] = id;  // cs + r < re <= cnt
            }
        }
        __syncthreads();
        if (!s_flag[0]) {
            cur ^= 1;
            break;
        }
        __syncthreads();  // every thread has read the flag
        if (tid == 0) s_flag[0] = 0u;
    }
    // Runs of equal local keys (equal first words): record each position's run
    // start; a run longer than kRunCap sends the bucket to the radix fallback.
    const uint16_t *ord0 = s_idx[cur];
    {
        const uint32_t j0 = PER * uint32_t(tid);
        uint32_t starts = 0;
        uint64_t prevk = (j0 > 0 && j0 - 1 < cnt) ? lkey(ord0[j0 - 1]) : 0ull;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = j0 + u;
            if (j < cnt) {
                const uint64_t k = lkey(ord0[j]);
                if (j == 0 || k != prevk) starts |= 1u << u;
                prevk = k;
            }
        }
        uint32_t cs, ce;
        run_carries<PER, kSortWG>(cnt, starts, &cs, &ce, s_rb);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = j0 + u;
            if (j >= cnt) break;
            if ((starts >> u) & 1u) cs = j;
            const uint32_t later = starts >> (u + 1);
            const uint32_t len = (later ? j + uint32_t(__ffs(later)) : ce) - cs;
            if (len > uint32_t(kRunCap)) s_flag[1] = 1u;
            if (len > 1) s_flag[0] = 1u;
            s_run[j] = uint16_t(cs);
        }
    }
    __syncthreads();
    if (s_flag[1]) {  // leave the bucket as it is for the radix fallback
        if (tid == 0) {
            const uint32_t slot = atomicAdd(&ovf[0], 1u);
            ovf[1 + 2 * slot] = start;
            ovf[2 + 2 * slot] = cnt;
        }
        return;
    }
    // First words, from the local keys (equal within a run, so already final).
    for (uint32_t j = tid; j < cnt; j += kSortWG) {
        const uint64_t l = lkey(ord0[j]);
        ck[start + j] = cp >= 64 ? lo : (pre | (l >> cp));
    }
    const bool fixup = s_flag[0] != 0u;
    __syncthreads();  // local keys are dead from here on
    uint64_t *stg = reinterpret_cast<uint64_t *>(&s_k[0][0]);  // 8*kCap bytes
    int done_arr = 0;  // arrays already written: 0 (first words), then -1 (row ids) or a word
    if (fixup) {
        for (int k = -1; k < int(words); ++k) {
            if (k == 0) continue;  // first words are equal within a run
            const int a = k < 0 ? -1 : int(words) - k;  // -1: row ids, then words w-1 .. 1
            uint64_t v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                v[u] = j >= cnt ? 0ull : a < 0 ? uint64_t(rid[start + j]) : ck[uint64_t(a) * n + start + j];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                if (j < cnt) stg[j] = v[u];
            }
            __syncthreads();
            const uint16_t *ord = s_idx[cur];
            uint16_t *dst = s_idx[cur ^ 1];
            for (uint32_t j = tid; j < cnt; j += kSortWG) {
                const uint16_t id = ord[j];
                const uint32_t s = s_run[j];
                const bool alone = s == j && (j + 1 == cnt || s_run[j + 1] != j);
                if (alone) {
                    dst[j] = id;
                    continue;
                }
                const uint64_t x = stg[id];
                uint32_t r = 0;
                for (uint32_t q = s; q < cnt && s_run[q] == s; ++q) {
                    const uint64_t xq = stg[ord[q]];
                    r += (xq < x || (xq == x && q < j)) ? 1u : 0u;  // stable
                }
                dst[s + r] = id;
            }
            __syncthreads();
            cur ^= 1;
            if (k == (words == 1 ? -1 : int(words) - 1)) {  // order final: write this array out
                const uint16_t *fin = s_idx[cur];
                if (a < 0) {
                    for (uint32_t j = tid; j < cnt; j += kSortWG) rid[start + j] = uint32_t(stg[fin[j]]);
                } else {
                    uint64_t *wk = ck + uint64_t(a) * n + start;
                    for (uint32_t j = tid; j < cnt; j += kSortWG) wk[j] = stg[fin[j]];
                }
                done_arr = a;
                __syncthreads();
            }
        }
    }
    // Permute the remaining arrays in place: stage each bucket slice in LDS
    // (coalesced load, all of a thread's loads in flight at once), then write
    // it back in sorted order (coalesced store).
    const uint16_t *ord = s_idx[cur];
    for (uint32_t k = 1; k < words; ++k) {
        if (int(k) == done_arr) continue;
        uint64_t *wk = ck + uint64_t(k) * n + start;
        uint64_t v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            v[u] = j < cnt ? wk[j] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            if (j < cnt) stg[j] = v[u];
        }
        __syncthreads();
        for (uint32_t j = tid; j < cnt; j += kSortWG) wk[j] = stg[ord[j]];
        __syncthreads();
    }
    if (done_arr == -1) return;
    uint32_t *stage32 = &s_k[0][0];
    uint32_t *rk = rid + start;
    {
        uint32_t v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            v[u] = j < cnt ? rk[j] : 0u;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            if (j < cnt) stage32[j] = v[u];
        }
    }
    __syncthreads();
    for (uint32_t j = tid; j < cnt; j += kSortWG) rk[j] = stage32[ord[j]];
}

struct LLayout {
    size_t bid, hist, starts, cursor, ovf, stats, sortws, total;
};

LLayout llayout(uint32_t words, uint64_t n, uint32_t B) {
    LLayout l{};
    size_t off = 0;
    l.bid = off;      off += align256(size_t(n) * 2);
    l.hist = off;     off += align256(size_t(B) * 4);
    l.starts = off;   off += align256(size_t(B + 1) * 4);
    l.cursor = off;   off += align256(size_t(B) * 4);
    l.ovf = off;      off += align256(size_t(2 * B + 1) * 4);
    l.stats = off;    off += align256(2 * 8);
    l.sortws = off;   off += aux_sort_workspace(words, n);
    l.total = off;
    return l;
}

BucketArgs bucket_args(const void *model, uint32_t B, uint16_t *bid, uint32_t *bid32, uint32_t *pred,
                       uint32_t *hist) {
    return BucketArgs{params_of(model), thresholds_of(model), B, splitter_stride(B), bid, bid32, pred, hist};
}

ckey_status assign_launch(int mode, const uint64_t *w0, uint64_t n, const BucketArgs &ba,
                          unsigned long long *stats, hipStream_t st) {
    if (n == 0) return CKEY_OK;
    const size_t lds = bucket_lds_bytes(ba, mode);
    const uint64_t blocks = (n + kBucketKeysPerWG - 1) / kBucketKeysPerWG;
    set_bucket_lds_limit(reinterpret_cast<const void *>(k_bucket_assign<0>));
    set_bucket_lds_limit(reinterpret_cast<const void *>(k_bucket_assign<1>));
    const int pr = prof_begin(st, mode ? "assign_learned" : "assign_splitter");
    if (mode)
        hipLaunchKernelGGL(k_bucket_assign<1>, dim3(uint32_t(blocks)), dim3(kBucketWG), lds, st, w0, n, ba, stats);
    else
        hipLaunchKernelGGL(k_bucket_assign<0>, dim3(uint32_t(blocks)), dim3(kBucketWG), lds, st, w0, n, ba, stats);
    prof_end(st, pr);
    return launch_status();
}

}  // namespace

bool learned_b_ok(uint32_t b_log2) { return b_log2 >= 8 && b_log2 <= 16; }

size_t learned_workspace(uint32_t words, uint32_t nbits, uint64_t n, uint32_t b_log2) {
    const size_t a = llayout(words, n, 1u << b_log2).total;
    const size_t r = radix_workspace(words, nbits, n, 8, 32);
    return a > r ? a : r;
}

namespace {

struct LPtrs {
    uint16_t *bid;
    uint32_t *hist, *starts, *cursor, *ovf;
};

LPtrs lptrs(void *ws, uint32_t words, uint64_t n, uint32_t B, LLayout &l) {
    l = llayout(words, n, B);
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    return LPtrs{reinterpret_cast<uint16_t *>(w8 + l.bid), reinterpret_cast<uint32_t *>(w8 + l.hist),
                 reinterpret_cast<uint32_t *>(w8 + l.starts), reinterpret_cast<uint32_t *>(w8 + l.cursor),
                 reinterpret_cast<uint32_t *>(w8 + l.ovf)};
}

// From bucket ids and the bucket histogram: group by bucket, sort each bucket,
// finish overflowing buckets with the radix sort.
ckey_status bucket_finish(uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid, uint64_t n,
                          const void *model, uint32_t b_log2, const LPtrs &q, const LLayout &l,
                          uint32_t *flags, void *ws, hipStream_t st) {
    const uint32_t B = 1u << b_log2;
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, st, q.hist, B, q.starts, q.cursor);
    CKEY_TRY(launch_status());
    // Group rows by bucket: a stable sort by the bucket id (two one-sweep passes).
    CKEY_TRY(aux_sort(ck, rid, q.bid, n, words, b_log2, q.hist, flags, w8 + l.sortws, st));
    const uint64_t *T = thresholds_of(model);
    {
        const int pr = prof_begin(st, "bucket_sort");
        if (n / B <= 1600) {  // small buckets: 2560-row capacity, 512 threads, 4 per CU
            auto kb = words == 1 ? k_bucket_sort<1, kCapSmall, 512> : words == 2 ? k_bucket_sort<2, kCapSmall, 512>
                    : words == 3 ? k_bucket_sort<3, kCapSmall, 512> : k_bucket_sort<0, kCapSmall, 512>;
            hipLaunchKernelGGL(kb, dim3(B), dim3(512), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf);
        } else {
            auto kb = words == 1 ? k_bucket_sort<1, kCapLarge, 1024> : words == 2 ? k_bucket_sort<2, kCapLarge, 1024>
                    : words == 3 ? k_bucket_sort<3, kCapLarge, 1024> : k_bucket_sort<0, kCapLarge, 1024>;
            hipLaunchKernelGGL(kb, dim3(B), dim3(1024), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf);
        }
        prof_end(st, pr);
    }
    CKEY_TRY(launch_status());
    // Overflowing buckets: read their ranges back and finish them with the radix sort.
    uint32_t novf = 0;
    CKEY_HIP_TRY(hipMemcpyAsync(&novf, q.ovf, 4, hipMemcpyDeviceToHost, st));
    CKEY_HIP_TRY(hipStreamSynchronize(st));
    if (novf == 0) return CKEY_OK;
    std::vector<uint32_t> ranges(2 * size_t(novf));
    CKEY_HIP_TRY(hipMemcpyAsync(ranges.data(), q.ovf + 1, ranges.size() * 4, hipMemcpyDeviceToHost, st));
    CKEY_HIP_TRY(hipStreamSynchronize(st));
    uint64_t rows = 0;
    for (uint32_t i = 0; i < novf; ++i) rows += ranges[2 * i + 1];
    if (novf > 64 || rows > n / 8) {
        // Widespread overflow (data the thresholds do not split): one radix
        // sort of everything by (key, row id) -- exact from any arrangement.
        CKEY_TRY(radix_sort(ck, n, words, nbits, rid, n, 8, 32, flags, ws, st));
    } else {
        for (uint32_t i = 0; i < novf; ++i) {
            const uint32_t s0 = ranges[2 * i], c = ranges[2 * i + 1];
            CKEY_TRY(radix_sort(ck + s0, n, words, nbits, rid + s0, c, 8, 32, flags, ws, st));
        }
    }
    if (flags) CKEY_TRY(fill_flag_or(flags, CKEY_FLAG_BUCKET_OVERFLOW, st));
    return CKEY_OK;
}

}  // namespace

ckey_status learned_sort(uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid, uint64_t n,
                         int mode, const void *model, uint32_t b_log2, uint32_t *flags, void *ws,
                         hipStream_t st) {
    if (n < 2) return CKEY_OK;
    const uint32_t B = 1u << b_log2;
    LLayout l;
    const LPtrs q = lptrs(ws, words, n, B, l);
    CKEY_TRY(fill_u32(q.hist, B, 0, st));
    CKEY_TRY(fill_u32(q.ovf, 1, 0, st));
    CKEY_TRY(assign_launch(mode, ck, n, bucket_args(model, B, q.bid, nullptr, nullptr, q.hist), nullptr, st));
    return bucket_finish(ck, words, nbits, rid, n, model, b_log2, q, l, flags, ws, st);
}

ckey_status compress_learned_sort(const KeySrc &k, const uint8_t *bm, uint64_t *ck, uint32_t words,
                                  uint32_t nbits, uint32_t *rid, int mode, const void *model,
                                  uint32_t b_log2, uint32_t *flags, void *ws, hipStream_t st) {
    const uint32_t B = 1u << b_log2;
    const uint64_t n = k.n;
    LLayout l;
    const LPtrs q = lptrs(ws, words, n, B, l);
    CKEY_TRY(fill_u32(q.hist, B, 0, st));
    CKEY_TRY(fill_u32(q.ovf, 1, 0, st));
    CKEY_TRY(compress_bucket_launch(k, bm, ck, words, rid, flags, mode,
                                    bucket_args(model, B, q.bid, nullptr, nullptr, q.hist), st));
    if (n < 2) return CKEY_OK;
    return bucket_finish(ck, words, nbits, rid, n, model, b_log2, q, l, flags, ws, st);
}

// ------------------------------------------------------------- model API --

size_t model_bytes(uint32_t b_log2) { return kOffT + (size_t(1) << b_log2) * 8; }

ckey_status model_init(void *model, uint64_t seed, hipStream_t st) {
    uint8_t *m8 = static_cast<uint8_t *>(model);
    hipLaunchKernelGGL(k_model_init, dim3(1), dim3(512), 0, st, reinterpret_cast<float *>(m8 + kOffParams),
                       reinterpret_cast<float *>(m8 + kOffM), reinterpret_cast<float *>(m8 + kOffV), seed);
    return launch_status();
}

ckey_status model_thresholds(void *model, uint32_t b_log2, const uint64_t *sorted, uint64_t m,
                             hipStream_t st) {
    const uint32_t B = 1u << b_log2;
    uint64_t *T = reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(model) + kOffT);
    hipLaunchKernelGGL(k_thresholds, dim3((B + 255) / 256), dim3(256), 0, st, sorted, m, T, B);
    return launch_status();
}

uint32_t grad_blocks(uint32_t M) {
    uint32_t g = (M + kWG - 1) / kWG;
    return g > 1024 ? 1024 : (g == 0 ? 1 : g);
}

size_t grad_workspace(uint32_t M) { return align256(size_t(grad_blocks(M)) * kNPad * 4); }

ckey_status model_grad(const void *model, const uint64_t *prefix, const float *target, uint64_t m,
                       uint32_t M, uint64_t seed, uint32_t step, float *grad, float *loss, void *ws,
                       hipStream_t st) {
    const uint32_t G = grad_blocks(M);
    float *partial = static_cast<float *>(ws);
    const int pr = prof_begin(st, "mlp_grad");
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(kWG), 0, st, params_of(model), prefix, target, m, M,
                       seed, step, partial);
    prof_end(st, pr);
    CKEY_TRY(launch_status());
    hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(512), 0, st, partial, G, grad, loss, nullptr,
                       nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 0u);
    return launch_status();
}

ckey_status model_train(void *model, const uint64_t *prefix, uint64_t m, uint32_t steps, uint32_t M,
                        float lr, float b1, float b2, float eps, uint64_t seed, float *loss_trace,
                        void *ws, hipStream_t st) {
    const uint32_t G = grad_blocks(M);
    float *partial = static_cast<float *>(ws);
    uint8_t *m8 = static_cast<uint8_t *>(model);
    float *p = reinterpret_cast<float *>(m8 + kOffParams);
    float *mm = reinterpret_cast<float *>(m8 + kOffM);
    float *vv = reinterpret_cast<float *>(m8 + kOffV);
    for (uint32_t s = 1; s <= steps; ++s) {
        const int pr = prof_begin(st, "mlp_grad");
        hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(kWG), 0, st, p, prefix, nullptr, m, M, seed, s,
                           partial);
        prof_end(st, pr);
        CKEY_TRY(launch_status());
        hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(512), 0, st, partial, G, nullptr,
                           loss_trace ? loss_trace + (s - 1) : nullptr, p, mm, vv, lr, b1, b2, eps, s);
        CKEY_TRY(launch_status());
    }
    return CKEY_OK;
}

ckey_status model_bucket(const void *model, uint32_t b_log2, int mode, const uint64_t *prefix,
                         uint64_t n, uint32_t *bucket, uint32_t *pred, unsigned long long *stats,
                         hipStream_t st) {
    return assign_launch(mode, prefix, n, bucket_args(model, 1u << b_log2, nullptr, bucket, pred, nullptr),
                         stats, st);
}

}  // namespace ckey
