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
// The MLP only predicts where to start looking: a search of T from the
// prediction always lands on the exact bucket, so exactness never depends on
// the network.  Up to 2^14 buckets T is in LDS and the search is a fixed-depth
// one over the 2^10 buckets around the guess (all of T when the key lies
// outside them); beyond, T is in memory and the search gallops outward from
// the guess; with statistics asked for it is exponential, then binary.  The
// splitter method needs no network: a binary search of T in LDS (beyond 2^14
// buckets, of a 1-in-S sample of T in LDS, then of T's run).
//
// Sort: assign buckets (+ histogram) -> scan -> group rows by bucket (a
// stable sort on the bucket id: two 7-bit passes) -> one workgroup per
// bucket sorts it in place in LDS by the offset of the first word from the
// bucket's lower threshold (a counting pass over its top bits, then a rank of
// each group of equal top bits by the whole offset), then orders runs of equal
// first words by the remaining words and the row id.  Buckets larger than the LDS capacity, or
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
constexpr int kCapHuge = 10240;  // second chance for buckets over those (one workgroup per CU)
constexpr int kRunCap = 32;      // max run of equal first words sorted in place

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

// Sum of v over the wave, returned to every lane: the DPP inclusive scan of
// wave_incl_scan (shifts within 16-lane rows, then the row broadcasts) in
// fp32, whose total lane 63 holds.  A fixed order, so the result is the same
// on every run.
__device__ __forceinline__ float wave_total(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Forward + backward on M samples; per-block partial sums (fixed order).
// target == nullptr: sample i = hash(seed, step, j) mod m, target (i+0.5)/m.
//
// Lane k of a wave owns hidden unit k: it holds the unit's five weights and
// bias and sums the unit's gradient over the wave's samples in registers.  A
// wave takes 64 samples at a time (lane j loads sample j's word and target
// and computes its features), then steps through them four at a time, each
// sample's features read from its lane as scalars; the one cross-lane sum per
// sample is the network output.  The gradient (mean squared error over M):
// dL/dy = 2(y - t)/M; w2[k] gets dy*h[k]; where unit k is active (a > 0),
// b1[k] gets dy*w2[k] and w1[k][c] gets dy*w2[k]*f[c]; b2 gets dy.
__global__ __launch_bounds__(kWG) void k_mlp_grad(const float *__restrict__ p,
                                                  const uint64_t *__restrict__ prefix,
                                                  const float *__restrict__ target, uint64_t m,
                                                  uint32_t M, uint64_t seed, uint32_t step,
                                                  float *__restrict__ partial) {
    static_assert(kH == 64, "one hidden unit per lane");
    constexpr int kQ = 4;  // samples in flight per step of a wave
    __shared__ float s_acc[kWG / 64][kNPad];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const float invM = 1.0f / float(M);
    float w1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w1[c] = p[4 * lane + c];
    const float b1 = p[4 * kH + lane], w2 = p[5 * kH + lane], b2 = p[6 * kH];
    float gw1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float gb1 = 0.0f, gw2 = 0.0f, gb2 = 0.0f, gl = 0.0f;
    for (uint64_t base = (uint64_t(blockIdx.x) * (kWG / 64) + wave) * 64; base < M;
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
        const uint32_t nv = uint32_t(min<uint64_t>(64, uint64_t(M) - base));
        for (uint32_t s0 = 0; s0 < nv; s0 += kQ) {
            float fs[kQ][4], h[kQ], y[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int src = int(min<uint32_t>(s0 + q, 63u));
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    fs[q][c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f[c]), src));
                float a = b1;
#pragma unroll
                for (int c = 0; c < 4; ++c) a = fmaf(w1[c], fs[q][c], a);
                h[q] = fmaxf(a, 0.0f);
                y[q] = w2 * h[q];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) y[q] = wave_total(y[q]) + b2;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int src = int(min<uint32_t>(s0 + q, 63u));
                const float ts = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), src));
                const float e = s0 + q < nv ? y[q] - ts : 0.0f;
                const float dy = 2.0f * e * invM;
                gw2 = fmaf(dy, h[q], gw2);
                const float g = h[q] > 0.0f ? dy * w2 : 0.0f;
                gb1 += g;
#pragma unroll
                for (int c = 0; c < 4; ++c) gw1[c] = fmaf(g, fs[q][c], gw1[c]);
                gb2 += dy;
                gl = fmaf(e * e, invM, gl);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s_acc[wave][4 * lane + c] = gw1[c];
    s_acc[wave][4 * kH + lane] = gb1;
    s_acc[wave][5 * kH + lane] = gw2;
    if (lane < kNPad - 6 * kH) {  // b2, the loss and the padding
        const int k = 6 * kH + lane;
        s_acc[wave][k] = k == 6 * kH ? gb2 : k == kLoss ? gl : 0.0f;
    }
    __syncthreads();
    for (int k = tid; k < kNPad; k += kWG) {
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kWG / 64; ++w) s += s_acc[w][k];
        partial[uint64_t(blockIdx.x) * kNPad + k] = s;
    }
}

// Sum G partial rows and then either write grad/loss or take an Adam step.
// Block b owns the kRedCols slots from b*kRedCols; its thread (r, c) sums rows
// r, r + kRedRows, ... of slot c in order (eight loads in flight), and the
// kRedRows sums are added in the order of r: a fixed order, the same on every
// run.
constexpr int kRedCols = 49, kRedRows = 10, kRedBlocks = kNPad / kRedCols;
static_assert(kRedCols * kRedBlocks == kNPad && kRedCols * kRedRows <= 512, "reduction layout");
__global__ __launch_bounds__(512) void k_mlp_reduce(const float *__restrict__ partial, uint32_t G,
                                                    float *__restrict__ grad_out,
                                                    float *__restrict__ loss_out, float *p, float *m,
                                                    float *v, float lr, float b1, float b2, float eps,
                                                    uint32_t t) {
    __shared__ float s_part[kRedRows][kRedCols];
    const int c = threadIdx.x % kRedCols, r = threadIdx.x / kRedCols;
    const int i = blockIdx.x * kRedCols + c;
    if (r < kRedRows) {
        float s = 0.0f;
        uint32_t g = uint32_t(r);
        for (; g + 7u * kRedRows < G; g += 8u * kRedRows) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = partial[uint64_t(g + u * kRedRows) * kNPad + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; g < G; g += kRedRows) s += partial[uint64_t(g) * kNPad + i];
        s_part[r][c] = s;
    }
    __syncthreads();
    if (r != 0 || i > kLoss) return;
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < kRedRows; ++q) s += s_part[q][c];
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
// Persistent: a workgroup loads the thresholds into LDS once and takes the
// chunks of kAssignChunk keys blockIdx.x, + gridDim.x, ...  Its packed 16-bit
// bucket counters are exact up to 65535: after a chunk, a pair of counters is
// added to the global histogram and cleared only when one of them could pass
// that with the next chunk's keys, and every pair after the workgroup's last
// chunk (keys spread over the buckets: one flush per workgroup).
constexpr uint64_t kAssignChunk = 32 * kBucketWG;
static_assert(kAssignChunk <= 65535, "a chunk fits the 16-bit counters");
template <int MODE>
__global__ __launch_bounds__(kBucketWG) void k_bucket_assign(const uint64_t *__restrict__ w0,
                                                             uint64_t n, BucketArgs ba,
                                                             unsigned long long *__restrict__ stats) {
    extern __shared__ uint32_t s_dyn[];
    bucket_lds_init<MODE>(ba, s_dyn);
    __syncthreads();
    uint32_t probes = 0, err = 0;
    for (uint64_t c = blockIdx.x; c * kAssignChunk < n; c += gridDim.x) {
        const uint64_t i0 = c * kAssignChunk;
        const uint64_t i1 = min<uint64_t>(n, i0 + kAssignChunk);
        if (MODE == 0 && !stats) {
            // Splitter: eight keys per thread, all their loads first, then their
            // searches interleaved (every threshold in LDS, or a sample of them).
            for (uint64_t b0 = i0 + threadIdx.x; b0 < i1; b0 += 8 * kBucketWG) {
                uint64_t x[8];
                uint32_t b[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    x[q] = r < i1 ? w0[r] : 0ull;
                }
                if (ba.S == 1)
                    splitter_search_n<8>(ba, s_dyn, x, b);
                else
                    splitter_search_sampled_n<8>(ba, s_dyn, x, b);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    if (r < i1) bucket_record<MODE>(ba, s_dyn, b[q], r);
                }
            }
        } else if (MODE == 1 && ba.S == 1 && !stats) {
            // Learned with every threshold in LDS: four keys' networks at once,
            // then the fixed-depth search around each guess.
            for (uint64_t b0 = i0 + threadIdx.x; b0 < i1; b0 += 4 * kBucketWG) {
                uint64_t x[4];
                uint32_t g[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    x[q] = r < i1 ? w0[r] : 0ull;
                }
                predict_bucket_n<4>(ba.p, x, ba.B, g);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    const uint32_t b = correct_bucket_window<512>(reinterpret_cast<const uint64_t *>(s_dyn), ba.B, x[q], g[q]);
                    if (r < i1) bucket_record<MODE>(ba, s_dyn, b, r);
                }
            }
        } else if (MODE == 1 && !stats) {
            // Learned beyond 2^14 buckets (T in memory): four keys' networks at
            // once, then their galloping searches of T from the guesses together.
            for (uint64_t b0 = i0 + threadIdx.x; b0 < i1; b0 += 4 * kBucketWG) {
                uint64_t x[4];
                uint32_t g[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    x[q] = r < i1 ? w0[r] : 0ull;
                }
                predict_bucket_n<4>(ba.p, x, ba.B, g);
                correct_bucket_n<4>(ba.T, ba.B, x, g, b);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t r = b0 + uint64_t(q) * kBucketWG;
                    if (r < i1) bucket_record<MODE>(ba, s_dyn, b[q], r);
                }
            }
        } else {  // with statistics (probes, guess error)
            for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBucketWG)
                (void)bucket_assign_one<MODE>(ba, s_dyn, w0[i], i, probes, err);
        }
        __syncthreads();
        const uint64_t nx = (c + gridDim.x) * kAssignChunk;
        bucket_lds_flush_before<MODE>(ba, s_dyn, nx < n ? uint32_t(min<uint64_t>(kAssignChunk, n - nx)) : 0u);
        __syncthreads();  // counters cleared before the next chunk's records
    }
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

// Exclusive scan of B counters by one 1024-thread workgroup -> starts[0..B].
// Thread t owns B/1024 consecutive counters (16-byte loads when that is a
// multiple of 4, i.e. B >= 4096).
__global__ __launch_bounds__(1024) void k_bucket_scan(const uint32_t *__restrict__ hist, uint32_t B,
                                                      uint32_t *__restrict__ starts) {
    __shared__ uint32_t s_w[16];
    const int tid = threadIdx.x;
    const uint32_t per = (B + 1023) / 1024;
    const uint32_t b0 = tid * per;
    const bool vec = (per & 3u) == 0;
    uint32_t sum = 0;
    if (vec) {
        for (uint32_t q = 0; q < per; q += 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(hist + b0 + q);
            sum += v.x + v.y + v.z + v.w;
        }
    } else {
        for (uint32_t q = 0; q < per; ++q)
            if (b0 + q < B) sum += hist[b0 + q];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_n<1024>(sum, s_w, tot);
    if (vec) {
        for (uint32_t q = 0; q < per; q += 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(hist + b0 + q);
            uint4 o;
            o.x = run;
            o.y = o.x + v.x;
            o.z = o.y + v.y;
            o.w = o.z + v.z;
            run = o.w + v.w;
            *reinterpret_cast<uint4 *>(starts + b0 + q) = o;
        }
    } else {
        for (uint32_t q = 0; q < per; ++q)
            if (b0 + q < B) {
                starts[b0 + q] = run;
                run += hist[b0 + q];
            }
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
// lies in [T[b], T[b+1]); the LDS sort key is the offset x - T[b], whose order
// and equal values are those of the first words.
//
// 1. Order by the offset: a counting pass over its top kG bits (kG = 12 for
//    1024 threads, 11 for 512; unstable -- the starting order is arbitrary)
//    puts the offsets in groups of equal top bits; a second counting pass
//    splits every group of g offsets over g counters by the next kG bits
//    (keys whose top bits carry little information, such as 3-bit codes of
//    4 letters, still end in small ranges); each offset then counts the
//    members of its range below it and equal to it, which gives its final
//    position and the run of equal offsets it belongs to.  A range larger
//    than kTieCap instead sends the bucket through an LSD over every varying
//    8-bit digit (the first pass unstable by LDS atomics, later ones stable by
//    wave ballots), after which runs are found by comparing neighbours.
// 2. Runs of equal offsets (equal first words) are ordered by the remaining
//    words and the row id: each array is staged in LDS and the members of
//    every run are ranked by it in parallel, stably (an LSD within the runs,
//    row ids first, then words w-1 .. 1).
// 3. The first words are written once the order is final; the other arrays
//    are staged in LDS (coalesced load) and written back in sorted order
//    (coalesced store).
//
// Buckets it cannot sort go to ovf as (bucket, start, count) triples after
// ovf[0] (their count).  Every thread of the workgroup calls it.
template <int WC, int kCap, int kSortWG>
__device__ __forceinline__ void sort_bucket(
    uint32_t b, uint64_t *__restrict__ ck, uint32_t *__restrict__ rid, uint64_t n, uint32_t words_rt,
    const uint32_t *__restrict__ starts, const uint64_t *__restrict__ T, uint32_t B,
    uint32_t *__restrict__ ovf) {
    constexpr int NW = kSortWG / 64;
    constexpr int PER = (kCap + kSortWG - 1) / kSortWG;
    constexpr uint32_t kTieCap = 256;
    static_assert(NW == 8 || NW == 16, "512 or 1024 threads");
    constexpr int kG = NW == 16 ? 12 : 11;  // counting-pass digit bits: 2^kG = 4 per thread
    // LSD fallback packing: row (kIdB bits) | digit (8) | rank in the wave's slice (kRkB bits)
    constexpr int kRkB = PER * 64 <= 512 ? 9 : PER * 64 <= 1024 ? 10 : 11;
    constexpr int kIdB = 32 - 8 - kRkB;
    static_assert(kCap <= (1 << kIdB) && kCap < 65535 && PER * 64 <= (1 << kRkB),
                  "packed rows, ranks and 16-bit positions");
    __shared__ uint64_t s_kg[kCap];      // offsets in group order (final order after an LSD);
                                         // afterwards staging of the other arrays
    __shared__ uint16_t s_idx[2][kCap];  // [1]: row of each group position, [0]: row of each
                                         // final position; then ping-pong
    __shared__ uint16_t s_run[kCap];     // second-pass counters, then the start of the run of
                                         // equal offsets at each position
    __shared__ uint16_t s_wc[NW][256];   // 2^kG packed 16-bit group counters, then starts;
                                         // per-wave digit counts of the LSD
    __shared__ uint32_t s_vary[4];       // AND, AND, OR, OR of the offsets' high and low halves
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint32_t s_flag[3];       // some run of equal offsets / a run longer than
                                         // kRunCap / a group larger than kTieCap
    __shared__ int32_t s_rb[2 * NW];     // run_carries exchange
    const uint32_t words = WC > 0 ? uint32_t(WC) : words_rt;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t start = starts[b];
    const uint32_t cnt = starts[b + 1] - start;
    auto overflow = [&]() {  // leave the bucket for the radix sort
        if (tid == 0) {
            const uint32_t slot = atomicAdd(&ovf[0], 1u);
            ovf[1 + 3 * slot] = b;
            ovf[2 + 3 * slot] = start;
            ovf[3 + 3 * slot] = cnt;
        }
    };
    if (cnt < 2) return;
    if (cnt > uint32_t(kCap)) {
        overflow();
        return;
    }
    const uint64_t lo = T[b], hi = (b + 1 < B) ? T[b + 1] - 1 : ~0ull;
    const uint64_t span = hi - lo;  // every offset is <= span
    const uint32_t gsh = (span >> kG) == 0 ? 0u : uint32_t(64 - __clzll(span)) - uint32_t(kG);
    uint32_t *gcnt = reinterpret_cast<uint32_t *>(&s_wc[0][0]);  // 2^kG packed 16-bit counters
    for (int t = tid; t < (1 << kG) / 2; t += kSortWG) gcnt[t] = 0u;
    for (int t = tid; t < kCap / 2; t += kSortWG) reinterpret_cast<uint32_t *>(s_run)[t] = 0u;
    if (tid < 4) s_vary[tid] = tid < 2 ? ~0u : 0u;
    if (tid < 3) s_flag[tid] = 0u;
    uint32_t a_and[2] = {~0u, ~0u}, a_or[2] = {0u, 0u};
    uint64_t xs[PER];
    uint32_t dg[PER];  // counting-pass digit << 16 | rank within the digit
#pragma unroll
    for (int u = 0; u < PER; ++u) {  // all loads first: PER in flight per thread
        const uint32_t j = tid + u * kSortWG;
        xs[u] = j < cnt ? ck[start + j] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t j = tid + u * kSortWG;
        dg[u] = 0u;
        if (j < cnt) {
            xs[u] -= lo;
            const uint32_t h32 = uint32_t(xs[u] >> 32), l32 = uint32_t(xs[u]);
            dg[u] = uint32_t(min<uint64_t>(xs[u] >> gsh, (1u << kG) - 1u)) << 16;  // x in [lo, hi]: no clamp
            a_and[0] &= h32;
            a_or[0] |= h32;
            a_and[1] &= l32;
            a_or[1] |= l32;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a_and[0] &= __shfl_xor(a_and[0], off, 64);
        a_and[1] &= __shfl_xor(a_and[1], off, 64);
        a_or[0] |= __shfl_xor(a_or[0], off, 64);
        a_or[1] |= __shfl_xor(a_or[1], off, 64);
    }
    __syncthreads();
    if (lane == 0) {
        atomicAnd(&s_vary[0], a_and[0]);
        atomicAnd(&s_vary[1], a_and[1]);
        atomicOr(&s_vary[2], a_or[0]);
        atomicOr(&s_vary[3], a_or[1]);
    }
    // Counting pass: rank within the digit (LDS atomics), scan, place.
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t j = tid + u * kSortWG;
        if (j < cnt) {
            const uint32_t d = dg[u] >> 16, h = 16u * (d & 1u);
            dg[u] |= (atomicAdd(&gcnt[d >> 1], 1u << h) >> h) & 0xFFFFu;
        }
    }
    __syncthreads();
    {
        const uint32_t w0 = gcnt[2 * tid], w1 = gcnt[2 * tid + 1];
        const uint32_t c0 = w0 & 0xFFFFu, c1 = w0 >> 16, c2 = w1 & 0xFFFFu, c3 = w1 >> 16;
        uint32_t all;
        const uint32_t ex = block_excl_scan_n<kSortWG>(c0 + c1 + c2 + c3, s_tmp, all);
        gcnt[2 * tid] = ex | ((ex + c0) << 16);
        gcnt[2 * tid + 1] = (ex + c0 + c1) | ((ex + c0 + c1 + c2) << 16);
    }
    __syncthreads();
    auto gstart = [&](uint32_t d) { return (gcnt[d >> 1] >> (16u * (d & 1u))) & 0xFFFFu; };
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t j = tid + u * kSortWG;
        if (j < cnt) {
            const uint32_t pos = gstart(dg[u] >> 16) + (dg[u] & 0xFFFFu);
            s_kg[pos] = xs[u];
            s_idx[1][pos] = uint16_t(j);
        }
    }
    __syncthreads();
    // Second counting pass, within the groups: a group of g offsets starting
    // at gs gets counters gs .. gs+g-1, and an offset goes to counter
    // gs + (its next kG bits * g >> kG) -- order-preserving, and about one
    // offset per counter when those bits are spread.
    uint32_t *cnt2 = reinterpret_cast<uint32_t *>(s_run);  // kCap packed 16-bit counters
    uint64_t kv[PER];
    uint32_t ip[PER], sb[PER];  // row | counter << 16 (then | position << 16); rank, then start | count << 16
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t p = tid + u * kSortWG;
        if (p >= cnt) continue;
        kv[u] = s_kg[p];
        const uint32_t d = uint32_t(min<uint64_t>(kv[u] >> gsh, (1u << kG) - 1u));
        const uint32_t gs = gstart(d), g = (d + 1 < (1u << kG) ? gstart(d + 1) : cnt) - gs;
        const uint64_t low = kv[u] & ((1ull << gsh) - 1ull);
        const uint32_t nx = gsh >= uint32_t(kG) ? uint32_t(low >> (gsh - kG)) : uint32_t(low << (kG - gsh));
        const uint32_t c = gs + ((nx * g) >> kG);
        const uint32_t h = 16u * (c & 1u);
        sb[u] = (atomicAdd(&cnt2[c >> 1], 1u << h) >> h) & 0xFFFFu;
        ip[u] = uint32_t(s_idx[1][p]) | (c << 16);
    }
    __syncthreads();
    {
        constexpr int W = (kCap / 2 + kSortWG - 1) / kSortWG;  // packed words per thread
        uint32_t v[W], c[2 * W], sum = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const uint32_t t = tid * W + i;
            v[i] = t < uint32_t(kCap / 2) ? cnt2[t] : 0u;
            c[2 * i] = v[i] & 0xFFFFu;
            c[2 * i + 1] = v[i] >> 16;
            sum += c[2 * i] + c[2 * i + 1];
        }
        uint32_t all;
        uint32_t ex = block_excl_scan_n<kSortWG>(sum, s_tmp, all);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const uint32_t t = tid * W + i;
            const uint32_t e0 = ex, e1 = ex + c[2 * i];
            ex = e1 + c[2 * i + 1];
            if (t < uint32_t(kCap / 2)) cnt2[t] = e0 | (e1 << 16);
        }
    }
    __syncthreads();
    auto start2 = [&](uint32_t c) { return (cnt2[c >> 1] >> (16u * (c & 1u))) & 0xFFFFu; };
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t p = tid + u * kSortWG;
        if (p >= cnt) continue;
        const uint32_t c = ip[u] >> 16;
        const uint32_t s2 = start2(c), e2 = c + 1 < cnt ? start2(c + 1) : cnt;
        const uint32_t pos = s2 + sb[u];
        s_kg[pos] = kv[u];  // every read of the group order was before the barrier
        s_idx[1][pos] = uint16_t(ip[u]);
        ip[u] = (ip[u] & 0xFFFFu) | (pos << 16);
        sb[u] = s2 | ((e2 - s2) << 16);
    }
    __syncthreads();
    // Each offset counts the members of its counter's range below it and
    // equal to it: its final position and the run of equal offsets it is in.
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t p = tid + u * kSortWG;
        if (p >= cnt) continue;
        const uint32_t gs = sb[u] & 0xFFFFu, len = sb[u] >> 16, pos = ip[u] >> 16;
        uint32_t lt = 0, eq = 1, eqb = 0;
        if (len > kTieCap) {
            s_flag[2] = 1u;
        } else if (len > 1) {
            eq = 0;
            for (uint32_t q = gs; q < gs + len; ++q) {
                const uint64_t kq = s_kg[q];
                lt += kq < kv[u] ? 1u : 0u;
                eq += kq == kv[u] ? 1u : 0u;
                eqb += (kq == kv[u] && q < pos) ? 1u : 0u;
            }
        }
        const uint32_t fp = gs + lt + eqb;
        sb[u] = fp;
        s_idx[0][fp] = uint16_t(ip[u]);
        s_run[fp] = uint16_t(gs + lt);  // the counters were read before the barrier
        if (eq > 1) s_flag[0] = 1u;
        if (eq > uint32_t(kRunCap)) s_flag[1] = 1u;
    }
    __syncthreads();
    if (s_flag[2] == 0u) {  // offsets to final order
#pragma unroll
        for (int u = 0; u < PER; ++u)
            if (tid + u * kSortWG < cnt) s_kg[sb[u]] = kv[u];
    }
    __syncthreads();
    // With a fixed word count, the row ids and words 1..WC-1 are loaded into
    // registers once, all loads in flight together (before the first words
    // are stored: loads and stores retire in order).
    constexpr int NR = WC > 1 ? WC - 1 : 1;
    uint32_t rv[PER];
    uint64_t wv[NR][PER];
    auto load_rest = [&]() {
        if constexpr (WC > 0) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                const bool ok = j < cnt;
                rv[u] = ok ? rid[start + j] : 0u;
#pragma unroll
                for (int k = 0; k < WC - 1; ++k) wv[k][u] = ok ? ck[uint64_t(k + 1) * n + start + j] : 0ull;
            }
        }
    };
    if (s_flag[2] == 0u) {
        if (s_flag[1]) {
            overflow();
            return;
        }
        load_rest();
        // First words (equal within a run of equal offsets, so already final).
        for (uint32_t j = tid; j < cnt; j += kSortWG) ck[start + j] = lo + s_kg[j];
    } else {
        // LSD over every varying 8-bit digit of the offset, on group positions
        // (ping-pong s_idx[0] <-> s_run), then everything moved to final order.
        const uint32_t vary[2] = {s_vary[0] ^ s_vary[2], s_vary[1] ^ s_vary[3]};
        // Digits of the 64-bit offset, 0 = least significant; d < 4 is in the low half.
        auto digit_varies = [&](int d) { return ((vary[d < 4 ? 1 : 0] >> (8 * (d & 3))) & 0xFFu) != 0; };
        for (uint32_t j = tid; j < cnt; j += kSortWG) s_idx[0][j] = uint16_t(j);  // if nothing varies
        __syncthreads();
        // Each wave ranks a contiguous slice of Q elements (Q a multiple of 64) in
        // order, at most kRounds rounds of 64.
        constexpr int kRounds = PER;
        const uint32_t Q = ((cnt + NW * 64 - 1) / (NW * 64)) * 64;
        const uint32_t e0 = wave * Q, e1 = min(cnt, e0 + Q);
        const uint64_t lane_lt = (1ull << lane) - 1ull;
        uint32_t *cnt32 = reinterpret_cast<uint32_t *>(&s_wc[0][0]);  // 256 counters (unstable pass)
        int cur = 0;  // 0: s_idx[0], 1: s_run
        bool first = true;
        for (int d = 0; d < 8; ++d) {
            if (!digit_varies(d)) continue;
            const uint32_t shift = 8 * uint32_t(d);
            uint16_t *src = cur ? s_run : s_idx[0];
            uint16_t *dst = cur ? s_idx[0] : s_run;
            if (first) {
                // Unstable counting pass straight from the group order.
                first = false;
                if (tid < 256) cnt32[tid] = 0u;
                __syncthreads();
                for (uint32_t j = tid; j < cnt; j += kSortWG) atomicAdd(&cnt32[uint32_t(s_kg[j] >> shift) & 0xFFu], 1u);
                __syncthreads();
                const uint32_t c = tid < 256 ? cnt32[tid] : 0u;
                uint32_t all;
                const uint32_t ex = block_excl_scan_n<kSortWG>(c, s_tmp, all);
                if (tid < 256) cnt32[tid] = ex;
                __syncthreads();
                for (uint32_t j = tid; j < cnt; j += kSortWG) {
                    const uint32_t pos = atomicAdd(&cnt32[uint32_t(s_kg[j] >> shift) & 0xFFu], 1u);
                    s_run[pos] = uint16_t(j);
                }
                __syncthreads();
                cur = 1;
                continue;
            }
            for (int t = tid; t < NW * 256; t += kSortWG) (&s_wc[0][0])[t] = 0;
            __syncthreads();
            // per element: id << (8 + kRkB) | digit << kRkB | rank within the wave's slice
            uint32_t pk[kRounds];
#pragma unroll
            for (int u = 0; u < kRounds; ++u) {
                const uint32_t e = e0 + 64 * u + lane;
                const bool valid = e < e1;
                const uint32_t id = valid ? src[e] : 0u;
                const uint32_t dig = valid ? uint32_t(s_kg[id] >> shift) & 0xFFu : 0u;
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
                pk[u] = (id << (8 + kRkB)) | (dig << kRkB) | (old + below);
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
                if (e < e1)
                    dst[s_wc[wave][(pk[u] >> kRkB) & 0xFFu] + (pk[u] & ((1u << kRkB) - 1u))] =
                        uint16_t(pk[u] >> (8 + kRkB));
            }
            __syncthreads();
            cur ^= 1;
        }
        {
            const uint16_t *fin = cur ? s_run : s_idx[0];
            uint64_t kf[PER];
            uint32_t idf[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                if (j < cnt) {
                    const uint32_t g = fin[j];
                    kf[u] = s_kg[g];
                    idf[u] = s_idx[1][g];
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                if (j < cnt) {
                    s_kg[j] = kf[u];
                    s_idx[0][j] = uint16_t(idf[u]);
                }
            }
            __syncthreads();
        }
        // Runs of equal offsets from neighbour comparisons.
        const uint32_t j0 = PER * uint32_t(tid);
        uint32_t rs = 0;
        uint64_t prevk = (j0 > 0 && j0 - 1 < cnt) ? s_kg[j0 - 1] : 0ull;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = j0 + u;
            if (j < cnt) {
                const uint64_t k = s_kg[j];
                if (j == 0 || k != prevk) rs |= 1u << u;
                prevk = k;
            }
        }
        uint32_t cs, ce;
        run_carries<PER, kSortWG>(cnt, rs, &cs, &ce, s_rb);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = j0 + u;
            if (j >= cnt) break;
            if ((rs >> u) & 1u) cs = j;
            const uint32_t later = rs >> (u + 1);
            const uint32_t len = (later ? j + uint32_t(__ffs(later)) : ce) - cs;
            if (len > uint32_t(kRunCap)) s_flag[1] = 1u;
            if (len > 1) s_flag[0] = 1u;
            s_run[j] = uint16_t(cs);
        }
        __syncthreads();
        if (s_flag[1]) {
            overflow();
            return;
        }
        load_rest();
        for (uint32_t j = tid; j < cnt; j += kSortWG) ck[start + j] = lo + s_kg[j];
    }
    const bool fixup = s_flag[0] != 0u;
    int cur = 0;
    __syncthreads();  // offsets are dead from here on
    uint64_t *stg = s_kg;  // 8*kCap bytes
    // Rank the members of every run of equal offsets by the staged array,
    // stably: s_idx[cur] -> s_idx[cur ^ 1].
    auto rank_runs = [&]() {
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
    };
    if constexpr (WC > 0) {
        // Arrays from registers: a = -1 row ids, else word a.
        auto stage = [&](int a) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t j = tid + u * kSortWG;
                if (j < cnt) stg[j] = a < 0 ? uint64_t(rv[u]) : wv[a < 1 ? 0 : a - 1][u];
            }
        };
        auto put = [&](int a) {  // write the staged array a in sorted order
            const uint16_t *ord = s_idx[cur];
            if (a < 0) {
                for (uint32_t j = tid; j < cnt; j += kSortWG) rid[start + j] = uint32_t(stg[ord[j]]);
            } else {
                uint64_t *wk = ck + uint64_t(a) * n + start;
                for (uint32_t j = tid; j < cnt; j += kSortWG) wk[j] = stg[ord[j]];
            }
        };
        if (fixup) {
            // Members of runs get compact indices (by final position); their
            // later words and row ids are staged compactly, and each member is
            // ranked within its run by (word 1, .., word WC-1, row id) at once.
            constexpr int C = (kCap * 8) / (8 * (WC - 1) + 4);  // members staged at once
            uint16_t *map = s_idx[1];  // row -> compact index, 0xFFFF outside runs
            const uint16_t *ord = s_idx[0];
            uint32_t tot;
            {
                const uint32_t f0 = PER * uint32_t(tid);
                uint32_t mem = 0, nm = 0;
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const uint32_t f = f0 + u;
                    if (f < cnt) {
                        const uint32_t rs = s_run[f];
                        const bool alone = rs == f && (f + 1 == cnt || s_run[f + 1] != f);
                        if (!alone) {
                            mem |= 1u << u;
                            ++nm;
                        }
                    }
                }
                uint32_t c = block_excl_scan_n<kSortWG>(nm, s_tmp, tot);
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const uint32_t f = f0 + u;
                    if (f < cnt) map[ord[f]] = ((mem >> u) & 1u) ? uint16_t(c++) : uint16_t(0xFFFFu);
                }
            }
            __syncthreads();
            if (tot <= uint32_t(C)) {
                uint64_t *cw = s_kg;                                           // [WC-1][C] words
                uint32_t *cr = reinterpret_cast<uint32_t *>(s_kg + (WC - 1) * C);  // [C] row ids
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const uint32_t j = tid + u * kSortWG;
                    if (j < cnt) {
                        const uint32_t m = map[j];
                        if (m != 0xFFFFu) {
#pragma unroll
                            for (int k = 0; k < WC - 1; ++k) cw[k * C + m] = wv[k][u];
                            cr[m] = rv[u];
                        }
                    }
                }
                __syncthreads();
                uint32_t np[PER];  // new position | row << 16
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const uint32_t f = tid + u * kSortWG;
                    np[u] = ~0u;
                    if (f >= cnt) continue;
                    const uint32_t id = ord[f], c = map[id];
                    if (c == 0xFFFFu) continue;
                    uint64_t a[NR];
#pragma unroll
                    for (int k = 0; k < WC - 1; ++k) a[k] = cw[k * C + c];
                    const uint32_t ar = cr[c], rs = s_run[f];
                    // a run's members hold consecutive positions, and so
                    // consecutive compact indices: member q is cs + (q - rs)
                    const uint32_t cs = c - (f - rs);
                    uint32_t r = 0;
                    for (uint32_t q = rs; q < cnt && s_run[q] == rs; ++q) {
                        const uint32_t cq = cs + (q - rs);
                        int cmp = 0;  // -1: member q orders first
#pragma unroll
                        for (int k = 0; k < WC - 1; ++k) {
                            if (cmp == 0) {
                                const uint64_t x = cw[k * C + cq];
                                cmp = x < a[k] ? -1 : x > a[k] ? 1 : 0;
                            }
                        }
                        if (cmp == 0) cmp = cr[cq] < ar ? -1 : 0;
                        r += cmp < 0 ? 1u : 0u;
                    }
                    np[u] = (rs + r) | (id << 16);
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < PER; ++u)
                    if (np[u] != ~0u) s_idx[0][np[u] & 0xFFFFu] = uint16_t(np[u] >> 16);
                __syncthreads();
            } else {
                // Too many members to stage at once: LSD within the runs,
                // row ids, then words WC-1 .. 1.
#pragma unroll
                for (int k = -1; k < WC; ++k) {
                    if (k == 0) continue;
                    stage(k < 0 ? -1 : WC - k);
                    __syncthreads();
                    rank_runs();
                    __syncthreads();
                    cur ^= 1;
                }
            }
        }
#pragma unroll
        for (int a = 1; a < WC; ++a) {
            stage(a);
            __syncthreads();
            put(a);
            __syncthreads();
        }
        uint32_t *stage32 = reinterpret_cast<uint32_t *>(s_kg);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t j = tid + u * kSortWG;
            if (j < cnt) stage32[j] = rv[u];
        }
        __syncthreads();
        const uint16_t *ord = s_idx[cur];
        for (uint32_t j = tid; j < cnt; j += kSortWG) rid[start + j] = stage32[ord[j]];
        return;
    } else {
        // Wider keys: each array is loaded when it is needed.
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
                rank_runs();
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
        // (coalesced load, all of a thread's loads in flight at once), then
        // write it back in sorted order (coalesced store).
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
        uint32_t *stage32 = reinterpret_cast<uint32_t *>(s_kg);
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
}

// One workgroup per bucket; list (optional): the buckets to sort are
// list[1 + 3 i] for workgroup i (an overflow list of the smaller kernels),
// else bucket = workgroup.
template <int WC, int kCap, int kSortWG>
__global__ __launch_bounds__(kSortWG, (kCap > 5120 ? 4 : 8)) void k_bucket_sort(
    uint64_t *__restrict__ ck, uint32_t *__restrict__ rid, uint64_t n, uint32_t words_rt,
    const uint32_t *__restrict__ starts, const uint64_t *__restrict__ T, uint32_t B,
    uint32_t *__restrict__ ovf, const uint32_t *__restrict__ list) {
    const uint32_t b = list ? list[1 + 3 * blockIdx.x] : blockIdx.x;
    sort_bucket<WC, kCap, kSortWG>(b, ck, rid, n, words_rt, starts, T, B, ovf);
}

// Overflowing buckets when the host cannot be asked how many there are (a
// captured graph): every workgroup walks the overflow list of the first bucket
// sort (list[0] entries), sorting its share with the second-chance capacity;
// what still overflows goes to ovf2.  More than kMaxSecondChance entries
// (data the thresholds do not split) skip this and open the gate of the
// whole-array radix sort at once.
constexpr uint32_t kMaxSecondChance = 64;
template <int WC>
__global__ __launch_bounds__(1024, 4) void k_bucket_sort_again(
    uint64_t *__restrict__ ck, uint32_t *__restrict__ rid, uint64_t n, uint32_t words_rt,
    const uint32_t *__restrict__ starts, const uint64_t *__restrict__ T, uint32_t B,
    const uint32_t *__restrict__ list, uint32_t *__restrict__ ovf2, uint32_t *__restrict__ gate) {
    const uint32_t c = list[0];
    if (c > kMaxSecondChance) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *gate = 1u;
        return;
    }
    for (uint32_t i = blockIdx.x; i < c; i += gridDim.x) {
        __syncthreads();  // the previous bucket's LDS reads are done
        sort_bucket<WC, kCapHuge, 1024>(list[1 + 3 * i], ck, rid, n, words_rt, starts, T, B, ovf2);
    }
}

// Opens the fallback's gate when a bucket is still unsorted (and says so in
// the flags word); one thread.
__global__ void k_overflow_gate(const uint32_t *__restrict__ ovf2, uint32_t *__restrict__ gate,
                                uint32_t *__restrict__ flags) {
    const bool open = *gate != 0u || ovf2[0] != 0u;
    *gate = open ? 1u : 0u;
    if (open && flags) atomicOr(flags, CKEY_FLAG_BUCKET_OVERFLOW);
}

struct LLayout {
    size_t bid, hist, starts, ovf, ovf2, stats, sortws, total;
};

LLayout llayout(uint32_t words, uint64_t n, uint32_t B) {
    LLayout l{};
    size_t off = 0;
    l.bid = off;      off += align256(size_t(n) * 2);
    l.hist = off;     off += align256(size_t(B) * 4);
    l.starts = off;   off += align256(size_t(B + 1) * 4);
    l.ovf = off;      off += align256(size_t(3 * B + 1) * 4);
    l.ovf2 = off;     off += align256(size_t(3 * B + 1) * 4);
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
    const void *fn = mode ? reinterpret_cast<const void *>(k_bucket_assign<1>)
                          : reinterpret_cast<const void *>(k_bucket_assign<0>);
    raise_lds_limit(fn);
    // One pass of workgroups resident at once (each loads the thresholds once).
    const uint64_t blocks = std::min<uint64_t>((n + kBucketKeysPerWG - 1) / kBucketKeysPerWG,
                                               resident_grid(fn, kBucketWG, lds));
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

// The bucket layout and the fallback radix sort share the workspace from
// offset 0 (the radix sort starts once the lists are no longer needed); the
// gate of a captured fallback sits past both.
size_t gate_offset(uint32_t words, uint32_t nbits, uint64_t n, uint32_t b_log2) {
    const size_t a = llayout(words, n, 1u << b_log2).total;
    const size_t r = radix_workspace(words, nbits, n, 8, 32);
    return align256(a > r ? a : r);
}

size_t learned_workspace(uint32_t words, uint32_t nbits, uint64_t n, uint32_t b_log2) {
    return gate_offset(words, nbits, n, b_log2) + 256;
}

namespace {

struct LPtrs {
    uint16_t *bid;
    uint32_t *hist, *starts, *ovf, *ovf2;
};

LPtrs lptrs(void *ws, uint32_t words, uint64_t n, uint32_t B, LLayout &l) {
    l = llayout(words, n, B);
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    return LPtrs{reinterpret_cast<uint16_t *>(w8 + l.bid), reinterpret_cast<uint32_t *>(w8 + l.hist),
                 reinterpret_cast<uint32_t *>(w8 + l.starts),
                 reinterpret_cast<uint32_t *>(w8 + l.ovf), reinterpret_cast<uint32_t *>(w8 + l.ovf2)};
}

// From bucket ids and the bucket histogram: group by bucket, sort each bucket,
// finish overflowing buckets with the radix sort.  rid_identity: rid holds
// nothing yet and the row ids are 0..n-1 (generated by the first pass).
ckey_status bucket_finish(uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid,
                          bool rid_identity, uint64_t n, const void *model, uint32_t b_log2, const LPtrs &q, const LLayout &l,
                          uint32_t *flags, void *ws, hipStream_t st, uint32_t cap) {
    const uint32_t B = 1u << b_log2;
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, st, q.hist, B, q.starts);
    CKEY_TRY(launch_status());
    // Group rows by bucket: a stable sort by the bucket id (two one-sweep passes).
    CKEY_TRY(aux_sort(ck, rid, rid_identity, q.bid, n, words, b_log2, q.hist, flags, w8 + l.sortws, st));
    const uint64_t *T = thresholds_of(model);
    {
        const int pr = prof_begin(st, "bucket_sort");
        if (cap == 0) cap = n / B <= 1600 ? 1 : n / B <= 4400 ? 2 : 3;  // by the mean bucket size
        if (cap == 1) {  // small buckets: 2560-row capacity, 512 threads, 4 per CU
            auto kb = words == 1 ? k_bucket_sort<1, kCapSmall, 512> : words == 2 ? k_bucket_sort<2, kCapSmall, 512>
                    : words == 3 ? k_bucket_sort<3, kCapSmall, 512> : k_bucket_sort<0, kCapSmall, 512>;
            hipLaunchKernelGGL(kb, dim3(B), dim3(512), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf, nullptr);
        } else if (cap == 2) {  // 5120-row capacity, 1024 threads, 2 per CU
            auto kb = words == 1 ? k_bucket_sort<1, kCapLarge, 1024> : words == 2 ? k_bucket_sort<2, kCapLarge, 1024>
                    : words == 3 ? k_bucket_sort<3, kCapLarge, 1024> : k_bucket_sort<0, kCapLarge, 1024>;
            hipLaunchKernelGGL(kb, dim3(B), dim3(1024), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf, nullptr);
        } else {  // 10240-row capacity, 1 per CU
            auto kb = words == 1 ? k_bucket_sort<1, kCapHuge, 1024> : words == 2 ? k_bucket_sort<2, kCapHuge, 1024>
                    : words == 3 ? k_bucket_sort<3, kCapHuge, 1024> : k_bucket_sort<0, kCapHuge, 1024>;
            hipLaunchKernelGGL(kb, dim3(B), dim3(1024), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf, nullptr);
        }
        prof_end(st, pr);
    }
    CKEY_TRY(launch_status());
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    CKEY_HIP_TRY(hipStreamIsCapturing(st, &capture));
    if (capture != hipStreamCaptureStatusNone) {
        // Captured: no host round trip.  The second chance walks the list on
        // the device; a bucket it still cannot sort (or a widespread
        // overflow) opens the gate of one radix sort of everything by (key,
        // row id), exact from any arrangement, whose kernels are enqueued
        // always and return at once while the gate is closed.
        uint32_t *gate = reinterpret_cast<uint32_t *>(w8 + gate_offset(words, nbits, n, b_log2));
        CKEY_TRY(fill_u32(gate, 1, 0, st));
        CKEY_TRY(fill_u32(q.ovf2, 1, 0, st));
        int dev = 0, cus = 0;
        CKEY_HIP_TRY(hipGetDevice(&dev));
        CKEY_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const uint32_t grid = uint32_t(cus > 0 ? cus : 1);
        auto ka = words == 1 ? k_bucket_sort_again<1> : words == 2 ? k_bucket_sort_again<2>
                : words == 3 ? k_bucket_sort_again<3> : k_bucket_sort_again<0>;
        {
            const int pr = prof_begin(st, "bucket_sort_large");
            hipLaunchKernelGGL(ka, dim3(grid), dim3(1024), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf,
                               q.ovf2, gate);
            prof_end(st, pr);
        }
        CKEY_TRY(launch_status());
        hipLaunchKernelGGL(k_overflow_gate, dim3(1), dim3(1), 0, st, q.ovf2, gate, flags);
        CKEY_TRY(launch_status());
        return radix_sort(ck, n, words, nbits, rid, n, 8, 32, flags, ws, st, false, gate);
    }
    // Overflowing buckets (count, then (bucket, start, rows) triples).
    auto read_list = [&](const uint32_t *dev, std::vector<uint32_t> &v) -> ckey_status {
        uint32_t c = 0;
        CKEY_HIP_TRY(hipMemcpyAsync(&c, dev, 4, hipMemcpyDeviceToHost, st));
        CKEY_HIP_TRY(hipStreamSynchronize(st));
        v.assign(3 * size_t(c), 0u);
        if (c) {
            CKEY_HIP_TRY(hipMemcpyAsync(v.data(), dev + 1, v.size() * 4, hipMemcpyDeviceToHost, st));
            CKEY_HIP_TRY(hipStreamSynchronize(st));
        }
        return CKEY_OK;
    };
    std::vector<uint32_t> ov;
    CKEY_TRY(read_list(q.ovf, ov));
    uint32_t novf = uint32_t(ov.size() / 3);
    if (novf == 0) return CKEY_OK;
    uint64_t rows = 0;
    for (uint32_t i = 0; i < novf; ++i) rows += ov[3 * i + 2];
    if (novf > 64 || rows > n / 8) {
        // Widespread overflow (data the thresholds do not split): one radix
        // sort of everything by (key, row id) -- exact from any arrangement.
        CKEY_TRY(radix_sort(ck, n, words, nbits, rid, n, 8, 32, flags, ws, st));
        if (flags) CKEY_TRY(fill_flag_or(flags, CKEY_FLAG_BUCKET_OVERFLOW, st));
        return CKEY_OK;
    }
    // Second chance: the 10240-row in-LDS sort over the listed buckets.
    CKEY_TRY(fill_u32(q.ovf2, 1, 0, st));
    {
        auto kh = words == 1 ? k_bucket_sort<1, kCapHuge, 1024> : words == 2 ? k_bucket_sort<2, kCapHuge, 1024>
                : words == 3 ? k_bucket_sort<3, kCapHuge, 1024> : k_bucket_sort<0, kCapHuge, 1024>;
        const int pr = prof_begin(st, "bucket_sort_large");
        hipLaunchKernelGGL(kh, dim3(novf), dim3(1024), 0, st, ck, rid, n, words, q.starts, T, B, q.ovf2, q.ovf);
        prof_end(st, pr);
        CKEY_TRY(launch_status());
    }
    CKEY_TRY(read_list(q.ovf2, ov));
    novf = uint32_t(ov.size() / 3);
    if (novf == 0) return CKEY_OK;
    for (uint32_t i = 0; i < novf; ++i) {
        const uint32_t s0 = ov[3 * i + 1], c = ov[3 * i + 2];
        CKEY_TRY(radix_sort(ck + s0, n, words, nbits, rid + s0, c, 8, 32, flags, ws, st));
    }
    if (flags) CKEY_TRY(fill_flag_or(flags, CKEY_FLAG_BUCKET_OVERFLOW, st));
    return CKEY_OK;
}

}  // namespace

ckey_status learned_sort(uint64_t *ck, uint32_t words, uint32_t nbits, uint32_t *rid, uint64_t n,
                         int mode, const void *model, uint32_t b_log2, uint32_t *flags, void *ws,
                         hipStream_t st, uint32_t cap) {
    if (n < 2) return CKEY_OK;
    const uint32_t B = 1u << b_log2;
    LLayout l;
    const LPtrs q = lptrs(ws, words, n, B, l);
    CKEY_TRY(fill_u32(q.hist, B, 0, st));
    CKEY_TRY(fill_u32(q.ovf, 1, 0, st));
    CKEY_TRY(assign_launch(mode, ck, n, bucket_args(model, B, q.bid, nullptr, nullptr, q.hist), nullptr, st));
    return bucket_finish(ck, words, nbits, rid, false, n, model, b_log2, q, l, flags, ws, st, cap);
}

ckey_status compress_learned_sort(const KeySrc &k, const uint8_t *bm, uint64_t *ck, uint32_t words,
                                  uint32_t nbits, uint32_t *rid, int mode, const void *model,
                                  uint32_t b_log2, uint32_t *flags, void *ws, hipStream_t st, uint32_t cap) {
    const uint32_t B = 1u << b_log2;
    const uint64_t n = k.n;
    LLayout l;
    const LPtrs q = lptrs(ws, words, n, B, l);
    CKEY_TRY(fill_u32(q.hist, B, 0, st));
    CKEY_TRY(fill_u32(q.ovf, 1, 0, st));
    // The row ids start as 0..n-1: the first grouping pass generates them.
    const BucketArgs ba = bucket_args(model, B, q.bid, nullptr, nullptr, q.hist);
    // Splitter with every threshold in LDS: compression streams at copy speed
    // in small workgroups; the search then reads the first words again (8
    // bytes a key) in workgroups that hold all thresholds.  Together faster
    // than one kernel doing both at one 160 KB-LDS workgroup per CU.  With
    // only a sample in LDS (more than 2^14 buckets) the search reads T in
    // memory, and doing it while the keys are compressed hides those reads.
    ckey_status s = CKEY_ERR_UNSUPPORTED;
    if (mode == 1 || ba.S > 1)
        s = compress_bucket_launch(k, bm, ck, words, n < 2 ? rid : nullptr, flags, mode, ba, st);
    if (mode == 0 && s == CKEY_ERR_UNSUPPORTED) {
        CKEY_TRY(compress_launch(k, bm, ck, words, n < 2 ? rid : nullptr, flags, st));
        if (n >= 2) CKEY_TRY(assign_launch(mode, ck, n, ba, nullptr, st));
    } else {
        CKEY_TRY(s);
    }
    if (n < 2) return CKEY_OK;
    return bucket_finish(ck, words, nbits, rid, true, n, model, b_log2, q, l, flags, ws, st, cap);
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
    hipLaunchKernelGGL(k_mlp_reduce, dim3(kRedBlocks), dim3(512), 0, st, partial, G, grad, loss, nullptr,
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
        hipLaunchKernelGGL(k_mlp_reduce, dim3(kRedBlocks), dim3(512), 0, st, partial, G, nullptr,
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
