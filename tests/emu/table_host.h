// Host emulation of the persistent table-rebuild kernel (k_table.hip), used by
// a CPU test: the kernel source is compiled for the host with these
// definitions in place of the HIP runtime.  A workgroup is 256 threads with a
// std::barrier for __syncthreads and a 64-thread barrier per wave for ballots
// and DPP moves (the kernel's own scans, csrc/scan.h, run on a model of the
// DPP forms they use); many workgroups run at once on shared host memory with
// real atomics, so the work queue, the per-phase waits and the look-back run
// concurrently.  Every LDS array of a workgroup is its own heap block, so an
// address sanitizer build sees any out-of-bounds access to LDS or to the
// global buffers.
#pragma once
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <barrier>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <thread>
#include <vector>

#include <pthread.h>

#include "ckey.h"

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
typedef void *hipStream_t;
#define hipDeviceAttributeMultiprocessorCount 0

struct EmuTid {
    unsigned x;
};
struct EmuWG {
    void *lds[4];  // s_buf, u, s_tmp, s_item
    std::barrier<> *bar;
    std::barrier<> *wbar[4];
    int ballot[4][64];
    int dpp[4][64];
};
extern thread_local EmuTid threadIdx;
extern thread_local EmuWG *g_wg;
extern int g_nwg;

inline void __syncthreads() { g_wg->bar->arrive_and_wait(); }
// A wave's lanes all read before any writes (lockstep on the GPU).
#define EMU_WAVE_SYNC() g_wg->wbar[threadIdx.x / 64]->arrive_and_wait()
inline uint64_t __ballot(int pred) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    g_wg->ballot[w][l] = pred ? 1 : 0;
    g_wg->wbar[w]->arrive_and_wait();
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i)
        if (g_wg->ballot[w][i]) m |= 1ull << i;
    g_wg->wbar[w]->arrive_and_wait();
    return m;
}
// DPP move of a wave (the forms the scans use): every lane publishes src,
// then reads the lane its control word names.  row_shr:n (0x110 + n) reads
// lane - n of the same 16-lane row; row_bcast:15 (0x142) reads lane 15 of the
// previous row; row_bcast:31 (0x143) reads lane 31 (rows 2 and 3).  Rows
// outside row_mask (and banks outside bank_mask) keep `old`; a source outside
// the row reads 0 with bound_ctrl, else keeps `old`.
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    const int w = int(threadIdx.x) / 64, l = int(threadIdx.x) % 64, row = l / 16, in = l % 16;
    g_wg->dpp[w][l] = src;
    g_wg->wbar[w]->arrive_and_wait();
    int res = old;
    if (((row_mask >> row) & 1) && ((bank_mask >> (in / 4)) & 1)) {
        int from = -1;
        if ((ctrl & ~0xF) == 0x110) {
            const int sh = ctrl & 0xF;
            from = in >= sh ? l - sh : -1;
        } else if (ctrl == 0x142) {
            from = row > 0 ? 16 * row - 1 : -1;
        } else if (ctrl == 0x143) {
            from = row >= 2 ? 31 : -1;
        } else {
            abort();  // a form the emulation does not model
        }
        res = from >= 0 ? g_wg->dpp[w][from] : (bound_ctrl ? 0 : old);
    }
    g_wg->wbar[w]->arrive_and_wait();
    return res;
}
inline int __popc(uint32_t v) { return __builtin_popcount(v); }
inline int __popcll(uint64_t v) { return __builtin_popcountll(v); }
inline int __clzll(uint64_t v) { return __builtin_clzll(v); }
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_fence(a, b) std::atomic_thread_fence(std::memory_order_seq_cst)
// A waiting thread gives its CPU away for a while: with thousands of emulated
// threads on a few host cores, a bare yield would let a wait reach the
// kernel's spin limit before the awaited workgroup has been scheduled.
#define __builtin_amdgcn_s_sleep(x) std::this_thread::sleep_for(std::chrono::microseconds(20))
#define __HIP_MEMORY_SCOPE_AGENT 0
template <class T> inline T __hip_atomic_load(T *p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T> inline void __hip_atomic_store(T *p, T v, int, int) { __atomic_store_n(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T __hip_atomic_fetch_add(T *p, T v, int, int) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicOr(uint32_t *p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T min(T a, T b) { return a < b ? a : b; }
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace ckey {
constexpr int kWG = 256;
#define CKEY_TRY(expr)                \
    do {                              \
        ckey_status s_ = (expr);      \
        if (s_ != CKEY_OK) return s_; \
    } while (0)
#define CKEY_HIP_TRY(expr)                   \
    do {                                     \
        if ((expr) != 0) return CKEY_ERR_HIP; \
    } while (0)
inline ckey_status launch_status() { return CKEY_OK; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
struct KeySrc {
    const uint8_t *bytes;
    const uint64_t *offsets;
    uint64_t n;
    uint32_t L;
    uint32_t stride;
};
inline uint32_t key_word_bytes(const uint8_t *p, uint32_t j, uint32_t len) {
    uint32_t v = 0;
    for (int t = 0; t < 4; ++t) {
        const uint32_t q = 4 * j + t;
        v = (v << 8) | (q < len ? uint32_t(p[q]) : 0u);
    }
    return v;
}
inline uint32_t key_word_aligned(const uint8_t *p, uint32_t j, uint32_t len) {
    uint32_t w;
    memcpy(&w, p + 4 * j, 4);
    uint32_t v = __builtin_bswap32(w);
    const uint32_t have = len - 4 * j;
    if (have < 4) v &= ~(0xFFFFFFFFu >> (8 * have));
    return v;
}
inline uint32_t bitmap_word_bit(uint32_t p) { return 1u << (8 * ((p >> 3) & 3) + (7 - (p & 7))); }
inline ckey_status fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t) {
    for (uint64_t i = 0; i < n; ++i) p[i] = v;
    return CKEY_OK;
}
inline int prof_begin(hipStream_t, const char *) { return -1; }
inline void prof_end(hipStream_t, int) {}
struct TableIndex {
    KeySrc keys;
    const uint8_t *bitmap;
    uint32_t digit_bits;
    uint32_t *perm;
    uint64_t *ckeys_out;
    uint32_t *pair_pos;
    uint8_t *bitmap_out;
    uint32_t *flags;
};
ckey_status table_fused_plan(const TableIndex *ti, uint32_t count, void *ws, size_t *need, hipStream_t st);
}  // namespace ckey

// The kernel's own wave and workgroup scans (DPP moves modelled above).
#include "scan.h"

inline int hipGetDevice(int *d) {
    *d = 0;
    return 0;
}
inline int hipDeviceGetAttribute(int *v, int, int) {
    *v = 1;
    return 0;
}
template <class F> inline int hipOccupancyMaxActiveBlocksPerMultiprocessor(int *v, F, int, int) {
    *v = 1;
    return 0;
}
// g_nwg concurrent workgroups of 256 threads, whatever the requested grid;
// each thread a pthread with a small stack, so that many workgroups fit.
struct EmuThreadArg {
    std::function<void()> body;
};
inline void *emu_thread_main(void *p) {
    static_cast<EmuThreadArg *>(p)->body();
    return nullptr;
}
#define hipLaunchKernelGGL(K, G, B, S, ST, ...)                                                   \
    do {                                                                                           \
        std::vector<EmuWG *> wgs_;                                                                 \
        for (int w_ = 0; w_ < g_nwg; ++w_) {                                                       \
            EmuWG *e_ = new EmuWG();                                                               \
            e_->bar = new std::barrier<>(256);                                                     \
            for (int q_ = 0; q_ < 4; ++q_) e_->wbar[q_] = new std::barrier<>(64);                  \
            e_->lds[0] = malloc(8 * 4096);                                                         \
            e_->lds[1] = malloc(sizeof(TShared));                                                  \
            e_->lds[2] = malloc(16);                                                               \
            e_->lds[3] = malloc(16);                                                               \
            wgs_.push_back(e_);                                                                    \
        }                                                                                          \
        std::vector<EmuThreadArg> args_(size_t(g_nwg) * 256);                                     \
        std::vector<pthread_t> th_(args_.size());                                                  \
        pthread_attr_t at_;                                                                        \
        pthread_attr_init(&at_);                                                                   \
        pthread_attr_setstacksize(&at_, 1u << 20);                                                 \
        for (int w_ = 0; w_ < g_nwg; ++w_)                                                         \
            for (unsigned t_ = 0; t_ < 256; ++t_) {                                                \
                EmuThreadArg &a_ = args_[size_t(w_) * 256 + t_];                                   \
                a_.body = [&, t_, w_]() {                                                          \
                    threadIdx.x = t_;                                                              \
                    g_wg = wgs_[w_];                                                               \
                    K(__VA_ARGS__);                                                                \
                };                                                                                 \
                if (pthread_create(&th_[size_t(w_) * 256 + t_], &at_, emu_thread_main, &a_) != 0) \
                    abort();                                                                       \
            }                                                                                      \
        for (pthread_t &h_ : th_) pthread_join(h_, nullptr);                                       \
        pthread_attr_destroy(&at_);                                                                \
        for (EmuWG *e_ : wgs_) {                                                                   \
            for (int q_ = 0; q_ < 4; ++q_) { free(e_->lds[q_]); delete e_->wbar[q_]; }             \
            delete e_->bar;                                                                        \
            delete e_;                                                                             \
        }                                                                                          \
    } while (0)
