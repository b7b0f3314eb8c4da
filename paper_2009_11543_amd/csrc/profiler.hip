// Per-kernel timing with HIP events (benchmark support) and a plain copy
// kernel used to measure achievable HBM bandwidth and to calibrate hardware
// byte counters.
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace ckey {

namespace {

struct Rec {
    const char *name;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

__global__ void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n16) {
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += step)
        dst[i] = src[i];
}

}  // namespace

int prof_begin(hipStream_t st, const char *name) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_on) return -1;
    Rec r{name, take_event(), take_event()};
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, st);
    g_recs.push_back(r);
    return int(g_recs.size()) - 1;
}

void prof_end(hipStream_t st, int idx) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> g(g_mu);
    if (idx < int(g_recs.size())) (void)hipEventRecord(g_recs[idx].b, st);
}

}  // namespace ckey

using namespace ckey;

extern "C" {

ckey_status ckey_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_on = on != 0;
    return CKEY_OK;
}

ckey_status ckey_profile_read(const char *name, double *total_ms, uint64_t *launches) {
    std::lock_guard<std::mutex> g(g_mu);
    double t = 0;
    uint64_t c = 0;
    for (const Rec &r : g_recs) {
        if (name && std::string(name) != r.name) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return CKEY_ERR_HIP;
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return CKEY_ERR_HIP;
        t += ms;
        ++c;
    }
    if (total_ms) *total_ms = t;
    if (launches) *launches = c;
    return CKEY_OK;
}

ckey_status ckey_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_mu);
    for (const Rec &r : g_recs) {
        (void)hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    return CKEY_OK;
}

ckey_status ckey_bench_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (bytes == 0) return CKEY_OK;
    if (!dst || !src || bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 ||
        reinterpret_cast<uintptr_t>(src) % 16)
        return CKEY_ERR_INVALID;
    const uint64_t n16 = bytes / 16;
    uint64_t blocks = (n16 + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int p = prof_begin(st, "stream_copy");
    hipLaunchKernelGGL(k_stream_copy, dim3(uint32_t(blocks)), dim3(kWG), 0, st,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
    prof_end(st, p);
    return launch_status();
}

}  // extern "C"
