// Host stand-ins for the HIP definitions bucket.h uses, so that its device
// search functions can be compiled with g++ and checked on the CPU: one
// thread (threadIdx.x = 0, blockDim.x = 1) runs every cooperative loop whole.
#pragma once
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <cstddef>

#include "ckey.h"

#define __device__
#define __host__
#define __forceinline__ inline
typedef void *hipStream_t;

struct EmuDim {
    unsigned x;
};
static const EmuDim threadIdx{0}, blockDim{1};
inline int __clz(int v) { return v == 0 ? 32 : __builtin_clz(uint32_t(v)); }
inline int __ffs(uint32_t v) { return __builtin_ffs(int(v)); }  // 1 + index of the lowest set bit, 0 for 0
inline uint32_t atomicAdd(uint32_t *p, uint32_t v) {
    const uint32_t o = *p;
    *p = o + v;
    return o;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
    const unsigned long long o = *p;
    *p = o + v;
    return o;
}
template <class T> inline T min(T a, T b) { return a < b ? a : b; }

namespace ckey {
struct KeySrc {
    const uint8_t *bytes;
    const uint64_t *offsets;
    uint64_t n;
    uint32_t L;
    uint32_t stride;
};
}  // namespace ckey
