// Host-side baseline: the paper's own CPU pipeline for a rebuild -- key
// compression with 8-byte masks and PEXT (Sec. 5.1) and the row-column sort
// (Appendix A), a parallel comparison sort of (compressed key, record ID)
// sort keys -- run on the host cores to set beside the GPU path.  It is not
// part of the GPU library and nothing in the GPU library calls it.
//
// Row-column sort, as Appendix A describes it: with p threads, element size e
// and C bytes of last-level cache per thread, c = floor(C/e) and
// t = max(floor(sqrt(n/c)/p), 1).  The n elements form tp init blocks, each
// cut into sub-blocks of c elements.  (1) Each thread takes t init blocks:
// sorts each sub-block with the basic sort (quicksort around the pseudo-median
// of nine, insertion sort below a small size) and merges a block's sub-blocks
// with a tournament tree into a sorted block (second array).  (2) Thread i
// computes the i*n/p-split of the tp sorted blocks (how many elements of each
// block are among the i*n/p smallest), which together form the perfect
// p-partition.  (3) Thread i merges the i-th parts of all sorted blocks with a
// tournament tree into the i-th final block (first array).
//
// Beside it, the GCC parallel-mode sort (__gnu_parallel::sort, OpenMP) of the
// same (compressed key, record ID) records, and of (full key, record ID) by
// memcmp: the library sort the paper sets its row-column sort against.
#include <stdint.h>
#include <string.h>

#include <omp.h>

#include <algorithm>
#include <chrono>
#include <parallel/algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace {

template <int W>
struct Elem {
    uint64_t k[W];
    uint64_t rid;
};

template <int W>
inline bool less(const Elem<W> &a, const Elem<W> &b) {
    for (int w = 0; w < W; ++w)
        if (a.k[w] != b.k[w]) return a.k[w] < b.k[w];
    return a.rid < b.rid;
}

// ---------------------------------------------------------------- basic sort --

template <int W>
void insertion_sort(Elem<W> *a, size_t n) {
    for (size_t i = 1; i < n; ++i) {
        Elem<W> v = a[i];
        size_t j = i;
        while (j > 0 && less(v, a[j - 1])) {
            a[j] = a[j - 1];
            --j;
        }
        a[j] = v;
    }
}

template <int W>
size_t med3(const Elem<W> *a, size_t i, size_t j, size_t k) {
    return less(a[i], a[j]) ? (less(a[j], a[k]) ? j : (less(a[i], a[k]) ? k : i))
                            : (less(a[k], a[j]) ? j : (less(a[k], a[i]) ? k : i));
}

// Quicksort; the pivot is the median of the medians of three samples of three
// (Bentley and McIlroy's pseudo-median of nine) on large ranges.
template <int W>
void basic_sort(Elem<W> *a, size_t n) {
    while (n > 24) {
        size_t m;
        if (n > 40) {
            const size_t s = n / 8;
            const size_t x = med3(a, 0, s, 2 * s);
            const size_t y = med3(a, n / 2 - s, n / 2, n / 2 + s);
            const size_t z = med3(a, n - 1 - 2 * s, n - 1 - s, n - 1);
            m = med3(a, x, y, z);
        } else {
            m = med3(a, 0, n / 2, n - 1);
        }
        const Elem<W> piv = a[m];
        // Hoare partition around the pivot value
        size_t i = 0, j = n - 1;
        for (;;) {
            while (less(a[i], piv)) ++i;
            while (less(piv, a[j])) --j;
            if (i >= j) break;
            std::swap(a[i], a[j]);
            ++i;
            --j;
        }
        const size_t left = j + 1;  // [0, left) <= pivot <= [left, n)
        if (left < n - left) {
            basic_sort(a, left);
            a += left;
            n -= left;
        } else {
            basic_sort(a + left, n - left);
            n = left;
        }
    }
    insertion_sort(a, n);
}

// ------------------------------------------------------------ multiway merge --

struct Run {
    size_t b, e;  // [b, e) of the source array
};

// Tournament (winner) tree over k runs: node v holds the run that wins its
// subtree; popping the overall winner replays the path from its leaf.
template <int W>
void multiway_merge(const Elem<W> *src, const std::vector<Run> &runs, Elem<W> *out) {
    const size_t k = runs.size();
    if (k == 0) return;
    size_t cap = 1;
    while (cap < k) cap <<= 1;
    std::vector<Run> r(runs);
    std::vector<int64_t> tree(2 * cap, -1);  // -1: empty
    auto better = [&](int64_t x, int64_t y) -> int64_t {
        if (x < 0 || r[x].b >= r[x].e) return y;
        if (y < 0 || r[y].b >= r[y].e) return x;
        return less(src[r[y].b], src[r[x].b]) ? y : x;  // ties cannot occur (unique rids)
    };
    for (size_t i = 0; i < cap; ++i) tree[cap + i] = i < k ? int64_t(i) : -1;
    for (size_t v = cap - 1; v >= 1; --v) tree[v] = better(tree[2 * v], tree[2 * v + 1]);
    size_t o = 0;
    for (;;) {
        const int64_t w = tree[1];
        if (w < 0 || r[w].b >= r[w].e) break;
        out[o++] = src[r[w].b++];
        for (size_t v = (cap + size_t(w)) >> 1; v >= 1; v >>= 1) tree[v] = better(tree[2 * v], tree[2 * v + 1]);
    }
}

// ------------------------------------------------------------------ x-split --

// Number of elements of sorted block [b, e) that are less than v.
template <int W>
size_t count_less(const Elem<W> *a, const Run &blk, const Elem<W> &v) {
    size_t lo = blk.b, hi = blk.e;
    while (lo < hi) {
        const size_t mid = lo + (hi - lo) / 2;
        if (less(a[mid], v)) lo = mid + 1; else hi = mid;
    }
    return lo - blk.b;
}

// The x-split of sorted blocks: cut[i] = how many elements of block i are
// among the x smallest of all blocks.  Elements are distinct (the record ID is
// part of the sort key), so element v is among them iff fewer than x elements
// are less than v; within a block that holds for a prefix, found by binary
// search.
template <int W>
void x_split(const Elem<W> *a, const std::vector<Run> &blocks, size_t x, std::vector<size_t> &cut) {
    cut.assign(blocks.size(), 0);
    for (size_t i = 0; i < blocks.size(); ++i) {
        size_t lo = 0, hi = blocks[i].e - blocks[i].b;  // answer in [lo, hi]
        while (lo < hi) {
            const size_t mid = lo + (hi - lo + 1) / 2;  // is element mid-1 among the x smallest?
            const Elem<W> &v = a[blocks[i].b + mid - 1];
            size_t rank = 0;
            for (size_t m = 0; m < blocks.size() && rank < x; ++m) rank += count_less(a, blocks[m], v);
            if (rank < x) lo = mid; else hi = mid - 1;
        }
        cut[i] = lo;
    }
}

template <typename F>
void parallel(int p, F f) {
    std::vector<std::thread> th;
    for (int i = 1; i < p; ++i) th.emplace_back(f, i);
    f(0);
    for (auto &t : th) t.join();
}

template <int W>
void row_column_sort(Elem<W> *key, Elem<W> *temp, size_t n, int p, uint64_t cache_bytes, double *t_phase) {
    using clk = std::chrono::steady_clock;
    if (n < 2) return;
    const size_t e = sizeof(Elem<W>);
    const size_t c = std::max<size_t>(1, size_t(cache_bytes / e));
    const size_t t = std::max<size_t>(1, size_t(std::floor(std::sqrt(double(n) / double(c)) / p)));
    const size_t nb = t * size_t(p);  // init blocks
    std::vector<Run> blocks(nb);
    for (size_t i = 0; i < nb; ++i) blocks[i] = Run{n * i / nb, n * (i + 1) / nb};
    auto t0 = clk::now();
    parallel(p, [&](int th) {
        for (size_t j = 0; j < t; ++j) {
            const Run B = blocks[size_t(th) * t + j];
            std::vector<Run> subs;
            for (size_t s = B.b; s < B.e; s += c) {
                const size_t se = std::min(B.e, s + c);
                basic_sort(key + s, se - s);
                subs.push_back(Run{s, se});
            }
            multiway_merge(key, subs, temp + B.b);
        }
    });
    auto t1 = clk::now();
    std::vector<std::vector<size_t>> cuts(size_t(p) + 1);
    cuts[0].assign(nb, 0);
    cuts[size_t(p)].resize(nb);
    for (size_t i = 0; i < nb; ++i) cuts[size_t(p)][i] = blocks[i].e - blocks[i].b;
    parallel(p, [&](int th) {
        if (th >= 1) x_split(temp, blocks, n * size_t(th) / size_t(p), cuts[size_t(th)]);
    });
    auto t2 = clk::now();
    parallel(p, [&](int th) {
        std::vector<Run> parts(nb);
        for (size_t i = 0; i < nb; ++i)
            parts[i] = Run{blocks[i].b + cuts[size_t(th)][i], blocks[i].b + cuts[size_t(th) + 1][i]};
        multiway_merge(temp, parts, key + n * size_t(th) / size_t(p));
    });
    auto t3 = clk::now();
    if (t_phase) {
        t_phase[0] = std::chrono::duration<double>(t1 - t0).count();
        t_phase[1] = std::chrono::duration<double>(t2 - t1).count();
        t_phase[2] = std::chrono::duration<double>(t3 - t2).count();
    }
}

// ------------------------------------------------------------- compression --

// 8-byte masks of the bitmap (Sec. 5.1): each starts at the byte holding the
// next 1 not covered by the previous mask.
struct Window {
    uint32_t start;
    uint64_t mask;  // big-endian: byte start is the top byte
    uint32_t pc;
};

std::vector<Window> windows_of(const uint8_t *bm, uint32_t L) {
    std::vector<Window> w;
    uint32_t j = 0;
    while (j < L) {
        if (!bm[j]) { ++j; continue; }
        Window x{j, 0, 0};
        for (uint32_t q = 0; q < 8; ++q) x.mask = (x.mask << 8) | (j + q < L ? bm[j + q] : 0u);
        x.pc = uint32_t(__builtin_popcountll(x.mask));
        w.push_back(x);
        j += 8;
    }
    return w;
}

__attribute__((target("bmi2"))) inline uint64_t pext_hw(uint64_t v, uint64_t m) {
    return __builtin_ia32_pext_di(v, m);
}

inline uint64_t pext_sw(uint64_t v, uint64_t m) {
    uint64_t r = 0, bit = 1;
    for (; m; m &= m - 1, bit <<= 1)
        if (v & m & (~m + 1)) r |= bit;
    return r;
}

template <int W>
void compress_rows(const uint8_t *keys, size_t r0, size_t r1, uint32_t L, uint32_t stride,
                   const std::vector<Window> &win, bool hw, Elem<W> *out) {
    for (size_t i = r0; i < r1; ++i) {
        const uint8_t *k = keys + i * size_t(stride);
        Elem<W> el;
        for (int w = 0; w < W; ++w) el.k[w] = 0;
        el.rid = i;
        uint32_t off = 0;
        for (const Window &x : win) {
            uint8_t b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const uint32_t have = std::min<uint32_t>(8, L - x.start);
            memcpy(b, k + x.start, have);
            uint64_t v = 0;
            for (int q = 0; q < 8; ++q) v = (v << 8) | b[q];
            const uint64_t bits = hw ? pext_hw(v, x.mask) : pext_sw(v, x.mask);
            // append x.pc bits at offset off of the MSB-first string
            const uint32_t kw = off >> 6, o = off & 63u, end = o + x.pc;
            if (end <= 64) {
                el.k[kw] |= bits << (64 - end);
            } else {
                el.k[kw] |= bits >> (end - 64);
                el.k[kw + 1] |= bits << (128 - end);
            }
            off += x.pc;
        }
        out[i] = el;
    }
}

// sorter 0: row-column sort; 1: __gnu_parallel::sort on p OpenMP threads.
template <int W>
int run(const uint8_t *keys, uint64_t n, uint32_t L, uint32_t stride, const uint8_t *bitmap, int p,
        uint64_t cache_bytes, uint32_t *perm, uint64_t *ck_out, double *times, int sorter = 0) {
    using clk = std::chrono::steady_clock;
    std::vector<Elem<W>> key(n), temp(n);
    const std::vector<Window> win = windows_of(bitmap, L);
    const bool hw = __builtin_cpu_supports("bmi2");
    auto t0 = clk::now();
    parallel(p, [&](int th) {
        compress_rows<W>(keys, n * size_t(th) / size_t(p), n * size_t(th + 1) / size_t(p), L, stride, win,
                         hw, key.data());
    });
    auto t1 = clk::now();
    double ph[3] = {0, 0, 0};
    if (sorter == 0) {
        row_column_sort<W>(key.data(), temp.data(), n, p, cache_bytes, ph);
    } else {
        omp_set_num_threads(p);
        __gnu_parallel::sort(key.begin(), key.end(), [](const Elem<W> &a, const Elem<W> &b) { return less<W>(a, b); });
    }
    auto t2 = clk::now();
    for (size_t i = 0; i < n; ++i) {
        perm[i] = uint32_t(key[i].rid);
        if (ck_out)
            for (int w = 0; w < W; ++w) ck_out[size_t(w) * n + i] = key[i].k[w];
    }
    if (times) {
        times[0] = std::chrono::duration<double>(t1 - t0).count();
        times[1] = std::chrono::duration<double>(t2 - t1).count();
        times[2] = ph[0];
        times[3] = ph[1];
        times[4] = ph[2];
    }
    return 0;
}

}  // namespace

extern "C" {

// Compress fixed-width keys (n rows of `stride` bytes, key_bytes L) with
// `bitmap` (L bytes) into words = ceil(|D|/64) u64 per key (1..8), sort the
// (compressed key, record ID) pairs with the row-column sort on p threads and
// cache_bytes of cache per thread.  perm (uint32[n]) receives the record IDs in
// sorted order, ck_out (uint64[words*n], word-major, or NULL) the sorted
// compressed keys; times (or NULL): seconds of compression, sort, and the
// sort's three phases.  Returns 0, or -1 on bad arguments.
int rowcol_compress_sort(const uint8_t *keys, uint64_t n, uint32_t L, uint32_t stride,
                         const uint8_t *bitmap, uint32_t words, int p, uint64_t cache_bytes,
                         uint32_t *perm, uint64_t *ck_out, double *times) {
    if ((!keys && n) || !bitmap || L == 0 || stride < L || p < 1 || (!perm && n)) return -1;
    uint32_t nbits = 0;
    for (uint32_t j = 0; j < L; ++j) nbits += uint32_t(__builtin_popcount(bitmap[j]));
    const uint32_t need = nbits ? (nbits + 63) / 64 : 1;
    if (words != need) return -1;
    switch (words) {
        case 1: return run<1>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 2: return run<2>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 3: return run<3>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 4: return run<4>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 5: return run<5>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 6: return run<6>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 7: return run<7>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        case 8: return run<8>(keys, n, L, stride, bitmap, p, cache_bytes, perm, ck_out, times);
        default: return -1;
    }
}

// The same compression, then __gnu_parallel::sort of the (compressed key,
// record ID) records on p threads; arguments as rowcol_compress_sort (times[2..4]
// are 0).
int gnu_compress_sort(const uint8_t *keys, uint64_t n, uint32_t L, uint32_t stride,
                      const uint8_t *bitmap, uint32_t words, int p, uint32_t *perm, uint64_t *ck_out,
                      double *times) {
    if ((!keys && n) || !bitmap || L == 0 || stride < L || p < 1 || (!perm && n)) return -1;
    uint32_t nbits = 0;
    for (uint32_t j = 0; j < L; ++j) nbits += uint32_t(__builtin_popcount(bitmap[j]));
    const uint32_t need = nbits ? (nbits + 63) / 64 : 1;
    if (words != need) return -1;
    switch (words) {
        case 1: return run<1>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 2: return run<2>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 3: return run<3>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 4: return run<4>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 5: return run<5>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 6: return run<6>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 7: return run<7>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        case 8: return run<8>(keys, n, L, stride, bitmap, p, 0, perm, ck_out, times, 1);
        default: return -1;
    }
}

// __gnu_parallel::sort of the full keys: record IDs ordered by memcmp of the
// L key bytes, ties by record ID, on p threads.  perm (uint32[n]) receives
// the order; *seconds (or NULL) the sort time.  Returns 0, or -1 on bad
// arguments.
int gnu_full_sort(const uint8_t *keys, uint64_t n, uint32_t L, uint32_t stride, int p, uint32_t *perm,
                  double *seconds) {
    if ((!keys && n) || L == 0 || stride < L || p < 1 || (!perm && n)) return -1;
    for (uint64_t i = 0; i < n; ++i) perm[i] = uint32_t(i);
    auto t0 = std::chrono::steady_clock::now();
    omp_set_num_threads(p);
    __gnu_parallel::sort(perm, perm + n, [&](uint32_t a, uint32_t b) {
        const int c = memcmp(keys + size_t(a) * stride, keys + size_t(b) * stride, L);
        return c < 0 || (c == 0 && a < b);
    });
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

}  // extern "C"
