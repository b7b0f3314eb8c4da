// Host-side baseline: the paper's own CPU pipeline for a rebuild -- key
// compression with 8-byte masks and PEXT (Sec. 5.1) and the row-column sort
// (Appendix A), a parallel comparison sort of (compressed key, record ID)
// sort keys -- run on the host cores to set beside the GPU path.  It is not
// part of the GPU library and nothing in the GPU library calls it.
//
// What the row-column sort computes (Appendix A): the elements are cut into
// t*p equal segments for p threads, t chosen so that a segment holds about
// t*p runs of cache size (c elements, c*e bytes = the cache per thread).
// Every run is sorted in cache by a quicksort, each segment's runs are merged
// by a tournament into a sorted segment, the sorted segments are split at the
// ranks n*i/p (the "perfect partition": piece i of every segment holds
// exactly the elements of global rank [n*i/p, n*(i+1)/p)), and thread i
// merges the i-th pieces of all segments into its slice of the output.
//
// How it is built here: an iterative quicksort (explicit stack, pivot = a
// median of three medians of three on large ranges, insertion sort on short
// ones); a loser tree for every multi-way merge; and the split ranks found by
// a multi-sequence selection that keeps, per segment, a window [lo, hi) known
// to contain the cut, takes the middle element of the widest window as a
// pivot, counts its global rank with one binary search per segment, and
// shrinks every window to one side of the pivot's position until all windows
// are empty.
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

// ----------------------------------------------------------------- run sort --

template <int W>
void insertion_sort(Elem<W> *a, size_t n) {
    for (size_t i = 1; i < n; ++i) {
        if (!less(a[i], a[i - 1])) continue;
        Elem<W> v = a[i];
        size_t j = i;
        do {
            a[j] = a[j - 1];
        } while (--j > 0 && less(v, a[j - 1]));
        a[j] = v;
    }
}

// Middle one of a[x], a[y], a[z] (distinct elements: record IDs differ).
template <int W>
const Elem<W> &mid3(const Elem<W> *a, size_t x, size_t y, size_t z) {
    const bool xy = less(a[x], a[y]), yz = less(a[y], a[z]), xz = less(a[x], a[z]);
    if (xy == yz) return a[y];   // x < y < z or z < y < x
    return xy == xz ? a[z] : a[x];
}

// Quicksort of one cache-sized run without recursion: the larger side of
// every partition goes on a small explicit stack, the smaller is sorted next,
// so the stack never holds more than log2(n) ranges.
template <int W>
void run_sort(Elem<W> *a, size_t n) {
    struct Range { size_t b, n; };
    Range stack[64];
    int top = 0;
    stack[top++] = Range{0, n};
    while (top) {
        Range r = stack[--top];
        while (r.n > 16) {
            Elem<W> *x = a + r.b;
            const size_t m = r.n;
            Elem<W> piv;
            if (m >= 64) {
                const size_t q = m / 8, h = m / 2;
                const Elem<W> lo = mid3(x, 0, q, 2 * q), md = mid3(x, h - q, h, h + q),
                              hi = mid3(x, m - 1 - 2 * q, m - 1 - q, m - 1);
                const Elem<W> three[3] = {lo, md, hi};
                piv = mid3(three, 0, 1, 2);
            } else {
                piv = mid3(x, 0, m / 2, m - 1);
            }
            // Two cursors meet: left of i nothing exceeds the pivot, right of
            // j nothing is below it; the pivot itself stops both scans.
            size_t i = 0, j = m - 1;
            for (;;) {
                while (less(x[i], piv)) ++i;
                while (less(piv, x[j])) --j;
                if (i >= j) break;
                std::swap(x[i++], x[j--]);
            }
            const size_t left = j + 1;
            Range small{r.b, left}, large{r.b + left, m - left};
            if (small.n > large.n) std::swap(small, large);
            stack[top++] = large;
            r = small;
        }
        insertion_sort(a + r.b, r.n);
    }
}

// ---------------------------------------------------------------- loser tree --

struct Seq {
    size_t b, e;  // [b, e) of the source array
};

// k-way merge by a loser tree: each inner node keeps the sequence that lost
// the match played there, node 0 the overall winner; after the winner's head
// is output only the matches on its leaf-to-root path are replayed.
template <int W>
void loser_merge(const Elem<W> *src, const std::vector<Seq> &in, Elem<W> *out) {
    const size_t k = in.size();
    if (k == 0) return;
    if (k == 1) {
        std::copy(src + in[0].b, src + in[0].e, out);
        return;
    }
    std::vector<Seq> q(in);
    // an exhausted sequence loses every match
    auto beats = [&](size_t u, size_t v) {
        if (q[u].b == q[u].e) return false;
        if (q[v].b == q[v].e) return true;
        return less(src[q[u].b], src[q[v].b]);
    };
    std::vector<size_t> node(k);   // node[1..k-1]: losers; node[0]: winner
    // Build bottom-up: leaves are k + s for sequence s; play every inner match.
    std::vector<size_t> win(2 * k);
    for (size_t s = 0; s < k; ++s) win[k + s] = s;
    for (size_t v = k - 1; v >= 1; --v) {
        const size_t a = win[2 * v], b = win[2 * v + 1];
        const bool ab = beats(a, b);
        win[v] = ab ? a : b;
        node[v] = ab ? b : a;
    }
    node[0] = win[1];
    size_t o = 0;
    for (;;) {
        size_t w = node[0];
        if (q[w].b == q[w].e) break;  // the winner is empty: every sequence is
        out[o++] = src[q[w].b++];
        for (size_t v = (k + w) >> 1; v >= 1; v >>= 1) {
            if (beats(node[v], w)) std::swap(node[v], w);
        }
        node[0] = w;
    }
}

// ---------------------------------------------------------- perfect partition --

// Elements of sorted sequence s below v.
template <int W>
size_t rank_in(const Elem<W> *a, const Seq &s, const Elem<W> &v) {
    return size_t(std::lower_bound(a + s.b, a + s.e, v, less<W>) - (a + s.b));
}

// Multi-sequence selection: cut[i] = how many elements of sorted sequence i
// have global rank below x (elements are distinct).  Window [lo[i], hi[i])
// of sequence i holds the positions not yet known to be below or above the
// cut; a pivot from the widest window settles at least half of it.
template <int W>
void select_cut(const Elem<W> *a, const std::vector<Seq> &seqs, size_t x, std::vector<size_t> &cut) {
    const size_t k = seqs.size();
    std::vector<size_t> lo(k, 0), hi(k), pos(k);
    for (size_t i = 0; i < k; ++i) hi[i] = seqs[i].e - seqs[i].b;
    for (;;) {
        size_t wi = k, width = 0;
        for (size_t i = 0; i < k; ++i)
            if (hi[i] - lo[i] > width) { width = hi[i] - lo[i]; wi = i; }
        if (wi == k) break;
        const Elem<W> &v = a[seqs[wi].b + lo[wi] + width / 2];
        size_t r = 0;  // global rank of v
        for (size_t i = 0; i < k; ++i) { pos[i] = rank_in(a, seqs[i], v); r += pos[i]; }
        if (r < x) {         // v and everything below it is under the cut
            for (size_t i = 0; i < k; ++i) lo[i] = std::max(lo[i], pos[i] + (i == wi ? 1 : 0));
        } else {             // v and everything above it is over the cut
            for (size_t i = 0; i < k; ++i) hi[i] = std::min(hi[i], pos[i]);
        }
        for (size_t i = 0; i < k; ++i) hi[i] = std::max(hi[i], lo[i]);
    }
    cut = lo;
}

template <typename F>
void parallel(int p, F f) {
    std::vector<std::thread> th;
    for (int i = 1; i < p; ++i) th.emplace_back(f, i);
    f(0);
    for (auto &t : th) t.join();
}

// Row-column sort (Appendix A) of key[0, n) using temp[0, n); the result is
// back in key.  t_phase (or NULL): seconds of the segment sorts, the
// partition and the final merges.
template <int W>
void row_column_sort(Elem<W> *key, Elem<W> *temp, size_t n, int p, uint64_t cache_bytes, double *t_phase) {
    using clk = std::chrono::steady_clock;
    if (n < 2) return;
    const size_t P = size_t(p);
    const size_t c = std::max<size_t>(1, size_t(cache_bytes / sizeof(Elem<W>)));  // elements per run
    // segments per thread: a segment of n/(t p) elements holds n/(t p c) runs,
    // which balances the segment merge (runs per segment) against the final
    // merge (t p segments) when n/(t p c) = t p
    const size_t t = std::max<size_t>(1, size_t(std::sqrt(double(n) / double(c)) / double(P)));
    const size_t nseg = t * P;
    auto seg = [&](size_t s) { return Seq{n * s / nseg, n * (s + 1) / nseg}; };
    auto t0 = clk::now();
    parallel(p, [&](int th) {
        for (size_t s = size_t(th); s < nseg; s += P) {  // thread th: segments th, th + p, ...
            const Seq S = seg(s);
            std::vector<Seq> runs;
            for (size_t b = S.b; b < S.e; b += c) {
                const size_t e = std::min(S.e, b + c);
                run_sort(key + b, e - b);
                runs.push_back(Seq{b, e});
            }
            loser_merge(key, runs, temp + S.b);
        }
    });
    auto t1 = clk::now();
    std::vector<Seq> segs(nseg);
    for (size_t s = 0; s < nseg; ++s) segs[s] = seg(s);
    std::vector<std::vector<size_t>> cut(P + 1);
    cut[0].assign(nseg, 0);
    cut[P].resize(nseg);
    for (size_t s = 0; s < nseg; ++s) cut[P][s] = segs[s].e - segs[s].b;
    parallel(p, [&](int th) {
        if (th > 0) select_cut(temp, segs, n * size_t(th) / P, cut[size_t(th)]);
    });
    auto t2 = clk::now();
    parallel(p, [&](int th) {
        std::vector<Seq> piece(nseg);
        for (size_t s = 0; s < nseg; ++s)
            piece[s] = Seq{segs[s].b + cut[size_t(th)][s], segs[s].b + cut[size_t(th) + 1][s]};
        loser_merge(temp, piece, key + n * size_t(th) / P);
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
