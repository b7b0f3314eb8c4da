// Driver of the host build of bucket.h's search functions.  Reads from a
// directory written by the CPU test: m.txt = "B S nx", T.bin (uint64[B]),
// x.bin (uint64[nx]), g.bin (uint32[nx] start guesses), p.bin (float MLP
// parameters); writes one uint32[nx] file per search form, the network's
// guesses both ways, and the bucket histogram.
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "bucket.h"

using namespace ckey;

template <class T> static std::vector<T> rd(const std::string &p) {
    std::ifstream f(p, std::ios::binary);
    std::vector<char> c((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    std::vector<T> v(c.size() / sizeof(T));
    if (!v.empty()) memcpy(v.data(), c.data(), v.size() * sizeof(T));
    return v;
}
template <class T> static void wr(const std::string &p, const std::vector<T> &v) {
    std::ofstream f(p, std::ios::binary);
    f.write(reinterpret_cast<const char *>(v.data()), std::streamsize(v.size() * sizeof(T)));
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const std::string d = argv[1];
    uint32_t B, S;
    size_t nx;
    std::ifstream(d + "/m.txt") >> B >> S >> nx;
    const std::vector<uint64_t> T = rd<uint64_t>(d + "/T.bin");
    const std::vector<uint64_t> x = rd<uint64_t>(d + "/x.bin");
    const std::vector<uint32_t> g = rd<uint32_t>(d + "/g.bin");
    const std::vector<float> p = rd<float>(d + "/p.bin");
    if (T.size() != B || x.size() != nx || g.size() != nx) return 3;
    std::vector<uint32_t> hist(B, 0);
    BucketArgs a{p.data(), T.data(), B, S, nullptr, nullptr, nullptr, hist.data()};
    // Splitter: the LDS image the kernels build (bucket_lds_bytes of it).
    // Exactly the LDS the kernels allocate, so that the sanitizer sees any
    // access beyond it; stale contents stand for uninitialised LDS.
    std::vector<uint32_t> s0(bucket_lds_bytes(a, 0) / 4, 0xDEADBEEFu);
    std::vector<uint32_t> s1(bucket_lds_bytes(a, 1) / 4, 0xDEADBEEFu);
    bucket_lds_init<0>(a, s0.data());
    bucket_lds_init<1>(a, s1.data());
    std::vector<uint32_t> one(nx), many(nx), lcorr(nx), lwin(nx), lmany(nx), pr1(nx), pr4(nx);
    for (size_t i = 0; i < nx; ++i) {
        uint32_t probes = 0, guess = 0;
        one[i] = bucket_of<0>(a, s0.data(), x[i], probes, guess);
        const uint64_t *th = S == 1 ? reinterpret_cast<const uint64_t *>(s1.data()) : T.data();
        lcorr[i] = correct_bucket(th, B, x[i], g[i], probes);
        lwin[i] = correct_bucket_window<512>(th, B, x[i], g[i]);
        pr1[i] = predict_bucket(p.data(), x[i], B);
        bucket_record<0>(a, s0.data(), one[i], i);
        // Every 500 keys a flush as if 65530 more keys were to come: counters
        // above 5 go to the global histogram, the others stay in LDS.
        if ((i + 1) % 500 == 0) bucket_lds_flush_before<0>(a, s0.data(), 65530u);
    }
    for (size_t i = 0; i < nx; i += 8) {
        uint64_t xs[8];
        uint32_t b[8];
        for (int q = 0; q < 8; ++q) xs[q] = i + q < nx ? x[i + q] : 0;
        if (S == 1)
            splitter_search_n<8>(a, s0.data(), xs, b);
        else
            splitter_search_sampled_n<8>(a, s0.data(), xs, b);
        for (int q = 0; q < 8 && i + q < nx; ++q) many[i + q] = b[q];
    }
    for (size_t i = 0; i < nx; i += 4) {  // the learned correction of four keys at once, T in memory
        uint64_t xs[4];
        uint32_t gs[4], b[4];
        for (int q = 0; q < 4; ++q) {
            xs[q] = i + q < nx ? x[i + q] : 0;
            gs[q] = i + q < nx ? g[i + q] : 0;
        }
        correct_bucket_n<4>(T.data(), B, xs, gs, b);
        for (int q = 0; q < 4 && i + q < nx; ++q) lmany[i + q] = b[q];
    }
    for (size_t i = 0; i < nx; i += 4) {
        uint64_t xs[4];
        uint32_t gq[4];
        for (int q = 0; q < 4; ++q) xs[q] = i + q < nx ? x[i + q] : 0;
        predict_bucket_n<4>(p.data(), xs, B, gq);
        for (int q = 0; q < 4 && i + q < nx; ++q) pr4[i + q] = gq[q];
    }
    bucket_lds_flush_before<0>(a, s0.data(), 0u);  // the last: every pair
    wr(d + "/one.bin", one);
    wr(d + "/many.bin", many);
    wr(d + "/lcorr.bin", lcorr);
    wr(d + "/lwin.bin", lwin);
    wr(d + "/lmany.bin", lmany);
    wr(d + "/pr1.bin", pr1);
    wr(d + "/pr4.bin", pr4);
    wr(d + "/hist.bin", hist);
    return 0;
}
