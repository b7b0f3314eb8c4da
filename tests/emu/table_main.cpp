// Driver of the host emulation of the table-rebuild kernel: reads a table
// written by the CPU test (per index: m<i>.txt = "n L stride has_bitmap
// digit_bits has_offsets words", r<i>.bin rows, o<i>.bin offsets, b<i>.bin
// bitmap), runs table_fused_plan with g_nwg concurrent workgroups, and writes
// perm<i>.bin, bmo<i>.bin, pp<i>.bin, ck<i>.bin and flags<i>.txt.
#include <fstream>
#include <iterator>
#include <string>

#include "table_host.h"

thread_local EmuTid threadIdx;
thread_local EmuWG *g_wg;
int g_nwg = 1;

static std::vector<uint8_t> rd(const std::string &p) {
    std::ifstream f(p, std::ios::binary);
    return std::vector<uint8_t>((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
}
static void wr(const std::string &p, const void *d, size_t n) {
    std::ofstream f(p, std::ios::binary);
    f.write(static_cast<const char *>(d), std::streamsize(n));
}

int main(int argc, char **argv) {
    if (argc < 4) return 2;
    const std::string dir = argv[1];
    const int count = atoi(argv[2]);
    g_nwg = atoi(argv[3]);
    const size_t nidx = static_cast<size_t>(count);
    std::vector<ckey::TableIndex> ti(nidx);
    std::vector<std::vector<uint8_t>> bms(nidx);
    std::vector<uint64_t> nn(nidx);
    std::vector<uint32_t> LL(nidx), words(nidx);
    for (int i = 0; i < count; ++i) {
        const std::string s = std::to_string(i);
        std::ifstream m(dir + "/m" + s + ".txt");
        uint64_t n;
        uint32_t L, stride, hasbm, d, hasoff;
        m >> n >> L >> stride >> hasbm >> d >> hasoff >> words[size_t(i)];
        const std::vector<uint8_t> rows = rd(dir + "/r" + s + ".bin");
        uint8_t *keys = static_cast<uint8_t *>(malloc(std::max<size_t>(rows.size(), 1)));
        if (!rows.empty()) memcpy(keys, rows.data(), rows.size());
        uint64_t *offs = nullptr;
        if (hasoff) {
            const std::vector<uint8_t> o = rd(dir + "/o" + s + ".bin");
            offs = static_cast<uint64_t *>(malloc(o.size()));
            memcpy(offs, o.data(), o.size());
        }
        bms[size_t(i)].assign(L, 0xFF);
        if (hasbm) bms[size_t(i)] = rd(dir + "/b" + s + ".bin");
        nn[size_t(i)] = n;
        LL[size_t(i)] = L;
        ckey::TableIndex &t = ti[size_t(i)];
        t.keys = ckey::KeySrc{n ? keys : nullptr, offs, n, L, stride};
        t.bitmap = bms[size_t(i)].data();
        t.digit_bits = d;
        t.perm = n ? static_cast<uint32_t *>(malloc(4 * n)) : nullptr;
        t.ckeys_out = n ? static_cast<uint64_t *>(malloc(8 * n * words[size_t(i)])) : nullptr;
        t.pair_pos = n > 1 ? static_cast<uint32_t *>(malloc(4 * (n - 1))) : nullptr;
        t.bitmap_out = static_cast<uint8_t *>(malloc(L));
        t.flags = static_cast<uint32_t *>(calloc(1, 4));
    }
    size_t need = 0;
    if (ckey::table_fused_plan(ti.data(), uint32_t(count), nullptr, &need, nullptr) != CKEY_OK) return 3;
    void *ws = aligned_alloc(256, (need + 255) & ~size_t(255));
    if (ckey::table_fused_plan(ti.data(), uint32_t(count), ws, &need, nullptr) != CKEY_OK) return 4;
    for (int i = 0; i < count; ++i) {
        const std::string s = std::to_string(i);
        const uint64_t n = nn[size_t(i)];
        const ckey::TableIndex &t = ti[size_t(i)];
        wr(dir + "/perm" + s + ".bin", t.perm, 4 * n);
        wr(dir + "/bmo" + s + ".bin", t.bitmap_out, LL[size_t(i)]);
        if (n > 1) wr(dir + "/pp" + s + ".bin", t.pair_pos, 4 * (n - 1));
        wr(dir + "/ck" + s + ".bin", t.ckeys_out, 8 * n * words[size_t(i)]);
        std::ofstream(dir + "/flags" + s + ".txt") << *t.flags << "\n";
    }
    return 0;
}
