// Checks of the task-graph scheduler (fz_taskgraph.h) on the CPU: the
// stage lists of a compression and a decompression, and random access
// lists against a brute-force happens-before relation.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2509_20563_amd/csrc/fz_taskgraph.h"

using namespace fz;

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);   \
            fails++;                                                  \
        }                                                             \
    } while (0)

// happens-before from the stream order and the cross-stream waits
static std::vector<uint64_t> happens_before(const Schedule& s) {
    const int n = s.n;
    std::vector<uint64_t> hb(n, 0);  // hb[j]: tasks that finish before j starts
    std::vector<int> last(s.nstreams, -1);
    for (int j = 0; j < n; j++) {
        uint64_t h = 0;
        const int prev = last[s.stream[j]];
        if (prev >= 0) h |= (1ull << prev) | hb[prev];
        for (int i : s.deps[j]) {
            CHECK(i < j);
            h |= (1ull << i) | hb[i];
        }
        hb[j] = h;
        last[s.stream[j]] = j;
    }
    return hb;
}

static void check_orders_conflicts(const std::vector<std::vector<Acc>>& acc, const Schedule& s) {
    const int n = (int)acc.size();
    const auto hb = happens_before(s);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < j; i++) {
            bool c = false;
            for (const Acc& a : acc[i])
                for (const Acc& b : acc[j])
                    if (a.data == b.data && acc_conflict(a.mode, b.mode)) c = true;
            if (c) CHECK((hb[j] >> i) & 1);
        }
    // every kept edge joins two conflicting tasks
    for (int j = 0; j < n; j++)
        for (int i : s.deps[j]) {
            bool c = false;
            for (const Acc& a : acc[i])
                for (const Acc& b : acc[j])
                    if (a.data == b.data && acc_conflict(a.mode, b.mode)) c = true;
            CHECK(c);
        }
}

int main() {
    // data identities
    int x, range, flags, codes, tcnt, hist, toff, qctr, out, cw, cb, enc, total, tstart;
    // compression: reset, minmax, quant, scan_counts, codebook, encode, finalize
    std::vector<std::vector<Acc>> comp = {
        {{&range, ACC_W}, {&flags, ACC_W}, {&hist, ACC_W}, {&qctr, ACC_W}, {&cb, ACC_W}, {&enc, ACC_W},
         {&total, ACC_W}},
        {{&x, ACC_R}, {&range, ACC_RED}, {&flags, ACC_RED}},
        {{&x, ACC_R}, {&range, ACC_R}, {&codes, ACC_W}, {&tcnt, ACC_W}, {&hist, ACC_RED}, {&flags, ACC_RED}},
        {{&tcnt, ACC_R}, {&toff, ACC_W}, {&qctr, ACC_RW}, {&flags, ACC_RED}},
        {{&hist, ACC_RW}, {&out, ACC_W}, {&cw, ACC_W}, {&cb, ACC_W}, {&flags, ACC_RED}},
        {{&codes, ACC_R}, {&cw, ACC_R}, {&out, ACC_W}, {&tstart, ACC_W}, {&enc, ACC_W}, {&flags, ACC_RED}},
        {{&range, ACC_R}, {&qctr, ACC_R}, {&cb, ACC_R}, {&enc, ACC_R}, {&flags, ACC_RW}, {&total, ACC_W},
         {&out, ACC_W}, {&tcnt, ACC_R}, {&toff, ACC_R}, {&tstart, ACC_R}, {&x, ACC_R}}};
    Schedule s = schedule_tasks(comp, 4);
    CHECK(s.n == 7);
    // reset -> minmax -> quant -> {scan_counts, codebook -> encode} -> finalize
    CHECK(s.deps[1] == std::vector<int>({0}));
    CHECK(s.deps[2] == std::vector<int>({1}));
    CHECK(s.deps[3] == std::vector<int>({2}));
    CHECK(s.deps[4] == std::vector<int>({2}));
    CHECK(s.deps[5] == std::vector<int>({4}));
    CHECK(s.deps[6] == std::vector<int>({3, 5}));
    CHECK(s.width == 2 && s.nstreams == 2);
    CHECK(s.stream[3] != s.stream[4]);
    // scan_counts continues the quantiser's stream; the code and encoder branch
    // waits for the quantiser, the finaliser for the encoder
    CHECK(s.stream[3] == s.stream[2] && s.signal[2] && s.signal[5] && !s.signal[3] && !s.signal[0]);
    check_orders_conflicts(comp, s);
    // one stream only: a chain
    Schedule s1 = schedule_tasks(comp, 1);
    CHECK(s1.nstreams == 1);
    check_orders_conflicts(comp, s1);

    // decompression: lut, scan, oindex, decode, patch
    int in, lut, off, oidx, ohl, dec, res;
    std::vector<std::vector<Acc>> dcmp = {
        {{&flags, ACC_W}, {&oidx, ACC_W}, {&lut, ACC_W}, {&ohl, ACC_W}, {&dec, ACC_W}, {&in, ACC_R}},
        {{&in, ACC_R}, {&off, ACC_W}, {&flags, ACC_RED}},
        {{&in, ACC_R}, {&oidx, ACC_RW}, {&ohl, ACC_RED}, {&flags, ACC_RED}},
        {{&in, ACC_R}, {&off, ACC_R}, {&lut, ACC_R}, {&oidx, ACC_R}, {&res, ACC_W}, {&dec, ACC_RED},
         {&flags, ACC_RED}},
        {{&in, ACC_R}, {&res, ACC_RW}, {&flags, ACC_RED}}};
    s = schedule_tasks(dcmp, 4);
    CHECK(s.deps[1] == std::vector<int>({0}));
    CHECK(s.deps[2] == std::vector<int>({0}));
    CHECK(s.deps[3] == std::vector<int>({1, 2}));
    CHECK(s.deps[4] == std::vector<int>({3}));
    CHECK(s.width == 2 && s.stream[1] != s.stream[2]);
    check_orders_conflicts(dcmp, s);

    // independent tasks spread over the streams, the rest join stream 0
    std::vector<int> ids(8);
    std::vector<std::vector<Acc>> ind;
    for (int k = 0; k < 8; k++) ind.push_back({{&ids[k], ACC_W}});
    s = schedule_tasks(ind, 4);
    CHECK(s.width == 8 && s.nstreams == 4);
    for (int j = 0; j < 8; j++) CHECK(s.deps[j].empty());
    check_orders_conflicts(ind, s);

    // random access lists
    std::mt19937 rng(12345);
    std::vector<int> data(10);
    for (int trial = 0; trial < 2000; trial++) {
        const int n = 1 + (int)(rng() % 20);
        std::vector<std::vector<Acc>> acc(n);
        for (int j = 0; j < n; j++) {
            const int na = (int)(rng() % 4);
            for (int a = 0; a < na; a++) {
                static const int modes[4] = {ACC_R, ACC_W, ACC_RW, ACC_RED};
                acc[j].push_back({&data[rng() % data.size()], modes[rng() % 4]});
            }
        }
        const int ms = 1 + (int)(rng() % 4);
        Schedule r = schedule_tasks(acc, ms);
        CHECK(r.n == n && r.nstreams <= ms);
        check_orders_conflicts(acc, r);
    }
    std::printf("%d failed checks\n", fails);
    return fails ? 1 : 0;
}
