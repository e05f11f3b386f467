// Replays batch call sequences through the library's C ABI on the host-only
// stub runtime (hip_stub.cpp): compression and decompression batches of
// changing sizes and chain counts, interleaved, with graph replays,
// re-captures, the autotuner and single calls in between.  The stub fails
// the run if any captured node touches memory freed since its capture, if a
// graph is launched after being destroyed, or if a free does not match an
// allocation; the driver checks that replays return the same offsets and
// that everything is released at the end.  Exit status 0 = clean.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/fz.h"

extern "C" int hipstub_errors();
extern "C" size_t hipstub_live_allocations();

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);         \
            fprintf(stderr, "\n");                \
            g_fail++;                             \
        }                                         \
    } while (0)

struct Field {
    fz_params p;
    float* d = nullptr;
};

Field make(uint32_t ndim, uint64_t x, uint64_t y, uint64_t z, double eb, uint32_t mode, uint32_t pred) {
    Field f;
    memset(&f.p, 0, sizeof(f.p));
    f.p.ndim = ndim;
    f.p.dims[0] = x;
    f.p.dims[1] = y;
    f.p.dims[2] = z;
    f.p.eb_mode = mode;
    f.p.eb = eb;
    f.p.pred = pred;
    f.p.radius = 512;
    const uint64_t n = x * y * z;
    hipMalloc((void**)&f.d, 4 * n);
    for (uint64_t i = 0; i < n; i++) f.d[i] = (float)(i % 97) * 0.01f;
    return f;
}

struct Batch {
    std::vector<Field> f;
    std::vector<fz_params> p;
    std::vector<const float*> x;
    uint8_t* out = nullptr;
    uint64_t cap = 0;
    std::vector<uint64_t> offs;
    void finish() {
        for (const Field& a : f) {
            p.push_back(a.p);
            x.push_back(a.d);
        }
        cap = fz_compress_batch_bound((uint32_t)f.size(), p.data());
        hipMalloc((void**)&out, cap);
        offs.assign(f.size() + 1, 0);
    }
    void release() {
        for (Field& a : f) hipFree(a.d);
        hipFree(out);
    }
};

int compress(fz_ctx* c, Batch& b) {
    return fz_compress_batch(c, (uint32_t)b.f.size(), b.p.data(), b.x.data(), b.out, b.cap, b.offs.data(), nullptr);
}

// Decompress a packed batch into freshly allocated outputs (freed after).
int decompress(fz_ctx* c, const uint8_t* packed, const std::vector<uint64_t>& offs, const std::vector<fz_params>& p) {
    const uint32_t n = (uint32_t)p.size();
    std::vector<float*> outs(n);
    std::vector<uint64_t> ne(n);
    for (uint32_t i = 0; i < n; i++) {
        ne[i] = p[i].dims[0] * p[i].dims[1] * p[i].dims[2];
        hipMalloc((void**)&outs[i], 4 * ne[i]);
    }
    int rc = fz_decompress_batch(c, n, packed, offs.data(), outs.data(), ne.data(), nullptr);
    for (float* o : outs) hipFree(o);
    return rc;
}

Batch small_batch() {
    Batch b;
    const uint64_t hw[6][2] = {{40, 30}, {300, 260}, {77, 120}, {256, 31}, {45, 200}, {128, 64}};
    for (auto& s : hw) b.f.push_back(make(2, s[1], s[0], 1, 1e-3, 1, 0));
    b.f.push_back(make(3, 33, 40, 24, 1e-3, 1, 0));
    b.f.push_back(make(1, 5003, 1, 1, 1e-4, 1, 0));
    b.f.push_back(make(3, 13, 11, 10, 1e-7, 1, 0));
    b.f.push_back(make(3, 17, 31, 30, 2e-4, 0, 4));
    b.f.push_back(make(2, 70, 64, 1, 1e-3, 1, 2));
    b.finish();
    return b;
}

// The sequence of the autotuner case: a batch, the autotuner (twelve launch
// configurations, each captured, replayed and timed), the batch again.
void seq_autotune(fz_ctx* c) {
    Batch b = small_batch();
    CHECK(compress(c, b) == FZ_OK, "first batch");
    const std::vector<uint64_t> o0 = b.offs;
    CHECK(decompress(c, b.out, o0, b.p) == FZ_OK, "batch decompression");
    const int at = fz_batch_autotune(c, (uint32_t)b.f.size(), b.p.data(), b.x.data(), b.out, b.cap, nullptr);
    CHECK(at == FZ_OK || at == FZ_ERR_UNSUPPORTED, "autotune");
    CHECK(compress(c, b) == FZ_OK && b.offs == o0, "batch after tuning");
    CHECK(decompress(c, b.out, o0, b.p) == FZ_OK, "batch decompression after tuning");
    b.release();
}

// Single-call containers of fields packed at 16-byte offsets.
void pack_singles(fz_ctx* c, const std::vector<Field>& fs, uint8_t** packed, std::vector<uint64_t>& offs) {
    std::vector<std::vector<uint8_t>> conts;
    offs.assign(1, 0);
    for (const Field& f : fs) {
        const uint64_t cap = fz_compress_bound(&f.p);
        uint8_t* o = nullptr;
        hipMalloc((void**)&o, cap);
        uint64_t n = 0;
        CHECK(fz_compress(c, &f.p, f.d, o, cap, &n, nullptr) == FZ_OK, "single compress");
        conts.emplace_back(o, o + n);
        hipFree(o);
        offs.push_back(offs.back() + (n + 15) / 16 * 16);
    }
    hipMalloc((void**)packed, offs.back());
    memset(*packed, 0, offs.back());
    for (size_t k = 0; k < conts.size(); k++) memcpy(*packed + offs[k], conts[k].data(), conts[k].size());
}

// The sequence of the growth case: each kind of batch keeps its last
// graph while a call of the other kind with more fields grows that kind's
// buffers; the first description must then replay or re-capture cleanly.
void seq_growth(fz_ctx* c) {
    std::vector<float> sel(FZ_SELECTOR_PARAMS, 0.0f);
    for (int i = 16; i < 32; i++) sel[i] = 1.0f;
    CHECK(fz_selector_set(c, sel.data(), sel.size()) == FZ_OK, "selector");
    Batch big;
    big.f.push_back(make(3, 64, 64, 64, 1e-3, 1, 0));
    big.f.push_back(make(3, 56, 40, 48, 1e-3, 1, 3));
    big.finish();
    std::vector<Field> tiny;
    for (int i = 0; i < 80; i++) tiny.push_back(make(3, 8, 8, 8, 1e-3, 1, 0));
    std::vector<fz_params> tiny_p;
    for (const Field& f : tiny) tiny_p.push_back(f.p);

    CHECK(compress(c, big) == FZ_OK, "big batch");
    const std::vector<uint64_t> o1 = big.offs;
    uint8_t* packed40 = nullptr;
    std::vector<uint64_t> offs40;
    std::vector<Field> t40(tiny.begin(), tiny.begin() + 40);
    pack_singles(c, t40, &packed40, offs40);
    CHECK(decompress(c, packed40, offs40, std::vector<fz_params>(tiny_p.begin(), tiny_p.begin() + 40)) == FZ_OK,
          "40-field decompression");
    CHECK(compress(c, big) == FZ_OK && big.offs == o1, "big batch again");
    CHECK(decompress(c, big.out, big.offs, big.p) == FZ_OK, "big decompression");
    Batch t80;
    t80.f = tiny;
    t80.finish();
    CHECK(compress(c, t80) == FZ_OK, "80-field batch");
    CHECK(decompress(c, big.out, o1, big.p) == FZ_OK, "big decompression replay");
    CHECK(decompress(c, t80.out, t80.offs, t80.p) == FZ_OK, "80-field decompression");
    CHECK(compress(c, big) == FZ_OK && big.offs == o1, "big batch after the 80 fields");
    CHECK(decompress(c, big.out, o1, big.p) == FZ_OK, "big decompression at the end");
    hipFree(packed40);
    hipFree(t80.out);
    big.release();
    for (Field& f : tiny) hipFree(f.d);
}

}  // namespace

int main() {
    const size_t base = hipstub_live_allocations();
    for (int round = 0; round < 2; round++) {
        fz_ctx* c = nullptr;
        CHECK(fz_ctx_create(&c, 0, 0) == FZ_OK, "context");
        if (round == 0) {
            seq_autotune(c);
            seq_growth(c);
        } else {
            seq_growth(c);
            seq_autotune(c);
            seq_growth(c);
        }
        fz_ctx_destroy(c);
    }
    CHECK(hipstub_live_allocations() == base, "%zu allocations left", hipstub_live_allocations() - base);
    const int e = hipstub_errors();
    printf("batch replay: %d stub errors, %d failed checks\n", e, g_fail);
    return (e || g_fail) ? 1 : 0;
}
