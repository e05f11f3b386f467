// A host-only stand-in for the HIP runtime and the library's kernel
// launchers, for checking the library's host bookkeeping on a machine
// without a GPU (built with AddressSanitizer by tests/test_batch_lifetime.py).
//
// "Device" memory is host memory.  Every allocation is tracked; a kernel
// launch or an asynchronous copy is a node listing the buffers it touches.
// Outside a capture a node is checked at once; during a stream capture it
// joins the capture, and every launch of the instantiated graph checks all
// its nodes again: a node that references memory freed since the capture
// (or never allocated) is reported with the node's name and the run fails.
// Copies are carried out, so the host reads what the nodes copied.  Kernels
// compute nothing, except what the library's host code reads back: the
// container finaliser writes a header (valid layout, empty sections) and
// the size, field records and packing move sizes, offsets and containers,
// and the header gather copies headers.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2509_20563_amd/csrc/fz_kernels.h"

namespace {

struct Alloc {
    size_t size;
    bool host;
};
std::map<uintptr_t, Alloc> g_live;
int g_errors = 0;

struct Ref {
    const void* p;
    size_t bytes;  // 0 = only the address must lie in a live allocation
};
struct Node {
    std::string name;
    std::vector<Ref> refs;
    bool copy = false;
    void* dst = nullptr;
    const void* src = nullptr;
    size_t n = 0;
    std::function<void()> act;  // run when every reference is live
};

struct Capture;
struct Stream {
    Capture* cap = nullptr;
};
struct Capture {
    std::vector<Node> nodes;
    std::set<Stream*> members;
    Stream* origin = nullptr;
};
struct Event {
    Capture* cap = nullptr;  // recorded inside this capture
};
struct Graph {
    std::vector<Node> nodes;
};
struct Exec {
    std::vector<Node> nodes;
};
std::set<void*> g_graphs, g_execs, g_streams, g_events;
Stream g_null;

Stream* S(hipStream_t s) { return s ? reinterpret_cast<Stream*>(s) : &g_null; }

bool live(const void* p, size_t bytes) {
    if (!p) return true;
    const uintptr_t a = (uintptr_t)p;
    auto it = g_live.upper_bound(a);
    if (it == g_live.begin()) return false;
    --it;
    return a >= it->first && a + bytes <= it->first + it->second.size + (bytes ? 0 : 1);
}

void check(const Node& n, const char* when) {
    for (const Ref& r : n.refs)
        if (!live(r.p, r.bytes)) {
            fprintf(stderr, "hipstub: %s: node '%s' references %p (+%zu bytes) outside every live allocation\n", when,
                    n.name.c_str(), r.p, r.bytes);
            g_errors++;
        }
}

void run(const Node& n, const char* when) {
    const int before = g_errors;
    check(n, when);
    if (g_errors != before) return;
    if (n.copy) memmove(n.dst, n.src, n.n);
    if (n.act) n.act();
}

void submit(hipStream_t st, Node&& n) {
    Stream* s = S(st);
    if (s->cap) s->cap->nodes.push_back(std::move(n));
    else run(n, "eager launch");
}

void* track(size_t bytes, bool host) {
    void* p = malloc(bytes ? bytes : 1);
    memset(p, 0, bytes ? bytes : 1);
    g_live[(uintptr_t)p] = Alloc{bytes ? bytes : 1, host};
    return p;
}

hipError_t untrack(void* p, bool host) {
    if (!p) return hipSuccess;
    auto it = g_live.find((uintptr_t)p);
    if (it == g_live.end() || it->second.host != host) {
        fprintf(stderr, "hipstub: free of %p that is not a live %s allocation\n", p, host ? "pinned" : "device");
        g_errors++;
        return hipErrorInvalidValue;
    }
    g_live.erase(it);
    free(p);
    return hipSuccess;
}

}  // namespace

extern "C" int hipstub_errors() { return g_errors; }
extern "C" size_t hipstub_live_allocations() { return g_live.size(); }

// ------------------------------------------------------------- runtime API
hipError_t hipMalloc(void** p, size_t n) {
    *p = track(n, false);
    return hipSuccess;
}
hipError_t hipFree(void* p) { return untrack(p, false); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = track(n, true);
    return hipSuccess;
}
hipError_t hipHostFree(void* p) { return untrack(p, true); }

// Eager copies may involve host memory the caller owns: only addresses in
// tracked allocations are range-checked, the rest is left to the address
// sanitizer (a copy from freed heap memory is reported by it).  A copy
// captured into a graph must stay within tracked allocations.
bool owned(const void* p) {
    auto it = g_live.upper_bound((uintptr_t)p);
    if (it == g_live.begin()) return false;
    --it;
    return (uintptr_t)p < it->first + it->second.size;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    if (g_null.cap) {
        fprintf(stderr, "hipstub: synchronous copy during a capture\n");
        g_errors++;
    }
    Node c{"hipMemcpy", {}, true, dst, src, n};
    if (owned(dst)) c.refs.push_back({dst, n});
    if (owned(src)) c.refs.push_back({src, n});
    run(c, "hipMemcpy");
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t st) {
    const bool cap = S(st)->cap != nullptr;
    Node c{"hipMemcpyAsync", {}, true, dst, src, n};
    if (owned(dst) || cap) c.refs.push_back({dst, n});
    if (owned(src) || cap) c.refs.push_back({src, n});
    submit(st, std::move(c));
    return hipSuccess;
}

hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
    memset(p, 0, sizeof(*p));
    p->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    Stream* x = new Stream();
    g_streams.insert(x);
    *s = reinterpret_cast<hipStream_t>(x);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!g_streams.erase(s)) {
        g_errors++;
        return hipErrorInvalidValue;
    }
    delete S(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (S(s)->cap) {
        fprintf(stderr, "hipstub: synchronize of a capturing stream\n");
        g_errors++;
    }
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
    Event* x = new Event();
    g_events.insert(x);
    *e = reinterpret_cast<hipEvent_t>(x);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    if (!g_events.erase(e)) {
        g_errors++;
        return hipErrorInvalidValue;
    }
    delete reinterpret_cast<Event*>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    reinterpret_cast<Event*>(e)->cap = S(s)->cap;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    Capture* c = reinterpret_cast<Event*>(e)->cap;
    if (c && !S(s)->cap) {  // a fork: the stream joins the capture
        S(s)->cap = c;
        c->members.insert(S(s));
    }
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (S(s)->cap) return hipErrorIllegalState;
    Capture* c = new Capture();
    c->origin = S(s);
    c->members.insert(S(s));
    S(s)->cap = c;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    Capture* c = S(s)->cap;
    if (!c || c->origin != S(s)) return hipErrorIllegalState;
    for (Stream* m : c->members) m->cap = nullptr;
    Graph* gr = new Graph{std::move(c->nodes)};
    delete c;
    g_graphs.insert(gr);
    *g = reinterpret_cast<hipGraph_t>(gr);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    if (!g_graphs.count(g)) return hipErrorInvalidValue;
    Exec* e = new Exec{reinterpret_cast<Graph*>(g)->nodes};
    for (const Node& n : e->nodes) check(n, "instantiate");
    g_execs.insert(e);
    *x = reinterpret_cast<hipGraphExec_t>(e);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    if (!g_execs.count(x)) {
        fprintf(stderr, "hipstub: launch of a destroyed or unknown graph\n");
        g_errors++;
        return hipErrorInvalidValue;
    }
    if (S(s)->cap) return hipErrorIllegalState;
    for (const Node& n : reinterpret_cast<Exec*>(x)->nodes) run(n, "graph launch");
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    if (!g_execs.erase(x)) {
        g_errors++;
        return hipErrorInvalidValue;
    }
    delete reinterpret_cast<Exec*>(x);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    if (!g_graphs.erase(g)) {
        g_errors++;
        return hipErrorInvalidValue;
    }
    delete reinterpret_cast<Graph*>(g);
    return hipSuccess;
}

// -------------------------------------------------------- kernel launchers
namespace fz {

uint32_t scan_tiles(uint32_t n) { return (n + 1023) / 1024; }
uint32_t encode_groups(uint32_t ntiles) { return (ntiles + 11) / 12; }
uint32_t feature_tiles(uint32_t nblocks) { return (nblocks + 15) / 16; }

#define K(name, ...) submit(st, Node{name, {__VA_ARGS__}})
#define R(p) Ref{(const void*)(p), 0}

void launch_reset(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2, uint32_t n2,
                  uint64_t* d3, uint32_t n3, uint64_t, uint64_t, uint64_t) {
    K("reset", {misc, sizeof(Misc)}, {hist, 4ull * kHistCopies * kBins}, {d1, 8ull * n1}, {d2, 8ull * n2},
      {d3, 8ull * n3});
}
void launch_fill32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t) { K("fill32", {p, 4 * n}); }
void launch_minmax(hipStream_t st, const float* x, uint64_t N, int, Misc* misc, int) {
    K("minmax", {x, 4 * N}, {misc, sizeof(Misc)});
}
void launch_quant(hipStream_t st, int, const float* x, const Geom& g, uint32_t, double, int, Misc* misc,
                  uint32_t* hist, uint16_t* codes, uint32_t ntiles, uint32_t* tile_cnt, uint2* ostage, uint2* pstage,
                  int fixed, const uint8_t* bpred, int32_t* coef) {
    // the first-order instance (fixed 0) touches neither the map nor the
    // coefficients; a map is read when fixed < 0, coefficients written
    // for regression blocks
    K("quant", {x, 4 * g.N}, {misc, sizeof(Misc)}, {hist, 4ull * kBins}, {codes, 2ull * g.nblocks * kBlockElems},
      {tile_cnt, 4ull * ntiles}, {ostage, 8ull * ntiles * kTileBlocks * kBlockElems},
      {pstage, 8ull * ntiles * kTileBlocks * kBlockElems}, {bpred, fixed < 0 ? g.nblocks : 0ull},
      {coef, fixed < 0 || fixed == 2 ? 16ull * g.nblocks : 0ull});
}
void launch_quant_shuffle(hipStream_t st, int, const float* x, const Geom& g, uint32_t, double, int, Misc* misc,
                          uint32_t*, uint32_t* slots, uint32_t ntiles, uint32_t* tile_cnt, uint2* ostage,
                          uint2* pstage) {
    // no histogram; the staging slots are the codes buffer
    K("quant_shuffle", {x, 4 * g.N}, {misc, sizeof(Misc)}, {slots, 2ull * g.nblocks * kBlockElems},
      {tile_cnt, 4ull * ntiles}, {ostage, 8ull * ntiles * kTileBlocks * kBlockElems},
      {pstage, 8ull * ntiles * kTileBlocks * kBlockElems});
}
void launch_trial(hipStream_t st, int, const float* x, const Geom& g, uint32_t, double, int, Misc* misc, uint32_t,
                  const uint32_t* cw_ref, uint8_t* choice, uint32_t* costs) {
    K("trial", {x, 4 * g.N}, {misc, sizeof(Misc)}, {cw_ref, 4ull * kBins}, {choice, g.nblocks},
      {costs, costs ? 12ull * g.nblocks : 0ull});
}
void launch_features(hipStream_t st, int, const float* x, const Geom& g, uint32_t, double, int, Misc* misc,
                     float* feat) {
    K("features", {x, 4 * g.N}, {misc, sizeof(Misc)}, {feat, 64ull * g.nblocks});
}
void launch_mlp(hipStream_t st, int, const float* feat, uint32_t n, const float* sel, float* yout, uint8_t* choice) {
    K("mlp", {feat, 64ull * n}, {sel, 4ull * kSelectorParams}, {yout, yout ? 12ull * n : 0ull}, {choice, n});
}
void launch_scan(hipStream_t st, int, const void* in, uint32_t n, uint64_t* out, uint64_t* desc, uint32_t* ctr,
                 Misc* misc, uint64_t) {
    K("scan", {in, n}, {out, 8ull * n}, {desc, 8ull * scan_tiles(n)}, {ctr, 4}, {misc, sizeof(Misc)});
}
void launch_codebook(hipStream_t st, uint32_t* hist, uint8_t* out_lens, uint32_t* cw, Misc* misc) {
    K("codebook", {hist, 4ull * kHistCopies * kBins}, {out_lens, kBins / 2}, {cw, 4ull * kBins},
      {misc, sizeof(Misc)});
}
void launch_encode(hipStream_t st, int, const uint16_t* codes, const Geom& g, const uint32_t* cw, Misc* misc,
                   uint32_t ntiles, uint8_t* out, uint64_t* desc, uint64_t* tile_start, uint32_t* tfirst,
                   uint32_t* tlast) {
    K("encode", {codes, 2ull * g.nblocks * kBlockElems}, {cw, 4ull * kBins}, {misc, sizeof(Misc)}, R(out),
      {desc, 8ull * encode_groups(ntiles)}, {tile_start, 8ull * ntiles}, {tfirst, 4ull * ntiles},
      {tlast, 4ull * ntiles});
}
void launch_finalize(hipStream_t st, const Geom& g, uint32_t mode, double eb, uint32_t pred, Misc* misc, uint8_t* out,
                     uint32_t ntiles, const uint64_t* tile_start, const uint32_t* tfirst, const uint32_t* tlast,
                     const uint32_t* tile_cnt, const uint64_t* tile_off, const uint2* ostage, const uint2* pstage,
                     const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coef, const float* x,
                     uint32_t) {
    Node nd{"finalize", {{misc, sizeof(Misc)}, R(out), {tile_start, 8ull * ntiles}, {tfirst, 4ull * ntiles},
                         {tlast, 4ull * ntiles}, {tile_cnt, 4ull * ntiles}, {tile_off, 8ull * ntiles}, R(ostage),
                         R(pstage), R(bpred), R(reg_idx), R(coef), {x, 4 * g.N}}};
    // a container whose header the library accepts: one bit per value, no
    // outliers or patches, regression coefficients for every block of a
    // regression-only field
    const Geom gg = g;
    nd.act = [=]() {
        const uint64_t bits = gg.N, words = (bits + 31) / 32;
        const bool map = pred == 3 || pred == 4;
        const uint64_t nreg = pred == 2 ? gg.nblocks : 0;
        const Layout L = make_layout(gg.nblocks, map, nreg, words, 0, 0);
        uint8_t h[kHdr] = {};
        auto put = [&](int o, uint64_t v, int n) {
            for (int k = 0; k < n; k++) h[o + k] = (uint8_t)(v >> (8 * k));
        };
        const double eb_abs = eb;
        uint64_t ebb, eab;
        memcpy(&ebb, &eb, 8);
        memcpy(&eab, &eb_abs, 8);
        put(0, kMagic, 4);
        put(4, kVersion, 2);
        put(8, gg.ndim, 4);
        put(12, pred, 4);
        for (int a = 0; a < 3; a++) put(16 + 8 * a, gg.n[a], 8);
        put(40, mode, 4);
        put(44, kRadius, 4);
        put(48, ebb, 8);
        put(56, eab, 8);
        put(64, L.total, 8);
        put(72, gg.nblocks, 4);
        put(84, words, 4);
        put(88, bits, 8);
        put(96, nreg, 4);
        memcpy(out, h, kHdr);
        misc->total_bytes = L.total;
    };
    submit(st, std::move(nd));
}
void launch_targets(hipStream_t st, const uint32_t* costs, uint64_t n, float* t) {
    K("targets", {costs, 12 * n}, {t, 12 * n});
}
void launch_feature_stats(hipStream_t st, const float* feat, uint64_t n, float* w) {
    K("feature_stats", {feat, 64 * n}, R(w));
}
void launch_train_batch(hipStream_t st, const float* w, const float* feat, const float*, const uint32_t*, uint32_t,
                        TrainScratch& s, float* loss_out) {
    K("train_batch", R(w), R(feat), R(s.Z), R(s.grad), R(loss_out));
}
void launch_adam(hipStream_t st, float* w, float* m, float* v, const float* g, int, float, float, float, float) {
    K("adam", {w, 4ull * kSelectorParams}, {m, 4ull * kSelectorParams}, {v, 4ull * kSelectorParams},
      {g, 4ull * kSelectorParams});
}
void launch_field_record(hipStream_t st, const Misc* misc, uint64_t slot, uint64_t* rec, int decode) {
    Node nd{"field_record", {{misc, sizeof(Misc)}, {rec, decode ? 40ull : 24ull}}};
    nd.act = [=]() {
        if (decode) {
            rec[0] = misc->flags;
            rec[1] = misc->code0_count;
            rec[2] = misc->nreg;
            rec[3] = misc->ohash_dec;
            rec[4] = misc->ohash_list;
        } else {
            rec[0] = slot;
            rec[1] = misc->total_bytes;
            rec[2] = misc->flags;
        }
    };
    submit(st, std::move(nd));
}
void launch_pack(hipStream_t st, const uint8_t* stage, const uint64_t* rec, uint64_t* offs, uint32_t n, uint8_t* out) {
    Node nd{"pack", {R(stage), {rec, 24ull * n}, {offs, 8ull * (n + 1)}, R(out)}};
    nd.act = [=]() {
        uint64_t o = 0;
        for (uint32_t i = 0; i < n; i++) {
            offs[i] = o;
            const uint64_t len = (rec[3 * i + 1] + 15) & ~15ull;
            if (!live(stage + rec[3 * i], len) || !live(out + o, len)) {
                fprintf(stderr, "hipstub: pack of field %u out of bounds\n", i);
                g_errors++;
                return;
            }
            memset(out + o, 0, len);
            memcpy(out + o, stage + rec[3 * i], rec[3 * i + 1]);
            o += len;
        }
        offs[n] = o;
    };
    submit(st, std::move(nd));
}
void launch_gather_headers(hipStream_t st, const uint8_t* in, const uint64_t* offs, uint32_t n, uint8_t* hdr) {
    // the one kernel carried out: the library parses its output on the host
    Node nd{"gather_headers", {R(in), {offs, 8ull * (n + 1)}, {hdr, (uint64_t)kHdr * n}}};
    if (S(st)->cap) {
        fprintf(stderr, "hipstub: header gather captured\n");
        g_errors++;
    }
    check(nd, "eager launch");
    for (uint32_t i = 0; i < n; i++) memcpy(hdr + (uint64_t)kHdr * i, in + offs[i], kHdr);
}
void launch_copy(hipStream_t st, const uint8_t* src, float* dst, uint64_t n) { K("copy", {src, 4 * n}, {dst, 4 * n}); }
void launch_reset_lut(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2, uint32_t n2,
                      uint64_t* d3, uint32_t n3, uint64_t, uint64_t, uint64_t, const uint8_t* lens, uint16_t* lut) {
    K("reset_lut", {misc, sizeof(Misc)}, {hist, 4ull * kBins}, {d1, 8ull * n1}, {d2, 8ull * n2}, {d3, 8ull * n3},
      {lens, kBins / 2}, {lut, 2ull * kLut});
}
void launch_outlier_index(hipStream_t st, const Geom& g, const uint32_t* opos, uint64_t n_out, uint2* oidx, Misc* misc) {
    K("outlier_index", {opos, 4 * n_out}, {oidx, 8ull * g.nblocks}, {misc, sizeof(Misc)});
}
void launch_decode(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t words, const uint64_t* off,
                   const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos, const int32_t* oval,
                   const uint2* oidx, uint64_t n_out, double, float* out, int, Misc* misc) {
    K("decode", {stream, 4 * words}, {off, 8ull * g.nblocks}, {chunks, 2ull * g.nblocks}, {lut, 2ull * kLut},
      {opos, 4 * n_out}, {oval, 4 * n_out}, {oidx, 8ull * g.nblocks}, {out, 4 * g.N}, {misc, sizeof(Misc)});
}
void launch_map_unpack(hipStream_t st, const uint8_t* map, uint32_t nblocks, uint8_t* bpred, Misc* misc) {
    K("map_unpack", {map, (nblocks + 3) / 4}, {bpred, nblocks}, {misc, sizeof(Misc)});
}
void launch_decode_pred(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t words, const uint64_t* off,
                        const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos, const int32_t* oval,
                        const uint2* oidx, uint64_t n_out, int32_t* res, int, const uint8_t* bpred,
                        const uint64_t* reg_idx, const int32_t* coefs, uint64_t nreg, double, float* out, int,
                        Misc* misc) {
    K("decode_pred", {stream, 4 * words}, {off, 8ull * g.nblocks}, {chunks, 2ull * g.nblocks}, {lut, 2ull * kLut},
      {opos, 4 * n_out}, {oval, 4 * n_out}, {oidx, 8ull * g.nblocks}, {res, 4ull * g.nblocks * kBlockElems},
      R(bpred), R(reg_idx), {coefs, 16 * nreg}, {out, 4 * g.N}, {misc, sizeof(Misc)});
}
void launch_decode_residuals(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t words,
                             const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                             const int32_t* oval, const uint2* oidx, uint64_t n_out, int32_t* res, int, Misc* misc) {
    K("decode_residuals", {stream, 4 * words}, {off, 8ull * g.nblocks}, {chunks, 2ull * g.nblocks},
      {lut, 2ull * kLut}, {opos, 4 * n_out}, {oval, 4 * n_out}, {oidx, 8ull * g.nblocks},
      {res, 4ull * g.nblocks * kBlockElems}, {misc, sizeof(Misc)});
}
uint32_t global_scan_tiles(uint64_t N) { return (uint32_t)((N + 2047) / 2048); }
void launch_global_inverse(hipStream_t st, const Geom& g, int32_t* q, uint64_t* desc, Misc* misc, double, float* out,
                           int) {
    K("global_inverse", {q, 4ull * g.nblocks * kBlockElems}, {desc, g.ndim == 1 ? 8ull * global_scan_tiles(g.N) : 0ull},
      {misc, sizeof(Misc)}, {out, 4 * g.N});
}
void launch_interp_inverse(hipStream_t st, const Geom& g, int32_t* q, double, float* out) {
    K("interp_inverse", {q, 4ull * g.N}, {out, 4 * g.N});
}
void launch_shuffle_copy(hipStream_t st, const Geom& g, const uint32_t* slots, const uint64_t* off, uint8_t* out,
                         uint64_t limit) {
    K("shuffle_copy", {slots, 2ull * g.nblocks * kBlockElems}, {off, 8ull * g.nblocks}, {out, limit});
}
void launch_unshuffle(hipStream_t st, const Geom& g, const uint32_t* masks, const uint32_t* kept, uint64_t nkept,
                      const uint64_t* off, const uint32_t* opos, const int32_t* oval, const uint2* oidx,
                      uint64_t n_out, double, float* out, Misc* misc) {
    K("unshuffle", {masks, 20ull * g.nblocks}, {kept, 4 * nkept}, {off, 8ull * g.nblocks}, {opos, 4 * n_out},
      {oval, 4 * n_out}, {oidx, 8ull * g.nblocks}, {out, 4 * g.N}, {misc, sizeof(Misc)});
}
void launch_patch(hipStream_t st, const Geom& g, const uint32_t* ppos, const uint32_t* pbits, uint64_t n_pat, float* out,
                  Misc* misc) {
    K("patch", {ppos, 4 * n_pat}, {pbits, 4 * n_pat}, {out, 4 * g.N}, {misc, sizeof(Misc)});
}

}  // namespace fz
