// Internal definitions shared by the HIP translation units of libfz.
// Geometry of the blocked field, device scratch layout, and device helpers
// (ordered float encoding, decoupled look-back, canonical Huffman ranks).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fz {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- constants
constexpr int kRadius = 512;      // residuals -511..511 map to codes 1..1023
constexpr int kBins = 1024;       // code 0 marks an outlier
// Copies of the global code histogram: workgroup w adds into copy
// w % kHistCopies, so at most 1/kHistCopies of the workgroups chain their
// atomics on one address; the codebook kernel sums the copies.
constexpr int kHistCopies = 16;
constexpr int kLmax = 12;         // longest Huffman codeword, LUT index width
constexpr int kLut = 1 << kLmax;  // decode table entries
constexpr int kHdr = 128;         // container header bytes
constexpr int kBlockElems = 512;  // values per full block
constexpr int kSegs = 64;         // 8-value segments per block
constexpr int kTileBlocks = 4;    // blocks per workgroup tile (256 threads)
constexpr uint32_t kMagic = 0x314D5A46u;  // "FZM1"
// block-feature selector network: 16 features, two hidden layers of 64,
// one output per predictor
// (version 2: the features are taken over a sample, the block's first 128
// positions in row-major order = segments 0..15, the lower box of the block)
constexpr int kNFeat = 16;
constexpr uint32_t kFeatureVersion = 2;
constexpr int kFeatSample = 128;
constexpr int kFeatSegs = kFeatSample / 8;
constexpr int kNHid = 64;
constexpr int kNOut = 3;
constexpr int kSelectorParams = 2 * kNFeat + kNHid * kNFeat + kNHid + kNHid * kNHid + kNHid + kNOut * kNHid + kNOut;
constexpr uint16_t kVersion = 1;

// prefix-scan kinds (fz_scan.hip)
enum { SCAN_COUNTS = 0, SCAN_CHUNKS = 2, SCAN_PMAP = 3, SCAN_MASKS = 4, SCAN_SLOTS = 5 };

// flag bits raised by kernels in Misc::flags
enum : uint32_t {
    F_NONFINITE = 1u,
    F_EB = 2u,
    F_OVERFLOW = 4u,   // outlier/patch totals saturate: the container goes verbatim
    F_CORRUPT = 8u,
    F_INTERNAL = 16u,
    F_TIMEOUT = 32u,   // a bounded look-back wait gave up
};

// Per-call device scratch, cleared by k_reset.
struct Misc {
    uint32_t flags;
    uint32_t mm_lo, mm_hi;     // order-preserving encodings of min and max
    uint32_t qtile_ctr;        // dynamic tile counters (look-back order)
    uint32_t stile_ctr;
    uint32_t code0_count;      // decode: outlier codes seen
    uint32_t mtile_ctr;        // predictor-map scan
    uint32_t map_off;          // per-block choice is first-order everywhere:
                               // written as a first-order container
    uint64_t total_bits_cb;    // sum hist[c] * len[c]
    uint64_t total_bits_enc;   // end of the last encoded tile (bit-shuffle
                               // codec: kept words)
    uint64_t n_out;            // outliers (inclusive count of the last tile)
    uint64_t n_pat;            // lossless patches
    uint64_t total_bytes;      // container size (non-verbatim)
    uint64_t verbatim;         // 1 when the packed container is not smaller
    double eb_abs;
    uint64_t off_chunks;       // container offsets of the chunk table and
    uint64_t off_stream;       // the stream (depend on the map/coefficients)
    uint64_t nreg;             // blocks predicted by regression
    // decode: sums of a hash of the positions of the outlier codes met and
    // of the positions in the outlier list (equal for a valid container)
    uint64_t ohash_dec, ohash_list;
};

// Hash of an outlier position for the decode-side consistency sums.
__host__ __device__ inline uint64_t pos_hash(uint32_t p) {
    uint64_t h = ((uint64_t)p + 1) * 0x9E3779B97F4A7C15ull;
    return h ^ (h >> 29);
}

// Term of one outlier position in the decoder's consistency check (the sum
// over the codes met against the sum over the stored list): the row of 8
// the position lies in, mixed, times 2^(position in the row).  The terms of
// one row sum to pos_hash(row) * (the row's 8-bit outlier mask), so a
// decoder may add a whole row at once.
__host__ __device__ inline uint64_t outlier_term(uint32_t p) { return pos_hash(p >> 3) << (p & 7); }

// Unsigned division by a runtime constant d <= 2^23 for numerators <= 2^23:
// q = (umulhi(n, m) + n) >> l with l = ceil(log2 d), m = 2^32 (2^l - d) / d + 1
// (Granlund & Montgomery; the sum cannot overflow for these ranges).
struct FastDiv {
    uint32_t m, l;
};

__host__ inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) l++;
    FastDiv f;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    f.l = l;
    return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f) {
#ifdef __HIP_DEVICE_COMPILE__
    return (__umulhi(n, f.m) + n) >> f.l;
#else
    return (uint32_t)(((((uint64_t)n * f.m) >> 32) + n) >> f.l);
#endif
}

// Field geometry: dims, block shape, block grid.
struct Geom {
    uint32_t ndim;
    uint32_t n[3];   // extents (unused axes 1)
    uint32_t bs[3];  // block extents: 1D 512; 2D 32x16; 3D 8x8x8
    uint32_t nb[3];  // blocks per axis
    uint32_t nblocks;
    uint64_t N;
    FastDiv dnb0, dnb1;  // division by nb[0] and nb[1]
};

// Block coordinates and real extents of block b.
struct BlockInfo {
    uint32_t bx, by, bz;
    uint32_t ex, ey, ez;
};

__host__ __device__ inline BlockInfo block_info(const Geom& g, uint32_t b) {
    BlockInfo r;
    const uint32_t t = fdiv(b, g.dnb0);
    r.bx = b - t * g.nb[0];
    r.bz = fdiv(t, g.dnb1);
    r.by = t - r.bz * g.nb[1];
    uint32_t x0 = r.bx * g.bs[0], y0 = r.by * g.bs[1], z0 = r.bz * g.bs[2];
    r.ex = min(g.bs[0], g.n[0] - x0);
    r.ey = min(g.bs[1], g.n[1] - y0);
    r.ez = min(g.bs[2], g.n[2] - z0);
    return r;
}

// Segment s (0..63) of a block = 8 consecutive values along x:
//   3D: row (ly, lz) = (s % 8, s / 8), x from 0;  2D: x from 8 * (s % 4), ly = s / 4;
//   1D: x from 8 * s.  In-block offset of value i of segment s is 8 * s + i.
template <int ND>
__host__ __device__ inline void seg_coords(uint32_t s, uint32_t& lx0, uint32_t& ly, uint32_t& lz) {
    if (ND == 3) { lx0 = 0; ly = s & 7; lz = s >> 3; }
    else if (ND == 2) { lx0 = 8 * (s & 3); ly = s >> 2; lz = 0; }
    else { lx0 = 8 * s; ly = 0; lz = 0; }
}

// Row-major index of the first value of segment s in block (bi), and the
// number of real values in the segment (0..8).
template <int ND>
__host__ __device__ inline uint64_t seg_index(const Geom& g, const BlockInfo& bi, uint32_t s, uint32_t& nvalid) {
    uint32_t lx0, ly, lz;
    seg_coords<ND>(s, lx0, ly, lz);
    if (ly >= bi.ey || lz >= bi.ez || lx0 >= bi.ex) {
        nvalid = 0;
        return 0;
    }
    nvalid = min(8u, bi.ex - lx0);
    uint64_t x = (uint64_t)bi.bx * g.bs[0] + lx0;
    uint64_t y = (uint64_t)bi.by * g.bs[1] + ly;
    uint64_t z = (uint64_t)bi.bz * g.bs[2] + lz;
    return x + (uint64_t)g.n[0] * (y + (uint64_t)g.n[1] * z);
}

// Container section offsets (each 16-byte aligned): header, code lengths,
// [predictor map, 2 bits per block, when predictors are chosen per block],
// [regression coefficients, 4 x i32 per regression block], chunk table,
// stream, outlier positions, outlier residuals, patch positions, patch bits.
struct Layout {
    uint64_t lens, map, coef, chunks, stream, opos, oval, ppos, pbits, total;
};

__host__ __device__ inline uint64_t align16(uint64_t v) { return (v + 15) & ~15ull; }

__host__ __device__ inline Layout make_layout(uint64_t nblocks, bool has_map, uint64_t nreg, uint64_t words,
                                              uint64_t nout, uint64_t npat) {
    Layout L;
    L.lens = kHdr;
    L.map = L.lens + kBins / 2;
    L.coef = align16(L.map + (has_map ? (nblocks + 3) / 4 : 0));
    L.chunks = align16(L.coef + 16 * nreg);
    L.stream = align16(L.chunks + 2 * nblocks);
    L.opos = align16(L.stream + 4 * words);
    L.oval = align16(L.opos + 4 * nout);
    L.ppos = align16(L.oval + 4 * nout);
    L.pbits = align16(L.ppos + 4 * npat);
    L.total = align16(L.pbits + 4 * npat);
    return L;
}

// Bit-shuffle codec (header flag bit 1): per block a 160-bit mask of the
// non-zero plane words (5 u32), then the kept words of all blocks; the
// outlier and patch sections as above.  lens, map and coef are unused
// (set to the mask section), chunks = the masks, stream = the kept words.
constexpr uint32_t kFlagShuffle = 2;
constexpr int kMaskWords = 5;
constexpr int kPlanes = 10;
constexpr uint32_t kSymOutlier = 1023;
__host__ __device__ inline Layout make_speed_layout(uint64_t nblocks, uint64_t words, uint64_t nout, uint64_t npat) {
    Layout L;
    L.lens = L.map = L.coef = L.chunks = kHdr;
    L.stream = align16(L.chunks + 4 * kMaskWords * nblocks);
    L.opos = align16(L.stream + 4 * words);
    L.oval = align16(L.opos + 4 * nout);
    L.ppos = align16(L.oval + 4 * nout);
    L.pbits = align16(L.ppos + 4 * npat);
    L.total = align16(L.pbits + 4 * npat);
    return L;
}

// Predictor modes (header field): 0, 1, 2 = that predictor in every block;
// 3 = chosen per block by the learned selector, 4 = by exhaustive trial.
constexpr uint32_t kPredSelected = 3, kPredTrial = 4;
__host__ __device__ inline bool pred_has_map(uint32_t pred) { return pred == kPredSelected || pred == kPredTrial; }

// Interpolation predictor (header predictor 5): over the whole field, not
// block-local.  Anchors (every coordinate a multiple of 8) are predicted by
// first-order Lorenzo on the anchor grid; a point whose coordinates are all
// multiples of s in {4, 2, 1} (not all of 2s) is interpolated along the
// first axis, in x, y, z order, on which it is an odd multiple of s, from
// the neighbours at -/+ s and -/+ 3s: cubic floor((-q[-3s] + 9 q[-s] +
// 9 q[+s] - q[+3s] + 8) / 16) when both 3s neighbours are inside, else
// floor((q[-s] + q[+s] + 1) / 2) when +s is, else q[-s].  Decoding rebuilds
// the anchors, then for s = 4, 2, 1 the points interpolated along z, then
// y, then x, each from points rebuilt before.
constexpr uint32_t kPredInterp = 5;

// Global first-order Lorenzo (header predictor 6): the Lorenzo formula with
// neighbours anywhere in the field (zero outside it); the inverse is the
// prefix sum along x of every row of the field, then along y, then along z.
constexpr uint32_t kPredGlobal = 6;

// Axis a point is interpolated along (-1 for an anchor) and its stride.
__host__ __device__ inline int interp_class(const uint32_t c[3], int nd, uint32_t& s) {
    uint32_t orc = 0;
    for (int a = 0; a < nd; a++) orc |= c[a];
    if ((orc & 7u) == 0) {
        s = 8;
        return -1;
    }
    s = (orc & 3u) == 0 ? 4u : ((orc & 1u) == 0 ? 2u : 1u);
    for (int a = 0; a < nd; a++)
        if (c[a] & s) return a;
    return -1;
}

// Prediction at c from the grid values q_at(x, y, z) (n: field extents).
template <class QAt>
__host__ __device__ inline int32_t interp_predict(const uint32_t c[3], const uint32_t n[3], int nd, QAt q_at) {
    uint32_t s;
    const int a = interp_class(c, nd, s);
    if (a < 0) {
        // Lorenzo on the anchor grid: +/- the neighbours 8 below in every
        // non-empty subset of the axes (odd subsets added), zero outside
        int64_t p = 0;
        for (int m = 1; m < (1 << nd); m++) {
            uint32_t d[3] = {c[0], c[1], c[2]};
            bool in = true;
            for (int k = 0; k < nd; k++)
                if (m >> k & 1) {
                    if (d[k] < 8) in = false;
                    else d[k] -= 8;
                }
            if (!in) continue;
            const int64_t v = q_at(d[0], d[1], d[2]);
            p += (__builtin_popcount((unsigned)m) & 1) ? v : -v;
        }
        return (int32_t)p;
    }
    uint32_t lo1[3] = {c[0], c[1], c[2]}, hi1[3] = {c[0], c[1], c[2]};
    lo1[a] -= s;
    hi1[a] += s;
    const uint32_t ca = c[a];
    const bool m3 = ca >= 3 * s, p1 = ca + s < n[a], p3 = ca + 3 * s < n[a];
    if (m3 && p3) {
        uint32_t lo3[3] = {c[0], c[1], c[2]}, hi3[3] = {c[0], c[1], c[2]};
        lo3[a] -= 3 * s;
        hi3[a] += 3 * s;
        const int64_t num = -(int64_t)q_at(lo3[0], lo3[1], lo3[2]) + 9 * (int64_t)q_at(lo1[0], lo1[1], lo1[2]) +
                            9 * (int64_t)q_at(hi1[0], hi1[1], hi1[2]) - (int64_t)q_at(hi3[0], hi3[1], hi3[2]);
        return (int32_t)((num + 8) >> 4);
    }
    if (p1)
        return (int32_t)(((int64_t)q_at(lo1[0], lo1[1], lo1[2]) + (int64_t)q_at(hi1[0], hi1[1], hi1[2]) + 1) >> 1);
    return q_at(lo1[0], lo1[1], lo1[2]);
}

// ------------------------------------------------------- device helpers
// Order-preserving map float -> u32 (unsigned compare = float compare).
__device__ inline uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float unord_f32(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Absolute bound from the mode: absolute, or eb times the value range
// (range 0 -> eb).  Returns false when the bound is out of [1e-300, 1e300].
__host__ __device__ inline bool resolve_eb(uint32_t mode, double eb, uint32_t mm_lo, uint32_t mm_hi, double* eb_abs) {
    double e = eb;
    if (mode == 1) {
        double range = (double)unord_f32(mm_hi) - (double)unord_f32(mm_lo);
        e = (range > 0.0) ? eb * range : eb;
    }
    *eb_abs = e;
    return e >= 1e-300 && e <= 1e300;
}

// ------------------------------------------------ prequantisation helper
// q = rint(x / 2eb) via x * (1 / 2eb) in double, round half to even.
// Patch when |t| >= 2^24 (q = 0) or when float(q * 2eb) misses the bound.
// Out of range, r and xh are meaningless but discarded: the value is a
// patch with q = 0 either way (the conversion of such r is the hardware's
// clamping one).
__device__ __forceinline__ int32_t prequant1(float xv, double e2, double inv, double eb_abs, bool& patch) {
    const double xd = (double)xv;
    const double t = xd * inv;
    const bool big = fabs(t) >= 16777216.0;
    const double r = __builtin_rint(t);
    const float xh = (float)(r * e2);
    patch = big || (fabs(xd - (double)xh) > eb_abs);
    const int32_t q = (int32_t)r;
    return big ? 0 : q;
}


// Per-call scratch reset: Misc (one thread) and the grid-stride clearing
// of the histogram copies and up to three descriptor/index arrays.
__device__ __forceinline__ void reset_misc(Misc* misc, uint64_t off_chunks, uint64_t off_stream, uint64_t nreg) {
    Misc m = {};
    m.mm_lo = 0xFFFFFFFFu;
    m.mm_hi = 0u;
    m.off_chunks = off_chunks;
    m.off_stream = off_stream;
    m.nreg = nreg;
    *misc = m;
}
__device__ __forceinline__ void clear_scratch(uint32_t gid, uint32_t stride, uint32_t* hist, uint64_t* d1,
                                              uint32_t n1, uint64_t* d2, uint32_t n2, uint64_t* d3, uint32_t n3) {
    for (uint32_t i = gid; i < (uint32_t)(kHistCopies * kBins); i += stride) hist[i] = 0;
    for (uint32_t i = gid; i < n1; i += stride) d1[i] = 0;
    for (uint32_t i = gid; i < n2; i += stride) d2[i] = 0;
    for (uint32_t i = gid; i < n3; i += stride) d3[i] = 0;
}

// Decoupled look-back (single-pass prefix scan over tiles taken in order
// from an atomic counter).  desc[t] holds status (2 high bits: 1 = tile
// aggregate, 2 = inclusive prefix) and a 62-bit payload combined by Op
// (associative and commutative).  Executed by one whole wave: lane i reads
// the descriptor of tile t-1-i, so one round trip covers 64 predecessors;
// the payloads up to the nearest inclusive one are reduced across the wave.
// The wait on a predecessor is bounded: after the spin limit the tile
// raises F_TIMEOUT and proceeds, so every wave always exits.  Returns the
// exclusive prefix in every lane.
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStInc = 2ull << 62;
constexpr uint64_t kPayload = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

template <class Op>
__device__ inline uint64_t wave_reduce64(uint64_t v, Op op) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = op(v, __shfl_xor(v, d, 64));
    return v;
}

template <class Op>
__device__ inline uint64_t lookback(uint64_t* desc, uint32_t t, uint64_t agg, Op op, uint32_t* flags) {
    const int lane = threadIdx.x & 63;
    if (t == 0) {
        if (lane == 0) __hip_atomic_store(&desc[0], kStInc | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0) __hip_atomic_store(&desc[t], kStAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t base = (int64_t)t - 1;
    uint32_t spins = 0;
    for (;;) {
        const int64_t j = base - lane;
        // before tile 0 there is an implicit inclusive prefix of 0
        const uint64_t d =
            j >= 0 ? __hip_atomic_load(&desc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kStInc;
        const uint32_t st = (uint32_t)(d >> 62);
        const uint64_t inc = __ballot(st == 2);
        const uint64_t notready = __ballot(st == 0);
        const int first = inc ? __ffsll((long long)inc) - 1 : 64;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
        if (notready & need) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(flags, F_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const uint64_t v = wave_reduce64(lane <= first ? (d & kPayload) : 0ull, op);
        excl = op(excl, v);
        if (first < 64) break;
        base -= 64;
    }
    if (lane == 0) __hip_atomic_store(&desc[t], kStInc | op(excl, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

struct OpAdd {
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return (a + b) & kPayload; }
};


// Two saturating 31-bit counters in one payload (outliers low, patches high).
struct OpPair31 {
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const {
        const uint64_t m = (1ull << 31) - 1;
        uint64_t lo = (a & m) + (b & m);
        uint64_t hi = (a >> 31) + (b >> 31);
        if (lo > m) lo = m;
        if (hi > m) hi = m;
        return lo | (hi << 31);
    }
};

// DPP data movement (gfx9 wave64): row_shr:k shifts within rows of 16
// lanes, row_bcast:15 / row_bcast:31 pass a row's last lane to later rows.
// Lanes with no source, or in rows outside ROWMASK, receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    const uint32_t lo = dpp32<CTRL, ROWMASK>((uint32_t)v);
    const uint32_t hi = dpp32<CTRL, ROWMASK>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Wave-level inclusive scan (64 lanes, all active): Hillis-Steele inside
// each row of 16 lanes, then row totals carried across rows.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp32<0x111, 0xf>(v);
    v += dpp32<0x112, 0xf>(v);
    v += dpp32<0x114, 0xf>(v);
    v += dpp32<0x118, 0xf>(v);
    v += dpp32<0x142, 0xa>(v);
    v += dpp32<0x143, 0xc>(v);
    return v;
}

template <class Op>
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v, Op op) {
    v = op(dpp64<0x111, 0xf>(v), v);
    v = op(dpp64<0x112, 0xf>(v), v);
    v = op(dpp64<0x114, 0xf>(v), v);
    v = op(dpp64<0x118, 0xf>(v), v);
    v = op(dpp64<0x142, 0xa>(v), v);
    v = op(dpp64<0x143, 0xc>(v), v);
    return v;
}

// Canonical Huffman code assignment inside one 1024-thread workgroup:
// thread t owns symbol t with length len (0 = unused).  Symbols are ordered
// by (length, symbol); each gets the first code of its length plus its rank.
// Produces code[t] and, in shared memory, count[L], first[L] and the
// symbols sorted by (length, symbol) (sorted[offset[L] + rank]).
struct CanonShared {
    uint32_t wave_cnt[kLmax + 1][16];
    uint32_t count[kLmax + 2];
    uint32_t first[kLmax + 2];
    uint32_t offset[kLmax + 2];
    uint16_t sorted[kBins];
};

__device__ inline uint32_t canonical_code(uint32_t len, CanonShared& sh) {
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t myrank = 0;
    for (int L = 1; L <= kLmax; L++) {
        uint64_t m = __ballot(len == (uint32_t)L);
        if (lane == 0) sh.wave_cnt[L][wave] = __popcll(m);
        if (len == (uint32_t)L) myrank = __popcll(m & ((1ull << lane) - 1));
    }
    __syncthreads();
    if (wave == 0) {
        // lane L (1..kLmax): exclusive prefix of its length's counts over
        // the waves; then first code and sorted offset per length, in order
        uint32_t c = 0;
        if (lane >= 1 && lane <= (uint32_t)kLmax)
            for (int w = 0; w < 16; w++) {
                const uint32_t v = sh.wave_cnt[lane][w];
                sh.wave_cnt[lane][w] = c;
                c += v;
            }
        uint32_t code = 0, off = 0;
        for (int L = 1; L <= kLmax; L++) {
            const uint32_t cL = (uint32_t)__shfl((int)c, L, 64);
            if (lane == (uint32_t)L) {
                sh.count[L] = cL;
                sh.first[L] = code;
                sh.offset[L] = off;
            }
            code = (code + cL) << 1;
            off += cL;
        }
    }
    __syncthreads();
    uint32_t code = 0;
    if (len > 0) {
        uint32_t r = sh.wave_cnt[len][wave] + myrank;
        code = sh.first[len] + r;
        sh.sorted[sh.offset[len] + r] = (uint16_t)t;
    }
    __syncthreads();
    return code;
}

// ------------------------------------------ wave-cooperative block inverse
// Inclusive prefix sums of the residuals of one block, lane = segment of
// 8 slots (3D: row (y, z) = (lane % 8, lane / 8); 2D: x from 8 (lane % 4),
// y = lane / 4; 1D: x from 8 lane).
template <int ND>
__device__ __forceinline__ void block_prefix(int32_t (&v)[8], uint32_t lane) {
#pragma unroll
    for (int i = 1; i < 8; i++) v[i] += v[i - 1];
    if (ND == 1) {
        // carry from the lanes before along x
        const uint32_t tot = (uint32_t)v[7];
        const uint32_t excl = wave_incl_scan(tot) - tot;
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] += (int32_t)excl;
        return;
    }
    if (ND == 2) {
        // x: carry from the (up to 3) lanes before in the same row of 4
        int32_t tot = v[7], carry = 0;
#pragma unroll
        for (int d = 1; d < 4; d <<= 1) {
            const int32_t o = __shfl_up(tot, d, 4);
            if ((lane & 3) >= (uint32_t)d) tot += o;
        }
        carry = tot - v[7];
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] += carry;
        // y: lanes 4 apart
#pragma unroll
        for (int d = 4; d < 64; d <<= 1) {
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int32_t o = __shfl_up(v[i], d, 64);
                if (lane >= (uint32_t)d) v[i] += o;
            }
        }
        return;
    }
    // 3D (the whole wave active): y within the 8 lanes of one z by DPP row
    // shifts (lanes whose source lies in the other z of the 16-lane row
    // masked), then z over lane bits 3-5 by butterflies: the partner's
    // running total of its 2^k z-levels, lane ^ 8 by a DPP row rotation,
    // lane ^ 16 and lane ^ 32 by the permlane swaps, added to the prefix of
    // the lanes in the upper half
    const uint32_t ly = lane & 7;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        // every cross-lane read by all lanes, outside the selects
        uint32_t a = (uint32_t)v[i];
        const uint32_t y1 = dpp32<0x111, 0xf>(a);
        a += ly >= 1 ? y1 : 0u;
        const uint32_t y2 = dpp32<0x112, 0xf>(a);
        a += ly >= 2 ? y2 : 0u;
        const uint32_t y4 = dpp32<0x114, 0xf>(a);
        a += ly >= 4 ? y4 : 0u;
        uint32_t tot = a;
        uint32_t o = dpp32<0x128, 0xf>(tot);  // lane ^ 8
        a += (lane & 8) ? o : 0u;
        tot += o;
        const auto s16 = __builtin_amdgcn_permlane16_swap(tot, tot, false, false);
        o = (lane & 16) ? s16[0] : s16[1];  // lane ^ 16
        a += (lane & 16) ? o : 0u;
        tot += o;
        const auto s32 = __builtin_amdgcn_permlane32_swap(tot, tot, false, false);
        o = (lane & 32) ? s32[0] : s32[1];  // lane ^ 32
        a += (lane & 32) ? o : 0u;
        v[i] = (int32_t)a;
    }
}


// ------------------------------------------------ bit-shuffle plane words
// Symbols of the bit-shuffle codec: a block's 512 slots form 16 groups of
// 32 symbols, each group 10 plane words (word p: bit p of the group's
// symbols, symbol j in bit j), word k = 10 group + plane.
constexpr int kShufGroups = kBlockElems / 32;
constexpr int kShufWords = kShufGroups * kPlanes;  // 160
// Slot of a block in the fused encoder's staging: 5 mask words, then the
// kept words in order (at most 160), 256 words per block.
constexpr int kShufSlot = 256;

// Symbol of a quantisation code: 0 (outlier) -> 1023, c -> zigzag(c - 512).
__device__ __forceinline__ uint32_t fold_code(uint32_t code) {
    const int32_t d = (int32_t)code - kRadius;
    const uint32_t z = ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
    return code ? z : kSymOutlier;
}

// 8 x 8 bit-matrix transpose (three delta swaps, Hacker's Delight 7-3):
// bit c of byte r moves to bit r of byte c.
__device__ __forceinline__ uint64_t transpose8(uint64_t x) {
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    return x ^ t ^ (t << 28);
}

// The plane words of one block, the whole wave active, lane = the 8
// consecutive slots 8 lane + j (symbols sym[j]; 4 lanes per group): each
// lane transposes its symbols' bits to one byte per plane, the quad's
// bytes are transposed across lanes (DPP swaps with lane ^ 1 and lane ^ 2,
// byte permutes) into the group's words, and a per-wave LDS buffer W of
// kShufWords returns them as word k = lane + 64 j in w[j].
__device__ __forceinline__ void shuffle_words(const uint32_t sym[8], uint32_t lane, uint32_t* W, uint32_t w[3]) {
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        lo |= (uint64_t)(sym[j] & 0xFFu) << (8 * j);
        hi |= (uint64_t)(sym[j] >> 8) << (8 * j);
    }
    const uint64_t tl = transpose8(lo), th = transpose8(hi);
    const uint32_t k4 = lane & 3;
    const uint32_t sel1 = (k4 & 1) ? 0x03070105u : 0x06020400u;
    const uint32_t sel2 = (k4 & 2) ? 0x03020706u : 0x05040100u;
    auto quad_t = [&](uint32_t v) {
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // lane ^ 1
        const uint32_t t1 = __builtin_amdgcn_perm(p1, v, sel1);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)t1, 0x4E, 0xF, 0xF, false);  // lane ^ 2
        return __builtin_amdgcn_perm(p2, t1, sel2);
    };
    // lane 4 g + k: the words of planes k, 4 + k (and 8 + k for k < 2)
    const uint32_t wa = quad_t((uint32_t)tl), wb = quad_t((uint32_t)(tl >> 32)), wc = quad_t((uint32_t)th);
    const uint32_t g0 = (lane >> 2) * kPlanes;
    W[g0 + k4] = wa;
    W[g0 + 4 + k4] = wb;
    if (k4 < 2) W[g0 + 8 + k4] = wc;
    __builtin_amdgcn_wave_barrier();
    w[0] = W[lane];
    w[1] = W[64 + lane];
    w[2] = lane < kShufWords - 128 ? W[128 + lane] : 0u;
    __builtin_amdgcn_wave_barrier();
}

}  // namespace fz
