// Decompression (FZModules Sec. 1 and Sec. 3.3.1 describe it as Huffman
// decoding of the quantisation codes plus scattering of the outliers into
// the reconstruction; the inverse of the Lorenzo predictor is a prefix sum):
//   k_reset_lut    - per-call reset; validates the code lengths, builds a
//                    4096-entry table
//   k_decode       - one lane per block: table-driven Huffman decode from a
//                    register bit buffer fed through a per-lane LDS ring,
//                    outlier overwrite, in-block prefix sums (inverse
//                    Lorenzo), dequantisation, row stores - codes never
//                    leave registers
//   k_patch        - lossless patches written over the reconstruction
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// ----------------------------------------------------------- decode table
// Entry for the 12-bit prefix v: ((symbol ^ radius) << 6) | length of the
// codeword that v starts with.  The length sits in the six bits a 64-bit
// shift takes its amount from, so the entry itself shifts the bit buffer,
// and bits 6..15 read as a signed 10-bit field are symbol - radius, the
// residual.  The lengths must describe a complete code (Kraft sum exactly
// 1, every length 1..12, at least two symbols).
// Executed by one whole workgroup of 1024 threads (thread = symbol).
__device__ __forceinline__ void build_lut(const uint8_t* __restrict__ lensp, uint16_t* __restrict__ lut,
                                          Misc* misc) {
    __shared__ CanonShared cs;
    __shared__ uint32_t rk[16], ru[16], rb[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t len = (lensp[t >> 1] >> (4 * (t & 1))) & 15u;
    const uint32_t bad = len > (uint32_t)kLmax ? 1u : 0u;
    uint32_t kr = (len && !bad) ? (1u << (kLmax - len)) : 0u;
    uint32_t used = len ? 1u : 0u;
    uint32_t bb = bad;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        kr += __shfl_xor(kr, d, 64);
        used += __shfl_xor(used, d, 64);
        bb += __shfl_xor(bb, d, 64);
    }
    if (lane == 0) {
        rk[wave] = kr;
        ru[wave] = used;
        rb[wave] = bb;
    }
    __syncthreads();
    uint32_t K = 0, U = 0, B = 0;
    for (int w = 0; w < 16; w++) {
        K += rk[w];
        U += ru[w];
        B += rb[w];
    }
    const bool ok = B == 0 && K == (uint32_t)kLut && U >= 2;
    if (!ok) {
        if (t == 0) atomicOr(&misc->flags, F_CORRUPT);
        for (uint32_t v = t; v < (uint32_t)kLut; v += 1024) lut[v] = 0;
        return;
    }
    canonical_code(len, cs);
    for (uint32_t v = t; v < (uint32_t)kLut; v += 1024) {
        uint16_t e = 0;
        for (int L = 1; L <= kLmax; L++) {
            const uint32_t c = cs.count[L];
            if (!c) continue;
            const uint32_t end = (cs.first[L] + c) << (kLmax - L);
            if (v < end) {
                const uint32_t idx = (v >> (kLmax - L)) - cs.first[L];
                e = (uint16_t)(((cs.sorted[cs.offset[L] + idx] ^ (uint32_t)kRadius) << 6) | (uint32_t)L);
                break;
            }
        }
        lut[v] = e;
    }
}

// The decompression's first kernel: the per-call reset (Misc by workgroup
// 0, the arrays by the whole grid) and the decode table, built by
// workgroup 0 once its reset of Misc is visible to its threads (the table
// build may flag a corrupt code in Misc).
__global__ __launch_bounds__(1024) void k_reset_lut(Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1,
                                                    uint64_t* d2, uint32_t n2, uint64_t* d3, uint32_t n3,
                                                    uint64_t off_chunks, uint64_t off_stream, uint64_t nreg,
                                                    const uint8_t* __restrict__ lensp, uint16_t* __restrict__ lut) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) reset_misc(misc, off_chunks, off_stream, nreg);
    clear_scratch(gid, gridDim.x * blockDim.x, hist, d1, n1, d2, n2, d3, n3);
    if (blockIdx.x != 0) return;
    __syncthreads();
    build_lut(lensp, lut, misc);
}

// ----------------------------------------------------------------- decode
// Each lane decodes one block.  The lane's part of the stream flows
//   HBM --(16-byte chunks, two chunks ahead, registers)--> LDS ring of 4
//   chunks --(one word ahead)--> 64-bit bit buffer in registers
// so the dependent chain per codeword is one table lookup and a shift; the
// global loads are waited for only when a chunk is written to the ring, two
// chunks after they were issued.
constexpr int kDecLanes = 256;  // lanes (blocks) per workgroup
constexpr int kRing = 16;       // ring words per lane (4 chunks of 4)

struct LaneDec {
    const uint4* chunks;  // stream as 16-byte chunks
    uint32_t nchunks;
    uint32_t* ring;       // &RING[lane]; ring word k at ring[k * kDecLanes]
    uint32_t w;           // absolute index of the next word to feed
    uint32_t nw;          // that word
    uint64_t buf;         // next stream bits, most significant first
    uint32_t nb;          // valid bits in buf
    uint4 pend;           // the chunk after the ring's newest, in flight

    __device__ __forceinline__ uint4 load_chunk(uint32_t k) const {
        return chunks[k < nchunks ? k : nchunks - 1];
    }
    __device__ __forceinline__ void put_chunk(uint32_t k, const uint4& v) {
        uint32_t* r = ring + ((k & 3) * 4) * kDecLanes;
        r[0] = v.x;
        r[kDecLanes] = v.y;
        r[2 * kDecLanes] = v.z;
        r[3 * kDecLanes] = v.w;
    }
    // entering chunk c: chunk c + 1 goes to the ring, chunk c + 2 is issued
    __device__ __forceinline__ void boundary(uint32_t c) {
        put_chunk(c + 1, pend);
        pend = load_chunk(c + 2);
    }
    __device__ __forceinline__ void advance() {
        w++;
        if ((w & 3) == 0) boundary(w >> 2);
        nw = ring[(w & (kRing - 1)) * kDecLanes];
    }
    __device__ __forceinline__ void init(uint64_t start) {
        const uint32_t w0 = (uint32_t)(start >> 5), c = w0 >> 2;
        // the ring holds the current chunk and the next; the one after is
        // in flight
        put_chunk(c, load_chunk(c));
        put_chunk(c + 1, load_chunk(c + 1));
        pend = load_chunk(c + 2);
        w = w0;
        nw = ring[(w & (kRing - 1)) * kDecLanes];
        buf = (uint64_t)nw << 32;
        advance();
        buf |= nw;
        advance();
        const uint32_t skip = (uint32_t)(start & 31);
        buf <<= skip;
        nb = 64 - skip;
    }
    // make at least 33 bits available (two codewords of <= 12 bits follow)
    __device__ __forceinline__ void refill() {
        if (nb <= 32) {
            buf |= (uint64_t)nw << (32 - nb);
            nb += 32;
            advance();
        }
    }
    // bits consumed since `start`: the words fed so far end at bit 32 w,
    // nb of them are still buffered
    __device__ __forceinline__ uint64_t consumed(uint64_t start) const {
        return (uint64_t)w * 32 - nb - start;
    }
};

// Residual of a table entry (symbol - radius; -radius for an outlier code).
__device__ __forceinline__ int32_t entry_residual(uint32_t e) { return (int32_t)(e << 16) >> 22; }

// One codeword: returns the table entry; a lane with valid == false
// consumes nothing.
__device__ __forceinline__ uint32_t dec_sym(LaneDec& ld, const uint16_t* LUT, bool valid) {
    const uint32_t e = LUT[(uint32_t)(ld.buf >> (64 - kLmax))];
    const uint32_t len = valid ? (e & 63u) : 0u;
    ld.buf <<= len;
    ld.nb -= len;
    return e;
}

// The block's outliers: the k-th outlier code of a block takes the k-th
// entry of the block's part of the position-sorted list.  The next value is
// prefetched into a register; positions are checked in aggregate (a hash
// sum over the codes met against one over the list, and sortedness of the
// list), not one by one.
struct OutQ {
    const int32_t* oval;
    uint64_t n_out;
    uint32_t oi;    // list index of the next outlier
    int32_t next;   // its value
    uint64_t hash;  // sum of outlier_term over the outlier codes met
    __device__ __forceinline__ void init(const int32_t* v, uint64_t n, uint32_t first) {
        oval = v;
        n_out = n;
        oi = first;
        hash = 0;
        next = n ? v[first < n ? first : n - 1] : 0;
    }
    __device__ __forceinline__ int32_t take(uint32_t pos) {
        const int32_t d = next;
        hash += outlier_term(pos);
        oi++;
        if (n_out) next = oval[(uint64_t)oi < n_out ? oi : (uint32_t)(n_out - 1)];
        return d;
    }
};

// Decode one row of 8 values (the first nvalid are real) into d[].
__device__ __forceinline__ void dec_row8(LaneDec& ld, const uint16_t* LUT, uint32_t nvalid, uint32_t pos0,
                                         OutQ& oq, int32_t d[8]) {
#pragma unroll
    for (int i = 0; i < 8; i++) {
        if ((i & 1) == 0) ld.refill();
        const bool valid = (uint32_t)i < nvalid;
        const uint32_t e = dec_sym(ld, LUT, valid);
        const int32_t r = entry_residual(e);
        d[i] = valid ? r : 0;
        if (valid && r == -kRadius) d[i] = oq.take(pos0 + i);
    }
}

// Workgroup totals of the outlier consistency data to Misc (called by all
// 256 threads at the end of a decoder; one pair of atomics per workgroup).
// `red` is LDS the caller no longer needs (12 words), reused after a
// barrier.
__device__ __forceinline__ void outlier_totals(uint32_t t, bool active, const OutQ& oq, uint32_t oi0,
                                               Misc* misc, uint32_t* red) {
    uint32_t c = active ? oq.oi - oi0 : 0u;
    uint64_t h = active ? oq.hash : 0ull;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        c += __shfl_xor(c, d, 64);
        h += __shfl_xor(h, d, 64);
    }
    __syncthreads();
    if ((t & 63) == 0) {
        const uint32_t w = t >> 6;
        red[3 * w] = c;
        red[3 * w + 1] = (uint32_t)h;
        red[3 * w + 2] = (uint32_t)(h >> 32);
    }
    __syncthreads();
    if (t == 0) {
        c = 0;
        h = 0;
        for (int w = 0; w < 4; w++) {
            c += red[3 * w];
            h += ((uint64_t)red[3 * w + 2] << 32) | red[3 * w + 1];
        }
        if (c) {
            atomicAdd(&misc->code0_count, c);
            atomicAdd((unsigned long long*)&misc->ohash_dec, (unsigned long long)h);
        }
    }
}

// Blocks the fast kernels take (full blocks) are skipped when skip is set.
__device__ __forceinline__ bool is_interior(const BlockInfo& bi, const uint32_t ib[3]) {
    return bi.bx < ib[0] && bi.by < ib[1] && bi.bz < ib[2];
}

template <int ND>
__global__ __launch_bounds__(256) void k_decode(
    Geom g, const uint32_t* __restrict__ stream, uint64_t nwords, const uint64_t* __restrict__ off,
    const uint16_t* __restrict__ chunks, const uint16_t* __restrict__ lut_g, const uint32_t* __restrict__ opos,
    const int32_t* __restrict__ oval, const uint2* __restrict__ oidx, uint64_t n_out, double e2,
    float* __restrict__ out, int vec, Misc* misc, int skip, uint32_t ib0, uint32_t ib1, uint32_t ib2) {
    __shared__ uint16_t LUT[kLut];
    __shared__ uint32_t RING[kDecLanes * kRing];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLut; i += 256) LUT[i] = lut_g[i];
    __syncthreads();
    const uint32_t b0 = blockIdx.x * 256 + t;
    const uint32_t b = b0 < g.nblocks ? b0 : g.nblocks - 1;  // inactive lanes idle until the final reduction
    const BlockInfo info = block_info(g, b);
    const uint32_t ib[3] = {ib0, ib1, ib2};
    const bool active = b0 < g.nblocks && !(skip && is_interior(info, ib));
    const uint64_t start = off[b];
    LaneDec ld;
    ld.chunks = reinterpret_cast<const uint4*>(stream);
    ld.nchunks = (uint32_t)((nwords + 3) / 4);  // >= 1: the host rejects an empty stream
    ld.ring = &RING[t];
    ld.init(active ? start : 0);
    OutQ oq;
    const uint32_t oi0 = n_out ? oidx[b].x : 0;
    oq.init(oval, n_out, oi0);
    bool bad = false;
    const uint32_t pos_b = b * kBlockElems;
    auto deq = [&](int32_t q) -> float { return (float)((double)q * e2); };
    auto store8 = [&](uint64_t idx, const float* v, uint32_t nvalid) {
        if (nvalid == 8 && vec) {
            f32x4* p = reinterpret_cast<f32x4*>(out + idx);
            f32x4 a = {v[0], v[1], v[2], v[3]};
            f32x4 c = {v[4], v[5], v[6], v[7]};
            __builtin_nontemporal_store(a, p);
            __builtin_nontemporal_store(c, p + 1);
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++)
                if (i < (int)nvalid) out[idx + i] = v[i];
        }
    };

    if (!active) {
        // nothing to decode
    } else if (ND == 3) {
        // q(x, y, z) = sum over the box; kept as the previous plane qp,
        // the column sums pr of this plane and the row sum rs
        int32_t qp[64];
#pragma unroll
        for (int i = 0; i < 64; i++) qp[i] = 0;
        const uint64_t x0 = (uint64_t)info.bx * 8;
        for (uint32_t z = 0; z < info.ez; z++) {
            int32_t pr[8];
#pragma unroll
            for (int i = 0; i < 8; i++) pr[i] = 0;
#pragma unroll
            for (int y = 0; y < 8; y++) {
                if ((uint32_t)y < info.ey) {
                    int32_t d[8];
                    dec_row8(ld, LUT, info.ex, pos_b + 8 * y + 64 * z, oq, d);
                    int32_t rs = 0;
                    float v[8];
#pragma unroll
                    for (int x = 0; x < 8; x++) {
                        rs += d[x];
                        pr[x] += rs;
                        qp[y * 8 + x] += pr[x];
                        v[x] = deq(qp[y * 8 + x]);
                    }
                    const uint64_t yg = (uint64_t)info.by * 8 + y, zg = (uint64_t)info.bz * 8 + z;
                    store8(x0 + (uint64_t)g.n[0] * (yg + (uint64_t)g.n[1] * zg), v, info.ex);
                }
            }
        }
    } else if (ND == 2) {
        int32_t qp[32];
#pragma unroll
        for (int i = 0; i < 32; i++) qp[i] = 0;
        for (uint32_t y = 0; y < info.ey; y++) {
            int32_t rs = 0;
            const uint64_t row = (uint64_t)info.bx * 32 + (uint64_t)g.n[0] * ((uint64_t)info.by * 16 + y);
#pragma unroll
            for (int x8 = 0; x8 < 4; x8++) {
                if ((uint32_t)(x8 * 8) < info.ex) {
                    int32_t d[8];
                    const uint32_t nv = min(8u, info.ex - x8 * 8);
                    dec_row8(ld, LUT, nv, pos_b + 32 * y + 8 * x8, oq, d);
                    float v[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        rs += d[i];
                        qp[x8 * 8 + i] += rs;
                        v[i] = deq(qp[x8 * 8 + i]);
                    }
                    store8(row + x8 * 8, v, nv);
                }
            }
        }
    } else {
        int32_t acc = 0;
        const uint64_t row = (uint64_t)b * kBlockElems;
        for (uint32_t i0 = 0; i0 < info.ex; i0 += 8) {
            int32_t d[8];
            const uint32_t nv = min(8u, info.ex - i0);
            dec_row8(ld, LUT, nv, pos_b + i0, oq, d);
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                acc += d[i];
                v[i] = deq(acc);
            }
            store8(row + i0, v, nv);
        }
    }
    if (active && ld.consumed(start) != chunks[b]) bad = true;
    if (bad) atomicOr(&misc->flags, F_CORRUPT);
    outlier_totals(t, active, oq, oi0, misc, reinterpret_cast<uint32_t*>(LUT));
}

// ------------------------------------------------ fast decode of full blocks
// Full (interior) blocks of a field whose rows are 16-byte aligned.  The
// lanes of a wave move through their blocks in lockstep, 8 codewords (one
// row) at a time, and every lane issues exactly one 16-byte stream load and
// one 16-byte outlier-value load per row, real or a dummy, landed in its
// LDS rings two rows later.  With a fixed number of memory operations per
// row, each wait covers only data requested two rows earlier; the codeword
// chain itself touches LDS and registers only.  Rings hold 4 chunks: a
// chunk is fetched only when the chunk it replaces can no longer be read.
constexpr int kORing = 16;  // outlier values per lane in LDS

struct FastDec {
    const uint4* S;       // stream chunks
    uint32_t nch;         // number of stream chunks (>= 1)
    uint32_t* sr;         // &SRING[lane]; ring word k at sr[k * kDecLanes]
    uint32_t w, s;        // position of the next unread bit: word, bit in it
    uint32_t sF, sEnd;    // next chunk to fetch; last chunk worth fetching
    uint4 sX[2];          // chunks in flight (by row parity) and their
    uint32_t sXi[2];      // indices (~0: dummy)
    const uint4* O;       // outlier values as chunks (16-byte aligned list)
    uint32_t och;         // number of outlier chunks
    const int32_t* oval;
    uint64_t n_out;
    uint32_t* orr;        // &ORING[lane]
    uint32_t oi, oend;    // next outlier index, end of the block's outliers
    uint32_t oF, oL;      // next outlier chunk to fetch; values < oL landed
    uint4 oX[2];
    uint32_t oXi[2];
    uint64_t hash;

    __device__ __forceinline__ void sput(uint32_t k, const uint4& v) {
        uint32_t* r = sr + ((k & 3) * 4) * kDecLanes;
        r[0] = v.x;
        r[kDecLanes] = v.y;
        r[2 * kDecLanes] = v.z;
        r[3 * kDecLanes] = v.w;
    }
    __device__ __forceinline__ void oput(uint32_t k, const uint4& v) {
        uint32_t* r = orr + ((k & 3) * 4) * kDecLanes;
        r[0] = v.x;
        r[kDecLanes] = v.y;
        r[2 * kDecLanes] = v.z;
        r[3 * kDecLanes] = v.w;
    }
    __device__ __forceinline__ uint4 sload(uint32_t k) const { return S[k < nch ? k : nch - 1]; }

    __device__ __forceinline__ void init(uint64_t start, uint32_t bits, const int32_t* ov, uint64_t nout,
                                         uint32_t first, uint32_t count) {
        const uint32_t w0 = (uint32_t)(start >> 5), c0 = w0 >> 2;
        const uint4 a = sload(c0), b = sload(c0 + 1), c = sload(c0 + 2);
        oval = ov;
        n_out = nout;
        oi = first;
        oend = first + count;
        const uint32_t q0 = first >> 2;
        const bool any = count != 0 && nout != 0;
        och = (uint32_t)((nout + 3) / 4);
        const uint32_t qa = q0 < och ? q0 : och - 1, qb = q0 + 1 < och ? q0 + 1 : och - 1;
        const uint4 oa = any ? O[qa] : S[0], ob = any ? O[qb] : S[0];
        sput(c0, a);
        sput(c0 + 1, b);
        sput(c0 + 2, c);
        sF = c0 + 3;
        sEnd = (uint32_t)((start + bits) >> 7) + 1;
        oput(q0, oa);
        oput(q0 + 1, ob);
        oF = q0 + 2;
        oL = any ? 4 * (q0 + 2) : 0;
        sXi[0] = sXi[1] = oXi[0] = oXi[1] = 0xFFFFFFFFu;
        hash = 0;
        w = w0;
        s = (uint32_t)(start & 31);
    }
    // row prologue for row parity P: land what row - 2 fetched, fetch anew
    template <int P>
    __device__ __forceinline__ void row_io() {
        if (sXi[P] != 0xFFFFFFFFu) sput(sXi[P], sX[P]);
        if (oXi[P] != 0xFFFFFFFFu) {
            oput(oXi[P], oX[P]);
            oL = 4 * (oXi[P] + 1);
        }
        const bool sreal = sF <= (w >> 2) + 3 && sF <= sEnd;
        sX[P] = sload(sreal ? sF : 0);
        sXi[P] = sreal ? sF : 0xFFFFFFFFu;
        sF += sreal ? 1u : 0u;
        const bool oreal = oF <= (oi >> 2) + 3 && 4 * oF < oend;
        const uint4* osrc = oreal ? &O[oF] : &S[0];
        oX[P] = *osrc;
        oXi[P] = oreal ? oF : 0xFFFFFFFFu;
        oF += oreal ? 1u : 0u;
    }
    // The 64 stream bits from the current position, most significant first,
    // read from the three ring words that hold them (four codewords of at
    // most 12 bits fit, so a row refills twice instead of topping up a word
    // at a time; the words past the last codeword may hold stale ring data,
    // which no codeword reaches).
    __device__ __forceinline__ uint64_t window() const {
        const uint32_t a = sr[(w & (kRing - 1)) * kDecLanes];
        const uint32_t b = sr[((w + 1) & (kRing - 1)) * kDecLanes];
        const uint32_t c = sr[((w + 2) & (kRing - 1)) * kDecLanes];
        const uint64_t hi = (((uint64_t)a << 32) | b) << s;
        return hi | ((((uint64_t)c) << s) >> 32);
    }
    __device__ __forceinline__ void skip(uint32_t used) {
        s += used;
        w += s >> 5;
        s &= 31u;
    }
    // 8 codewords of one row.  An outlier value not landed yet (a burst,
    // or a corrupt container) is fetched after the row by the whole wave,
    // so no global load sits inside the codeword loop.
    __device__ __forceinline__ void row8(const uint16_t* LUT, uint32_t pos0, int32_t d[8]) {
        // the codeword chain first, without branches: two halves of four
        // codewords, each from a fresh 64-bit window
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint64_t buf = window();
            uint32_t used = 0;
#pragma unroll
            for (int i = 4 * h; i < 4 * h + 4; i++) {
                const uint32_t e = LUT[(uint32_t)(buf >> (64 - kLmax))];
                buf <<= (e & 63u);
                used += e & 63u;
                d[i] = entry_residual(e);
            }
            skip(used);
        }
        // code 0 (an outlier) is the only one that decodes to -radius: a
        // wave whose row holds none skips the outlier handling
        const int32_t mn = min(min(min(d[0], d[1]), min(d[2], d[3])), min(min(d[4], d[5]), min(d[6], d[7])));
        if (!__ballot(mn == -kRadius)) return;
        // the row's outlier mask; the k-th outlier of the row takes list
        // entry oi + k, read from the ring when landed (index below oL),
        // without a branch per value
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) m |= (d[i] == -kRadius ? 1u : 0u) << i;
        const uint32_t cnt = (uint32_t)__popc(m);
        hash += pos_hash(pos0 >> 3) * (uint64_t)m;  // the row's outlier_term sum (pos0 % 8 == 0)
        const uint32_t nland = oL > oi ? min(cnt, oL - oi) : 0u;
        uint32_t mmask = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t k = (uint32_t)__popc(m & ((1u << i) - 1u));
            const int32_t v = (int32_t)orr[((oi + k) & (kORing - 1)) * kDecLanes];
            const bool out = (m >> i) & 1u;
            const bool land = k < nland;
            d[i] = out ? (land ? v : 0) : d[i];
            mmask |= (out && !land) ? (1u << i) : 0u;
        }
        const uint32_t m0 = oi + nland;
        oi += cnt;
        if (__ballot(mmask != 0)) {
#pragma unroll
            for (int i = 0; i < 8; i++)
                if (mmask & (1u << i)) {
                    const uint32_t k = m0 + __popc(mmask & ((1u << i) - 1u));
                    d[i] = n_out ? oval[(uint64_t)k < n_out ? k : (uint32_t)(n_out - 1)] : 0;
                }
            // wait here (vmcnt 0), so that rows without a miss carry no wait
            __builtin_amdgcn_s_waitcnt(0x0F70);
        }
    }
    __device__ __forceinline__ uint64_t consumed(uint64_t start) const {
        return (uint64_t)w * 32 + s - start;
    }
};

// RES = false: inverse Lorenzo, dequantisation and rows of floats (two
// float4 stores per row when VEC, rows 16-byte aligned; else eight dword
// stores); RES = true: residuals (int32, block-major) for the mapped decoder.
// MAP (with RES = false): each lane's block has its own predictor (the map,
// or fixed_pred >= 0): a first-order block is finished as above, a
// regression block adds its fixed-point plane to the residuals in place of
// the prefix sums, and a second-order block writes its residuals (its row
// stores carry first-order values that k_inverse_wave overwrites).
template <int ND, bool RES, bool VEC, bool XT = false, bool MAP = false, bool ROW = false>
__global__ __launch_bounds__(256) void k_decode_fast(Geom g, uint32_t ib0, uint32_t ib1, uint32_t nint,
                                                     const uint32_t* __restrict__ stream, uint64_t nwords,
                                                     const uint64_t* __restrict__ off,
                                                     const uint16_t* __restrict__ chunks,
                                                     const uint16_t* __restrict__ lut_g,
                                                     const int32_t* __restrict__ oval,
                                                     const uint2* __restrict__ oidx, uint64_t n_out, double e2,
                                                     float* __restrict__ out, int32_t* __restrict__ res, Misc* misc,
                                                     int fixed_pred, const uint8_t* __restrict__ bpred,
                                                     const uint64_t* __restrict__ reg_idx,
                                                     const int32_t* __restrict__ coefs, uint64_t nreg) {
    __shared__ uint16_t LUT[kLut];
    __shared__ uint32_t SRING[kDecLanes * kRing];
    __shared__ uint32_t ORING[kDecLanes * kORing];
    // XT (3D): a wave's rows of a step (consecutive blocks along x, one run,
    // or two where the wave wraps to the next row of blocks) are staged here
    // and stored so that lanes 2m and 2m+1 write block m's whole row: each
    // store instruction writes 32 rows back to back
    __shared__ f32x4 XS[XT ? 4 * 128 : 1];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLut; i += 256) LUT[i] = lut_g[i];
    __syncthreads();
    const uint32_t i0 = blockIdx.x * 256 + t;
    const bool active = i0 < nint;
    const uint32_t ii = active ? i0 : nint - 1;
    const uint32_t ibx = ii % ib0, r1 = ii / ib0, iby = r1 % ib1, ibz = r1 / ib1;
    // XT: output offset of this block's first row, and of the first rows of
    // the two blocks whose halves this lane stores (lanes m and 32 + m of the
    // wave, m = lane / 2, half lane % 2); a step adds the same offset to all
    const uint64_t xown = (uint64_t)ibx * 8 + (uint64_t)g.n[0] * ((uint64_t)iby * 8 +
                                                                  (uint64_t)g.n[1] * ((uint64_t)ibz * 8));
    uint64_t xa1 = 0, xa2 = 0;
    if (XT) {
        const uint32_t lane = t & 63, lo = (uint32_t)xown, hi = (uint32_t)(xown >> 32);
        const uint32_t m1 = lane >> 1, m2 = 32 + (lane >> 1);
        xa1 = ((uint64_t)(uint32_t)__shfl((int)hi, (int)m1, 64) << 32 | (uint32_t)__shfl((int)lo, (int)m1, 64)) +
              4 * (lane & 1);
        xa2 = ((uint64_t)(uint32_t)__shfl((int)hi, (int)m2, 64) << 32 | (uint32_t)__shfl((int)lo, (int)m2, 64)) +
              4 * (lane & 1);
    }
    const uint32_t b = ibx + g.nb[0] * (iby + g.nb[1] * ibz);
    const uint64_t start = off[b];
    const uint32_t bits = chunks[b];
    const uint2 oe = n_out ? oidx[b] : make_uint2(0u, 0u);
    const uint32_t first = oe.x, count = oe.y - oe.x;
    FastDec fd;
    fd.S = reinterpret_cast<const uint4*>(stream);
    fd.nch = (uint32_t)((nwords + 3) / 4);
    fd.sr = &SRING[t];
    fd.orr = &ORING[t];
    fd.O = reinterpret_cast<const uint4*>(oval);
    fd.init(start, bits, oval, n_out, first, count);
    const uint32_t pos_b = b * kBlockElems;
    // MAP: this lane's predictor; a regression block's plane as
    // floor((A + Bx u + By v + Bz w + 128) / 256), u = 2 lx - (bs0 - 1), ...
    bool lreg = false, lsec = false;
    int64_t cA = 0, cX = 0, cY = 0, cZ = 0;
    if (MAP) {
        const uint32_t p = fixed_pred >= 0 ? (uint32_t)fixed_pred : bpred[b];
        lsec = p == 1;
        lreg = p == 2;
        if (lreg) {
            const uint64_t r = fixed_pred >= 0 ? b : reg_idx[b];
            if (r < nreg) {
                const int4 c = reinterpret_cast<const int4*>(coefs)[r];
                cA = c.x;
                cX = c.y;
                cY = c.z;
                cZ = c.w;
            } else if (active) {
                atomicOr(&misc->flags, F_CORRUPT);
            }
        }
    }
    // plane at (lx = 0, ly, lz) + 128, the step along x is 2 Bx
    auto plane_row = [&](int32_t ly, int32_t lz) -> int64_t {
        return cA + 128 - cX * (int64_t)(g.bs[0] - 1) + cY * (int64_t)(2 * ly - ((int32_t)g.bs[1] - 1)) +
               cZ * (int64_t)(2 * lz - ((int32_t)g.bs[2] - 1));
    };
    // ROW (with RES): residuals as raw int32 bits, row-major, through the
    // field's store path (out is the residual field)
    auto deq = [&](int32_t q) -> float { return ROW ? __int_as_float(q) : (float)((double)q * e2); };
    auto store8 = [&](uint64_t idx, const int32_t* q) {
        if (VEC) {
            f32x4* p = reinterpret_cast<f32x4*>(out + idx);
            const f32x4 a = {deq(q[0]), deq(q[1]), deq(q[2]), deq(q[3])};
            const f32x4 c = {deq(q[4]), deq(q[5]), deq(q[6]), deq(q[7])};
            if (XT) {
                const uint32_t lane = t & 63;
                f32x4* xs = &XS[(t >> 6) * 128];
                xs[2 * lane] = a;
                xs[2 * lane + 1] = c;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const f32x4 u = xs[lane], v = xs[64 + lane];
                // an inactive lane decodes the interior's last block (its
                // clamped index): its staged row is that block's own row
                const uint64_t roff = idx - xown;
                __builtin_nontemporal_store(u, reinterpret_cast<f32x4*>(out + xa1 + roff));
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(out + xa2 + roff));
            } else {
                __builtin_nontemporal_store(a, p);
                __builtin_nontemporal_store(c, p + 1);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++) __builtin_nontemporal_store(deq(q[i]), out + idx + i);
        }
    };
    auto store_res = [&](uint32_t pos0, const int32_t* d) {
        int4* dst = reinterpret_cast<int4*>(res + pos0);
        dst[0] = make_int4(d[0], d[1], d[2], d[3]);
        dst[1] = make_int4(d[4], d[5], d[6], d[7]);
    };
    if (ND == 3) {
        const uint64_t x0 = (uint64_t)ibx * 8;
        int32_t qp[64];
#pragma unroll
        for (int i = 0; i < 64; i++) qp[i] = 0;
        for (uint32_t z = 0; z < 8; z++) {
            int32_t pr[8];
#pragma unroll
            for (int i = 0; i < 8; i++) pr[i] = 0;
#pragma unroll
            for (int y = 0; y < 8; y++) {
                if (y & 1) fd.row_io<1>(); else fd.row_io<0>();
                int32_t d[8];
                const uint32_t pos0 = pos_b + 8 * y + 64 * z;
                fd.row8(LUT, pos0, d);
                if (RES && ROW) {
                    const uint64_t yg = (uint64_t)iby * 8 + y, zg = (uint64_t)ibz * 8 + z;
                    store8(x0 + (uint64_t)g.n[0] * (yg + (uint64_t)g.n[1] * zg), d);
                } else if (RES) {
                    store_res(pos0, d);
                } else {
                    int32_t rs = 0, q[8];
#pragma unroll
                    for (int x = 0; x < 8; x++) {
                        rs += d[x];
                        pr[x] += rs;
                        qp[y * 8 + x] += pr[x];
                        q[x] = qp[y * 8 + x];
                    }
                    if (MAP) {
                        if (lsec) store_res(pos0, d);
                        int64_t sv = plane_row(y, (int32_t)z);
#pragma unroll
                        for (int x = 0; x < 8; x++) {
                            const int32_t rq = (int32_t)((uint32_t)d[x] + (uint32_t)(int32_t)(sv >> 8));
                            q[x] = lreg ? rq : q[x];
                            sv += 2 * cX;
                        }
                    }
                    const uint64_t yg = (uint64_t)iby * 8 + y, zg = (uint64_t)ibz * 8 + z;
                    store8(x0 + (uint64_t)g.n[0] * (yg + (uint64_t)g.n[1] * zg), q);
                }
            }
        }
    } else if (ND == 2) {
        int32_t qp[32];
#pragma unroll
        for (int i = 0; i < 32; i++) qp[i] = 0;
        for (uint32_t y = 0; y < 16; y++) {
            int32_t rs = 0;
            const uint64_t row = (uint64_t)ibx * 32 + (uint64_t)g.n[0] * ((uint64_t)iby * 16 + y);
#pragma unroll
            for (int x8 = 0; x8 < 4; x8++) {
                if (x8 & 1) fd.row_io<1>(); else fd.row_io<0>();
                int32_t d[8];
                const uint32_t pos0 = pos_b + 32 * y + 8 * x8;
                fd.row8(LUT, pos0, d);
                if (RES && ROW) {
                    store8(row + x8 * 8, d);
                } else if (RES) {
                    store_res(pos0, d);
                } else {
                    int32_t q[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        rs += d[i];
                        qp[x8 * 8 + i] += rs;
                        q[i] = qp[x8 * 8 + i];
                    }
                    if (MAP) {
                        if (lsec) store_res(pos0, d);
                        int64_t sv = plane_row((int32_t)y, 0) + 2 * cX * (int64_t)(8 * x8);
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            const int32_t rq = (int32_t)((uint32_t)d[i] + (uint32_t)(int32_t)(sv >> 8));
                            q[i] = lreg ? rq : q[i];
                            sv += 2 * cX;
                        }
                    }
                    store8(row + x8 * 8, q);
                }
            }
        }
    } else {
        int32_t acc = 0;
        const uint64_t row = (uint64_t)b * kBlockElems;
        for (uint32_t s2 = 0; s2 < 32; s2++) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (h) fd.row_io<1>(); else fd.row_io<0>();
                int32_t d[8];
                const uint32_t i0s = 16 * s2 + 8 * h;
                fd.row8(LUT, pos_b + i0s, d);
                if (RES && ROW) {
                    store8(row + i0s, d);
                } else if (RES) {
                    store_res(pos_b + i0s, d);
                } else {
                    int32_t q[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        acc += d[i];
                        q[i] = acc;
                    }
                    if (MAP) {
                        if (lsec) store_res(pos_b + i0s, d);
                        int64_t sv = plane_row(0, 0) + 2 * cX * (int64_t)i0s;
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            const int32_t rq = (int32_t)((uint32_t)d[i] + (uint32_t)(int32_t)(sv >> 8));
                            q[i] = lreg ? rq : q[i];
                            sv += 2 * cX;
                        }
                    }
                    store8(row + i0s, q);
                }
            }
        }
    }
    bool bad = false;
    if (active && (fd.consumed(start) != bits || fd.oi != first + count)) bad = true;
    if (bad) atomicOr(&misc->flags, F_CORRUPT);
    OutQ oq;
    oq.oi = fd.oi;
    oq.hash = fd.hash;
    outlier_totals(t, active, oq, first, misc, reinterpret_cast<uint32_t*>(LUT));
}

// ---------------------------------------------- per-block predictor decode
// Containers whose blocks use the second-order Lorenzo or regression
// predictor decode in two steps: residuals per block to scratch (lane per
// block, same Huffman and outlier handling as k_decode), then one wave per
// block applies that block's inverse in LDS and writes the field.

// 2-bit predictor map of the container -> one byte per block
__global__ __launch_bounds__(256) void k_map_unpack(const uint8_t* __restrict__ map, uint32_t nblocks,
                                                    uint8_t* __restrict__ bpred, Misc* misc) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nblocks) return;
    const uint8_t v = (uint8_t)((map[b >> 2] >> (2 * (b & 3))) & 3u);
    if (v > 2) atomicOr(&misc->flags, F_CORRUPT);
    bpred[b] = v > 2 ? 0 : v;
}

template <int ND>
__global__ __launch_bounds__(256) void k_decode_res(Geom g, const uint32_t* __restrict__ stream, uint64_t nwords,
                                                    const uint64_t* __restrict__ off,
                                                    const uint16_t* __restrict__ chunks,
                                                    const uint16_t* __restrict__ lut_g,
                                                    const uint32_t* __restrict__ opos, const int32_t* __restrict__ oval,
                                                    const uint2* __restrict__ oidx, uint64_t n_out,
                                                    int32_t* __restrict__ res, Misc* misc, int skip, uint32_t ib0,
                                                    uint32_t ib1, uint32_t ib2, int rowmajor) {
    __shared__ uint16_t LUT[kLut];
    __shared__ uint32_t RING[kDecLanes * kRing];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLut; i += 256) LUT[i] = lut_g[i];
    __syncthreads();
    const uint32_t b0 = blockIdx.x * 256 + t;
    const uint32_t b = b0 < g.nblocks ? b0 : g.nblocks - 1;
    const BlockInfo info = block_info(g, b);
    const uint32_t ib[3] = {ib0, ib1, ib2};
    const bool active = b0 < g.nblocks && !(skip && is_interior(info, ib));
    const uint64_t start = off[b];
    LaneDec ld;
    ld.chunks = reinterpret_cast<const uint4*>(stream);
    ld.nchunks = (uint32_t)((nwords + 3) / 4);  // >= 1: the host rejects an empty stream
    ld.ring = &RING[t];
    ld.init(active ? start : 0);
    OutQ oq;
    const uint32_t oi0 = n_out ? oidx[b].x : 0;
    oq.init(oval, n_out, oi0);
    bool bad = false;
    const uint32_t pos_b = b * kBlockElems;
    if (active) {
        // rows of 8 along x in block order; residuals stored block-major, or
        // row-major (the real values only)
        for (uint32_t lz = 0; lz < info.ez; lz++)
            for (uint32_t ly = 0; ly < info.ey; ly++)
                for (uint32_t lx0 = 0; lx0 < info.ex; lx0 += 8) {
                    int32_t d[8];
                    const uint32_t nv = min(8u, info.ex - lx0);
                    const uint32_t pos0 = pos_b + lx0 + g.bs[0] * (ly + g.bs[1] * lz);
                    dec_row8(ld, LUT, nv, pos0, oq, d);
                    if (rowmajor) {
                        const uint64_t o = (uint64_t)info.bx * g.bs[0] + lx0 +
                                           (uint64_t)g.n[0] * ((uint64_t)info.by * g.bs[1] + ly +
                                                               (uint64_t)g.n[1] * ((uint64_t)info.bz * g.bs[2] + lz));
                        for (uint32_t i = 0; i < nv; i++) res[o + i] = d[i];
                    } else {
                        int4* dst = reinterpret_cast<int4*>(res + pos0);
                        dst[0] = make_int4(d[0], d[1], d[2], d[3]);
                        dst[1] = make_int4(d[4], d[5], d[6], d[7]);
                    }
                }
    }
    if (active && ld.consumed(start) != chunks[b]) bad = true;
    if (bad) atomicOr(&misc->flags, F_CORRUPT);
    outlier_totals(t, active, oq, oi0, misc, reinterpret_cast<uint32_t*>(LUT));
}

// The blocks the fast decoder leaves as residuals (edge blocks, and
// second-order blocks, or all blocks of a second-order container): one wave
// per block, lane = segment of 8 values along x (as the residual layout),
// the inverse as prefix sums in registers and across lanes (twice for the
// second order: prefix sums along different axes commute) or the
// regression plane added, then dequantised row stores.  With interior_done
// the interior blocks other than second-order ones are already written.
template <int ND>
__global__ __launch_bounds__(256) void k_inverse_wave(Geom g, const int32_t* __restrict__ res, int fixed_pred,
                                                      const uint8_t* __restrict__ bpred,
                                                      const uint64_t* __restrict__ reg_idx,
                                                      const int32_t* __restrict__ coefs, uint64_t nreg, double e2,
                                                      float* __restrict__ out, int vec, Misc* misc, uint32_t ib0,
                                                      uint32_t ib1, uint32_t ib2, int interior_done) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * 4;
    const uint32_t ib[3] = {ib0, ib1, ib2};
    bool bad = false;
    for (uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6); b < g.nblocks; b += nw) {
        const uint32_t p = fixed_pred >= 0 ? (uint32_t)fixed_pred : bpred[b];
        const BlockInfo bi = block_info(g, b);
        if (interior_done && p != 1 && is_interior(bi, ib)) continue;
        const int4* src = reinterpret_cast<const int4*>(res + (uint64_t)b * kBlockElems + 8 * lane);
        const int4 r0 = src[0], r1 = src[1];
        int32_t v[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
        uint32_t lx0, ly, lz;
        seg_coords<ND>(lane, lx0, ly, lz);
        if (p <= 1) {
            block_prefix<ND>(v, lane);
            if (p == 1) block_prefix<ND>(v, lane);
        } else {
            const uint64_t r = fixed_pred >= 0 ? b : reg_idx[b];
            int4 c = make_int4(0, 0, 0, 0);
            if (r < nreg) c = reinterpret_cast<const int4*>(coefs)[r];
            else bad = true;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int64_t sum = (int64_t)c.x + (int64_t)c.y * (2 * (int32_t)(lx0 + i) - ((int32_t)bi.ex - 1)) +
                                    (int64_t)c.z * (2 * (int32_t)ly - ((int32_t)bi.ey - 1)) +
                                    (int64_t)c.w * (2 * (int32_t)lz - ((int32_t)bi.ez - 1)) + 128;
                v[i] = (int32_t)((uint32_t)v[i] + (uint32_t)(int32_t)(sum >> 8));
            }
        }
        uint32_t nvalid;
        const uint64_t row = seg_index<ND>(g, bi, lane, nvalid);
        if (nvalid) {
            float f[8];
#pragma unroll
            for (int i = 0; i < 8; i++) f[i] = (float)((double)v[i] * e2);
            if (nvalid == 8 && vec && (row & 3) == 0) {
                f32x4* o4 = reinterpret_cast<f32x4*>(out + row);
                o4[0] = f32x4{f[0], f[1], f[2], f[3]};
                o4[1] = f32x4{f[4], f[5], f[6], f[7]};
            } else {
#pragma unroll
                for (int i = 0; i < 8; i++)
                    if ((uint32_t)i < nvalid) out[row + i] = f[i];
            }
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&misc->flags, F_CORRUPT);
}

// ------------------------------------------------------ outlier block index
// Per block, the list index of its first outlier (oidx[b].x) and one past
// its last (oidx[b].y), both left at zero for a block without outliers
// (cleared beforehand); the list must be strictly increasing; the sum of pos_hash
// over the list for the decode-side check.  Each thread takes groups of 4
// consecutive entries (one 16-byte load when the list is aligned), its
// neighbours at the group edges by two scalar loads that hit the cache
// lines of the adjacent lanes; the workgroup reduces its hash and flag and
// adds them with one atomic each (few workgroups, so few same-address
// atomics: these serialise at the memory side).
__device__ __forceinline__ void outlier_entry(uint64_t i, uint32_t p, bool has_prev, uint32_t prev, bool has_next,
                                              uint32_t next, uint32_t nblocks, uint2* __restrict__ oidx, uint64_t& h,
                                              bool& bad) {
    const uint32_t b = p >> 9;
    bad |= (has_prev && prev >= p) || b >= nblocks;
    h += outlier_term(p);
    if (b < nblocks && (!has_prev || (prev >> 9) != b)) oidx[b].x = (uint32_t)i;
    if (b < nblocks && (!has_next || (next >> 9) != b)) oidx[b].y = (uint32_t)(i + 1);
}

__global__ __launch_bounds__(256) void k_outlier_index(const uint32_t* __restrict__ opos, uint64_t n_out,
                                                       uint32_t nblocks, uint2* __restrict__ oidx, int vec,
                                                       Misc* misc) {
    const uint32_t t = threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t ngroups = (n_out + 3) / 4;
    uint64_t h = 0;
    bool bad = false;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + t; q < ngroups; q += stride) {
        const uint64_t i0 = 4 * q;
        uint32_t v[4];
        if (vec && i0 + 4 <= n_out) {
            const uint4 a = *reinterpret_cast<const uint4*>(opos + i0);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) v[k] = i0 + k < n_out ? opos[i0 + k] : 0u;
        }
        const uint32_t prev = i0 ? opos[i0 - 1] : 0u;
        const uint32_t next = i0 + 4 < n_out ? opos[i0 + 4] : 0u;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint64_t i = i0 + k;
            if (i < n_out)
                outlier_entry(i, v[k], i > 0, k ? v[k - 1] : prev, i + 1 < n_out, k < 3 ? v[k + 1] : next, nblocks,
                              oidx, h, bad);
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) h += __shfl_xor(h, d, 64);
    __shared__ uint64_t sh[4];
    if ((t & 63) == 0) sh[t >> 6] = h;
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (t == 0) {
        const uint64_t hs = sh[0] + sh[1] + sh[2] + sh[3];
        if (hs) atomicAdd((unsigned long long*)&misc->ohash_list, (unsigned long long)hs);
        if (any_bad) atomicOr(&misc->flags, F_CORRUPT);
    }
}

// ----------------------------------------------------------------- patches
template <int ND>
__global__ __launch_bounds__(256) void k_patch(Geom g, const uint32_t* __restrict__ ppos,
                                               const uint32_t* __restrict__ pbits, uint64_t n_pat,
                                               float* __restrict__ out, Misc* misc) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pat; i += stride) {
        const uint32_t pos = ppos[i];
        const uint32_t b = pos >> 9, local = pos & 511u;
        bool ok = b < g.nblocks && (i == 0 || ppos[i - 1] < pos);
        if (ok) {
            const BlockInfo info = block_info(g, b);
            uint32_t lx, ly, lz;
            if (ND == 3) { lx = local & 7; ly = (local >> 3) & 7; lz = local >> 6; }
            else if (ND == 2) { lx = local & 31; ly = local >> 5; lz = 0; }
            else { lx = local; ly = 0; lz = 0; }
            ok = lx < info.ex && ly < info.ey && lz < info.ez;
            if (ok) {
                const uint64_t x = (uint64_t)info.bx * g.bs[0] + lx;
                const uint64_t y = (uint64_t)info.by * g.bs[1] + ly;
                const uint64_t z = (uint64_t)info.bz * g.bs[2] + lz;
                out[x + (uint64_t)g.n[0] * (y + (uint64_t)g.n[1] * z)] = __uint_as_float(pbits[i]);
            }
        }
        if (!ok) atomicOr(&misc->flags, F_CORRUPT);
    }
}

// ------------------------------------------------------------- launchers
// Verbatim container: the raw floats.
__global__ __launch_bounds__(256) void k_copy(const uint8_t* __restrict__ src, float* __restrict__ dst, uint64_t n,
                                              int vec) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const float* s = reinterpret_cast<const float*>(src);
    if (vec) {
        const f32x4* s4 = reinterpret_cast<const f32x4*>(s);
        f32x4* d4 = reinterpret_cast<f32x4*>(dst);
        for (uint64_t i = gid; i < n / 4; i += stride) d4[i] = s4[i];
        for (uint64_t i = (n & ~3ull) + gid; i < n; i += stride) dst[i] = s[i];
    } else {
        for (uint64_t i = gid; i < n; i += stride) dst[i] = s[i];
    }
}

void launch_copy(hipStream_t st, const uint8_t* src, float* dst, uint64_t n) {
    const int vec = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
    uint64_t grid = (n / 4 + 255) / 256;
    if (grid > 2048) grid = 2048;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)grid), dim3(256), 0, st, src, dst, n, vec);
}

void launch_reset_lut(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2,
                      uint32_t n2, uint64_t* d3, uint32_t n3, uint64_t off_chunks, uint64_t off_stream,
                      uint64_t nreg, const uint8_t* lens_packed, uint16_t* lut) {
    uint32_t n = n1 > n2 ? n1 : n2;
    if (n3 > n) n = n3;
    uint32_t grid = (n + 1023) / 1024;
    if (grid < 1) grid = 1;
    if (grid > 256) grid = 256;
    hipLaunchKernelGGL(k_reset_lut, dim3(grid), dim3(1024), 0, st, misc, hist, d1, n1, d2, n2, d3, n3, off_chunks,
                       off_stream, nreg, lens_packed, lut);
}

namespace {
// Full blocks per axis (the fast kernels' domain).
struct Interior {
    uint32_t ib[3];
    uint32_t n;
};
Interior interior_of(const Geom& g) {
    Interior r;
    uint64_t n = 1;
    for (int a = 0; a < 3; a++) {
        r.ib[a] = a < (int)g.ndim ? g.n[a] / g.bs[a] : 1u;
        n *= r.ib[a];
    }
    r.n = (uint32_t)n;
    return r;
}

}  // namespace

// Outlier list index and list hash (before either decoder).
void launch_outlier_index(hipStream_t st, const Geom& g, const uint32_t* opos, uint64_t n_out, uint2* oidx,
                          Misc* misc) {
    // ofirst and oend were cleared by the call's reset kernel
    if (!n_out) return;
    // about 16 groups of 4 entries per thread, at most 1024 workgroups
    uint64_t og = (n_out + 4 * 16 * 256 - 1) / (4 * 16 * 256);
    if (og > 1024) og = 1024;
    const int vec = ((uintptr_t)opos & 15) == 0;
    hipLaunchKernelGGL(k_outlier_index, dim3((uint32_t)og), dim3(256), 0, st, opos, n_out, g.nblocks, oidx,
                       vec, misc);
}

void launch_decode(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                   const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                   const int32_t* oval, const uint2* oidx, uint64_t n_out, double e2, float* out,
                   int vec, Misc* misc) {
    const Interior I = interior_of(g);
    const bool fast = I.n > 0;
    if (fast) {
        const uint32_t fg = (I.n + 255) / 256;
#define FZ_FAST(NDV, V)                                                                                               \
    hipLaunchKernelGGL((k_decode_fast<NDV, false, V>), dim3(fg), dim3(256), 0, st, g, I.ib[0], I.ib[1], I.n, stream, \
                       stream_words, off, chunks, lut, oval, oidx, n_out, e2, out, (int32_t*)nullptr, misc, -1,      \
                       (const uint8_t*)nullptr, (const uint64_t*)nullptr, (const int32_t*)nullptr, (uint64_t)0)
        if (vec && g.ndim == 3 && I.ib[0] % 64 == 0) {
            // staged row stores where a wave covers one run of 64 blocks
            // along x (measured: 512^3 decodes 37% faster at 1e-2; a 384^3
            // field, 48 blocks per run and ~1.7 workgroups per CU, decoded
            // 8% slower staged than with the strided stores)
            hipLaunchKernelGGL((k_decode_fast<3, false, true, true>), dim3(fg), dim3(256), 0, st, g, I.ib[0], I.ib[1],
                               I.n, stream, stream_words, off, chunks, lut, oval, oidx, n_out, e2, out,
                               (int32_t*)nullptr, misc, -1, (const uint8_t*)nullptr, (const uint64_t*)nullptr,
                               (const int32_t*)nullptr, (uint64_t)0);
        } else if (vec) {
            if (g.ndim == 3) FZ_FAST(3, true);
            else if (g.ndim == 2) FZ_FAST(2, true);
            else FZ_FAST(1, true);
        } else {
            if (g.ndim == 3) FZ_FAST(3, false);
            else if (g.ndim == 2) FZ_FAST(2, false);
            else FZ_FAST(1, false);
        }
#undef FZ_FAST
    }
    if (fast && I.n == g.nblocks) return;
    const uint32_t grid = (g.nblocks + 255) / 256;
    const int skip = fast ? 1 : 0;
#define FZ_GEN(NDV)                                                                                                 \
    hipLaunchKernelGGL(k_decode<NDV>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut, opos, \
                       oval, oidx, n_out, e2, out, vec, misc, skip, I.ib[0], I.ib[1], I.ib[2])
    if (g.ndim == 3) FZ_GEN(3);
    else if (g.ndim == 2) FZ_GEN(2);
    else FZ_GEN(1);
#undef FZ_GEN
}

void launch_map_unpack(hipStream_t st, const uint8_t* map, uint32_t nblocks, uint8_t* bpred, Misc* misc) {
    hipLaunchKernelGGL(k_map_unpack, dim3((nblocks + 255) / 256), dim3(256), 0, st, map, nblocks, bpred, misc);
}

void launch_decode_pred(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                        const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                        const int32_t* oval, const uint2* oidx, uint64_t n_out, int32_t* res,
                        int fixed_pred, const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coefs,
                        uint64_t nreg, double e2, float* out, int vec, Misc* misc) {
    const Interior I = interior_of(g);
    // interior blocks: the fast decoder finishes first-order and regression
    // blocks (a second-order container only gets its residuals there)
    const bool fused = I.n && fixed_pred != 1;
    if (I.n) {
        const uint32_t fg = (I.n + 255) / 256;
#define FZ_ARGS                                                                                                     \
    dim3(fg), dim3(256), 0, st, g, I.ib[0], I.ib[1], I.n, stream, stream_words, off, chunks, lut, oval, oidx, n_out, \
        e2, out, res, misc, fixed_pred, bpred, reg_idx, coefs, nreg
        if (!fused) {
            if (g.ndim == 3) hipLaunchKernelGGL((k_decode_fast<3, true, false>), FZ_ARGS);
            else if (g.ndim == 2) hipLaunchKernelGGL((k_decode_fast<2, true, false>), FZ_ARGS);
            else hipLaunchKernelGGL((k_decode_fast<1, true, false>), FZ_ARGS);
        } else if (vec && g.ndim == 3 && I.ib[0] % 64 == 0) {
            hipLaunchKernelGGL((k_decode_fast<3, false, true, true, true>), FZ_ARGS);
        } else if (vec) {
            if (g.ndim == 3) hipLaunchKernelGGL((k_decode_fast<3, false, true, false, true>), FZ_ARGS);
            else if (g.ndim == 2) hipLaunchKernelGGL((k_decode_fast<2, false, true, false, true>), FZ_ARGS);
            else hipLaunchKernelGGL((k_decode_fast<1, false, true, false, true>), FZ_ARGS);
        } else {
            if (g.ndim == 3) hipLaunchKernelGGL((k_decode_fast<3, false, false, false, true>), FZ_ARGS);
            else if (g.ndim == 2) hipLaunchKernelGGL((k_decode_fast<2, false, false, false, true>), FZ_ARGS);
            else hipLaunchKernelGGL((k_decode_fast<1, false, false, false, true>), FZ_ARGS);
        }
#undef FZ_ARGS
    }
    const uint32_t grid = (g.nblocks + 255) / 256;
    const int skip = I.n ? 1 : 0;
    uint32_t wg = (g.nblocks + 3) / 4;
    if (wg > 8192) wg = 8192;
#define FZ_DRES(NDV)                                                                                                \
    if (I.n != g.nblocks)                                                                                           \
        hipLaunchKernelGGL(k_decode_res<NDV>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks,   \
                           lut, opos, oval, oidx, n_out, res, misc, skip, I.ib[0], I.ib[1], I.ib[2], 0);         \
    hipLaunchKernelGGL(k_inverse_wave<NDV>, dim3(wg), dim3(256), 0, st, g, res, fixed_pred, bpred, reg_idx, coefs,  \
                       nreg, e2, out, vec, misc, I.ib[0], I.ib[1], I.ib[2], fused ? 1 : 0)
    if (g.ndim == 3) {
        FZ_DRES(3);
    } else if (g.ndim == 2) {
        FZ_DRES(2);
    } else {
        FZ_DRES(1);
    }
#undef FZ_DRES
}

void launch_decode_residuals(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                             const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                             const int32_t* oval, const uint2* oidx, uint64_t n_out, int32_t* res, int vec,
                             Misc* misc) {
    // row-major int32 residuals through the field's store path (staged row
    // stores where a wave covers one run of 64 blocks along x)
    const Interior I = interior_of(g);
    float* rf = reinterpret_cast<float*>(res);
    if (I.n) {
        const uint32_t fg = (I.n + 255) / 256;
#define FZ_ARGS                                                                                                     \
    dim3(fg), dim3(256), 0, st, g, I.ib[0], I.ib[1], I.n, stream, stream_words, off, chunks, lut, oval, oidx, n_out, \
        0.0, rf, (int32_t*)nullptr, misc, 0, (const uint8_t*)nullptr, (const uint64_t*)nullptr,                    \
        (const int32_t*)nullptr, (uint64_t)0
        if (vec && g.ndim == 3 && I.ib[0] % 64 == 0)
            hipLaunchKernelGGL((k_decode_fast<3, true, true, true, false, true>), FZ_ARGS);
        else if (vec) {
            if (g.ndim == 3) hipLaunchKernelGGL((k_decode_fast<3, true, true, false, false, true>), FZ_ARGS);
            else if (g.ndim == 2) hipLaunchKernelGGL((k_decode_fast<2, true, true, false, false, true>), FZ_ARGS);
            else hipLaunchKernelGGL((k_decode_fast<1, true, true, false, false, true>), FZ_ARGS);
        } else {
            if (g.ndim == 3) hipLaunchKernelGGL((k_decode_fast<3, true, false, false, false, true>), FZ_ARGS);
            else if (g.ndim == 2) hipLaunchKernelGGL((k_decode_fast<2, true, false, false, false, true>), FZ_ARGS);
            else hipLaunchKernelGGL((k_decode_fast<1, true, false, false, false, true>), FZ_ARGS);
        }
#undef FZ_ARGS
    }
    if (I.n == g.nblocks) return;
    const uint32_t grid = (g.nblocks + 255) / 256;
    const int skip = I.n ? 1 : 0;
#define FZ_DRES(NDV)                                                                                              \
    hipLaunchKernelGGL(k_decode_res<NDV>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut, \
                       opos, oval, oidx, n_out, res, misc, skip, I.ib[0], I.ib[1], I.ib[2], 1)
    if (g.ndim == 3) FZ_DRES(3);
    else if (g.ndim == 2) FZ_DRES(2);
    else FZ_DRES(1);
#undef FZ_DRES
}

void launch_patch(hipStream_t st, const Geom& g, const uint32_t* ppos, const uint32_t* pbits, uint64_t n_pat,
                  float* out, Misc* misc) {
    if (n_pat == 0) return;
    uint64_t grid = (n_pat + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_patch<3>, dim3((uint32_t)grid), dim3(256), 0, st, g, ppos, pbits, n_pat, out, misc);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_patch<2>, dim3((uint32_t)grid), dim3(256), 0, st, g, ppos, pbits, n_pat, out, misc);
    else
        hipLaunchKernelGGL(k_patch<1>, dim3((uint32_t)grid), dim3(256), 0, st, g, ppos, pbits, n_pat, out, misc);
}

}  // namespace fz
