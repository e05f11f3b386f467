// Decompression (FZModules Sec. 1 and Sec. 3.3.1 describe it as Huffman
// decoding of the quantisation codes plus scattering of the outliers into
// the reconstruction; the inverse of the Lorenzo predictor is a prefix sum):
//   k_lut          - validates the code lengths, builds a 4096-entry table
//   k_decode       - one lane per block: table-driven Huffman decode from a
//                    per-lane window staged in LDS, outlier overwrite,
//                    in-block prefix sums (inverse Lorenzo), dequantisation,
//                    row stores - codes never leave registers
//   k_patch        - lossless patches written over the reconstruction
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// ----------------------------------------------------------- decode table
// Entry for the 12-bit prefix v: (length << 10) | symbol of the codeword
// that v starts with.  The lengths must describe a complete code (Kraft sum
// exactly 1, every length 1..12, at least two symbols).
__global__ __launch_bounds__(1024) void k_lut(const uint8_t* __restrict__ lensp, uint16_t* __restrict__ lut,
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
                e = (uint16_t)((L << 10) | cs.sorted[cs.offset[L] + idx]);
                break;
            }
        }
        lut[v] = e;
    }
}

// ----------------------------------------------------------------- decode
constexpr int kWin = 20;      // words staged per lane and round (5 x 16 B)
constexpr int kDecLanes = 256;

// A lane's window of the stream in LDS, column-major across the workgroup:
// word k of lane l is at k * 256 + l, so lanes reading their own word k land
// in distinct banks whatever k each lane is at.
struct LaneStream {
    const uint32_t* stream;
    uint64_t nwords;
    uint32_t* win;   // &WIN[lane]
    uint64_t aw;     // first staged word (multiple of 4)
    uint32_t rel;    // bit position relative to aw * 32

    // Stage the words holding the next 32 codewords (at most 384 bits).
    __device__ __forceinline__ void stage(uint64_t bitpos) {
        aw = (bitpos >> 5) & ~3ull;
        rel = (uint32_t)(bitpos - aw * 32);
        uint32_t w[kWin];
        if (aw + kWin <= nwords) {
            const uint4* s4 = reinterpret_cast<const uint4*>(stream + aw);
#pragma unroll
            for (int k = 0; k < kWin / 4; k++) {
                const uint4 v = s4[k];
                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kWin; k++) w[k] = (aw + k < nwords) ? stream[aw + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kWin; k++) win[k * kDecLanes] = w[k];
    }
    // the 64 stream bits starting at the current position, MSB first
    __device__ __forceinline__ uint64_t peek64() const {
        const uint32_t wi = rel >> 5, sh = rel & 31;
        const uint32_t w0 = win[wi * kDecLanes], w1 = win[(wi + 1) * kDecLanes];
        return (((uint64_t)w0 << 32) | w1) << sh;
    }
    __device__ __forceinline__ uint64_t bitpos() const { return aw * 32 + rel; }
};

// The block's outliers are read four at a time from the position-sorted
// list into registers (positions p, residuals v); past the end of the list
// positions read as 0xFFFFFFFF.
__device__ __forceinline__ void load_outliers(const uint32_t* __restrict__ opos, const int32_t* __restrict__ oval,
                                              uint64_t n, uint32_t i, uint4& p, int4& v) {
    if ((uint64_t)i + 4 <= n) {
        // the list start is only 4-byte aligned: four dword loads
        p = make_uint4(opos[i], opos[i + 1], opos[i + 2], opos[i + 3]);
        v = make_int4(oval[i], oval[i + 1], oval[i + 2], oval[i + 3]);
    } else {
        p.x = (uint64_t)i < n ? opos[i] : 0xFFFFFFFFu;
        p.y = (uint64_t)i + 1 < n ? opos[i + 1] : 0xFFFFFFFFu;
        p.z = (uint64_t)i + 2 < n ? opos[i + 2] : 0xFFFFFFFFu;
        p.w = 0xFFFFFFFFu;
        v.x = (uint64_t)i < n ? oval[i] : 0;
        v.y = (uint64_t)i + 1 < n ? oval[i + 1] : 0;
        v.z = (uint64_t)i + 2 < n ? oval[i + 2] : 0;
        v.w = 0;
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_decode(
    Geom g, const uint32_t* __restrict__ stream, uint64_t nwords, const uint64_t* __restrict__ off,
    const uint16_t* __restrict__ chunks, const uint16_t* __restrict__ lut_g, const uint32_t* __restrict__ opos,
    const int32_t* __restrict__ oval, const uint32_t* __restrict__ ofirst, uint64_t n_out, double e2,
    float* __restrict__ out, int vec, Misc* misc) {
    __shared__ uint16_t LUT[kLut];
    __shared__ uint32_t WIN[kDecLanes * kWin];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLut; i += 256) LUT[i] = lut_g[i];
    __syncthreads();
    const uint32_t b0 = blockIdx.x * 256 + t;
    const bool active = b0 < g.nblocks;
    const uint32_t b = active ? b0 : g.nblocks - 1;  // inactive lanes idle until the final reduction
    const BlockInfo info = block_info(g, b);
    const uint64_t start = off[b];
    LaneStream ls;
    ls.stream = stream;
    ls.nwords = nwords;
    ls.win = &WIN[t];
    uint32_t code0 = 0;
    bool bad = false;
    const uint32_t pos_b = b * kBlockElems;
    // the block's outliers are consecutive in the position-sorted list,
    // starting at ofirst[b] (meaningful only for blocks that have outliers:
    // every use is bounds- and position-checked)
    uint32_t onext = 0, ok = 0;
    uint4 op4 = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    int4 ov4 = make_int4(0, 0, 0, 0);
    if (n_out) {
        onext = ofirst[b];
        load_outliers(opos, oval, n_out, onext, op4, ov4);
    }

    // decode one codeword; code 0 takes the next outlier residual
    auto next = [&](uint32_t pos) -> int32_t {
        const uint64_t v = ls.peek64();
        const uint32_t e = LUT[(uint32_t)(v >> (64 - kLmax))];
        ls.rel += e >> 10;
        const uint32_t sym = e & 1023u;
        if (sym) return (int32_t)sym - kRadius;
        code0++;
        const uint32_t pk = ok == 0 ? op4.x : ok == 1 ? op4.y : ok == 2 ? op4.z : op4.w;
        int32_t d = ok == 0 ? ov4.x : ok == 1 ? ov4.y : ok == 2 ? ov4.z : ov4.w;
        if (pk != pos) {
            bad = true;
            d = 0;
        }
        if (++ok == 4) {
            onext += 4;
            ok = 0;
            load_outliers(opos, oval, n_out, onext, op4, ov4);
        }
        return d;
    };
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

    ls.aw = 0;
    ls.rel = 0;
    uint64_t bp = start;
    if (!active) {
        // nothing to decode
    } else if (ND == 3) {
        int32_t qp[64];
#pragma unroll
        for (int i = 0; i < 64; i++) qp[i] = 0;
        const uint64_t x0 = (uint64_t)info.bx * 8;
        for (uint32_t z = 0; z < info.ez; z++) {
            int32_t pr[8];
#pragma unroll
            for (int i = 0; i < 8; i++) pr[i] = 0;
#pragma unroll
            for (int half = 0; half < 2; half++) {
                ls.stage(bp);
#pragma unroll
                for (int yy = 0; yy < 4; yy++) {
                    const int y = half * 4 + yy;
                    if ((uint32_t)y < info.ey) {
                        int32_t rs = 0;
                        float v[8];
#pragma unroll
                        for (int x = 0; x < 8; x++) {
                            int32_t d = 0;
                            if ((uint32_t)x < info.ex) d = next(pos_b + x + 8 * y + 64 * z);
                            rs += d;
                            pr[x] += rs;
                            qp[y * 8 + x] += pr[x];
                            v[x] = deq(qp[y * 8 + x]);
                        }
                        const uint64_t yg = (uint64_t)info.by * 8 + y, zg = (uint64_t)info.bz * 8 + z;
                        store8(x0 + (uint64_t)g.n[0] * (yg + (uint64_t)g.n[1] * zg), v, info.ex);
                    }
                }
                bp = ls.bitpos();
            }
        }
    } else if (ND == 2) {
        int32_t qp[32];
#pragma unroll
        for (int i = 0; i < 32; i++) qp[i] = 0;
        for (uint32_t y = 0; y < info.ey; y++) {
            ls.stage(bp);
            int32_t rs = 0;
            const uint64_t row = (uint64_t)info.bx * 32 + (uint64_t)g.n[0] * ((uint64_t)info.by * 16 + y);
#pragma unroll
            for (int x8 = 0; x8 < 4; x8++) {
                float v[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const int x = x8 * 8 + i;
                    int32_t d = 0;
                    if ((uint32_t)x < info.ex) d = next(pos_b + x + 32 * y);
                    rs += d;
                    qp[x] += rs;
                    v[i] = deq(qp[x]);
                }
                if ((uint32_t)(x8 * 8) < info.ex) store8(row + x8 * 8, v, min(8u, info.ex - x8 * 8));
            }
            bp = ls.bitpos();
        }
    } else {
        int32_t acc = 0;
        const uint64_t row = (uint64_t)b * kBlockElems;
        for (uint32_t r = 0; r * 32 < info.ex; r++) {
            ls.stage(bp);
#pragma unroll
            for (int k8 = 0; k8 < 4; k8++) {
                float v[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const uint32_t idx = r * 32 + k8 * 8 + i;
                    int32_t d = 0;
                    if (idx < info.ex) d = next(pos_b + idx);
                    acc += d;
                    v[i] = deq(acc);
                }
                const uint32_t i0 = r * 32 + k8 * 8;
                if (i0 < info.ex) store8(row + i0, v, min(8u, info.ex - i0));
            }
            bp = ls.bitpos();
        }
    }
    if (active && bp - start != chunks[b]) bad = true;
    if (bad) atomicOr(&misc->flags, F_CORRUPT);
    uint32_t c = active ? code0 : 0u;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((t & 63) == 0 && c) atomicAdd(&misc->code0_count, c);
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
                                                    const uint32_t* __restrict__ ofirst, uint64_t n_out,
                                                    int32_t* __restrict__ res, Misc* misc) {
    __shared__ uint16_t LUT[kLut];
    __shared__ uint32_t WIN[kDecLanes * kWin];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLut; i += 256) LUT[i] = lut_g[i];
    __syncthreads();
    const uint32_t b0 = blockIdx.x * 256 + t;
    const bool active = b0 < g.nblocks;
    const uint32_t b = active ? b0 : g.nblocks - 1;
    const BlockInfo info = block_info(g, b);
    const uint64_t start = off[b];
    LaneStream ls;
    ls.stream = stream;
    ls.nwords = nwords;
    ls.win = &WIN[t];
    uint32_t code0 = 0;
    bool bad = false;
    const uint32_t pos_b = b * kBlockElems;
    uint32_t onext = 0, ok = 0;
    uint4 op4 = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    int4 ov4 = make_int4(0, 0, 0, 0);
    if (n_out) {
        onext = ofirst[b];
        load_outliers(opos, oval, n_out, onext, op4, ov4);
    }
    uint64_t bp = start;
    if (active) {
        ls.stage(bp);
        uint32_t cnt = 0;
        for (uint32_t lz = 0; lz < info.ez; lz++)
            for (uint32_t ly = 0; ly < info.ey; ly++)
                for (uint32_t lx = 0; lx < info.ex; lx++) {
                    if (cnt == 32) {
                        bp = ls.bitpos();
                        ls.stage(bp);
                        cnt = 0;
                    }
                    const uint32_t pos = pos_b + lx + g.bs[0] * (ly + g.bs[1] * lz);
                    const uint64_t v = ls.peek64();
                    const uint32_t e = LUT[(uint32_t)(v >> (64 - kLmax))];
                    ls.rel += e >> 10;
                    const uint32_t sym = e & 1023u;
                    int32_t d = (int32_t)sym - kRadius;
                    if (!sym) {
                        code0++;
                        const uint32_t pk = ok == 0 ? op4.x : ok == 1 ? op4.y : ok == 2 ? op4.z : op4.w;
                        d = ok == 0 ? ov4.x : ok == 1 ? ov4.y : ok == 2 ? ov4.z : ov4.w;
                        if (pk != pos) {
                            bad = true;
                            d = 0;
                        }
                        if (++ok == 4) {
                            onext += 4;
                            ok = 0;
                            load_outliers(opos, oval, n_out, onext, op4, ov4);
                        }
                    }
                    res[pos] = d;
                    cnt++;
                }
        bp = ls.bitpos();
    }
    if (active && bp - start != chunks[b]) bad = true;
    if (bad) atomicOr(&misc->flags, F_CORRUPT);
    uint32_t c = active ? code0 : 0u;
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1) c += __shfl_xor(c, dd, 64);
    if ((t & 63) == 0 && c) atomicAdd(&misc->code0_count, c);
}

// One wave (workgroup of 64) per block: residuals -> grid values in LDS by
// the block's inverse, then dequantised row stores.
template <int ND>
__global__ __launch_bounds__(64) void k_inverse(Geom g, const int32_t* __restrict__ res, int fixed_pred,
                                                const uint8_t* __restrict__ bpred,
                                                const uint64_t* __restrict__ reg_idx,
                                                const int32_t* __restrict__ coefs, uint64_t nreg, double e2,
                                                float* __restrict__ out, int vec, Misc* misc) {
    __shared__ int32_t A[kBlockElems];
    const uint32_t b = blockIdx.x;
    const uint32_t lane = threadIdx.x;
    const BlockInfo info = block_info(g, b);
    const uint32_t p = fixed_pred >= 0 ? (uint32_t)fixed_pred : bpred[b];
    const int32_t* rb = res + (uint64_t)b * kBlockElems;
    {
        const int4* src = reinterpret_cast<const int4*>(rb + 8 * lane);
        int4* dst = reinterpret_cast<int4*>(&A[8 * lane]);
        dst[0] = src[0];
        dst[1] = src[1];
    }
    __syncthreads();
    const uint32_t bs0 = g.bs[0], bs1 = g.bs[1];
    const uint32_t ext[3] = {info.ex, info.ey, info.ez};
    if (p <= 1) {
        // inclusive prefix sums along x, y, z (twice each for the second order)
        const int passes = p == 1 ? 2 : 1;
        for (int axis = 0; axis < (int)ND; axis++) {
            const uint32_t len = ext[axis];
            const uint32_t stride = axis == 0 ? 1 : (axis == 1 ? bs0 : bs0 * bs1);
            const uint32_t nlines = kBlockElems / (axis == 0 ? bs0 : (axis == 1 ? bs1 : 8));
            if (ND == 1) {
                // one line of 512: lane-local prefix over 8, wave scan of totals
                for (int rep = 0; rep < passes; rep++) {
                    int32_t v[8];
                    int32_t acc = 0;
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        acc += A[8 * lane + i];
                        v[i] = acc;
                    }
                    const int32_t incl = (int32_t)wave_incl_scan((uint32_t)acc);
                    const int32_t excl = incl - acc;
#pragma unroll
                    for (int i = 0; i < 8; i++) A[8 * lane + i] = v[i] + excl;
                    __syncthreads();
                }
            } else {
                for (uint32_t line = lane; line < nlines; line += 64) {
                    // base of this line: the remaining coordinates
                    uint32_t base;
                    if (axis == 0) base = line * bs0;
                    else if (axis == 1) base = (line % bs0) + (line / bs0) * bs0 * bs1;
                    else base = line;
                    for (int rep = 0; rep < passes; rep++) {
                        int32_t acc = 0;
                        for (uint32_t i = 0; i < len; i++) {
                            acc += A[base + i * stride];
                            A[base + i * stride] = acc;
                        }
                    }
                }
                __syncthreads();
            }
        }
    } else {
        // regression: add the fixed-point plane back
        // a map that selects more regression blocks than the container
        // holds coefficients for is corrupt (checked again on the host)
        const uint64_t r = fixed_pred >= 0 ? b : reg_idx[b];
        int4 c = make_int4(0, 0, 0, 0);
        if (r < nreg) c = reinterpret_cast<const int4*>(coefs)[r];
        else if (lane == 0) atomicOr(&misc->flags, F_CORRUPT);
        for (uint32_t k = lane; k < kBlockElems; k += 64) {
            const uint32_t lx = k % bs0, ly = (k / bs0) % bs1, lz = k / (bs0 * bs1);
            if (lx < info.ex && ly < info.ey && lz < info.ez) {
                const int64_t sum = (int64_t)c.x + (int64_t)c.y * (2 * (int32_t)lx - ((int32_t)info.ex - 1)) +
                                    (int64_t)c.z * (2 * (int32_t)ly - ((int32_t)info.ey - 1)) +
                                    (int64_t)c.w * (2 * (int32_t)lz - ((int32_t)info.ez - 1)) + 128;
                A[k] += (int32_t)(sum >> 8);
            }
        }
        __syncthreads();
    }
    // dequantise and store: lane = segment of 8 values along x
    uint32_t lx0, ly, lz;
    seg_coords<ND>(lane, lx0, ly, lz);
    if (ly < info.ey && lz < info.ez && lx0 < info.ex) {
        const uint32_t nv = min(8u, info.ex - lx0);
        const uint64_t idx = ((uint64_t)info.bx * g.bs[0] + lx0) +
                             (uint64_t)g.n[0] * (((uint64_t)info.by * g.bs[1] + ly) +
                                                 (uint64_t)g.n[1] * ((uint64_t)info.bz * g.bs[2] + lz));
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (float)((double)A[8 * lane + i] * e2);
        if (nv == 8 && vec) {
            f32x4* q4 = reinterpret_cast<f32x4*>(out + idx);
            const f32x4 a = {v[0], v[1], v[2], v[3]};
            const f32x4 c = {v[4], v[5], v[6], v[7]};
            q4[0] = a;
            q4[1] = c;
        } else {
            for (uint32_t i = 0; i < nv; i++) out[idx + i] = v[i];
        }
    }
}

// ------------------------------------------------------ outlier block index
// ofirst[b] = index of the first outlier of block b (blocks with outliers).
__global__ __launch_bounds__(256) void k_outlier_index(const uint32_t* __restrict__ opos, uint64_t n_out,
                                                       uint32_t nblocks, uint32_t* __restrict__ ofirst) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += stride) {
        const uint32_t b = opos[i] >> 9;
        if (b < nblocks && (i == 0 || (opos[i - 1] >> 9) != b)) ofirst[b] = (uint32_t)i;
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
void launch_lut(hipStream_t st, const uint8_t* lens_packed, uint16_t* lut, Misc* misc) {
    hipLaunchKernelGGL(k_lut, dim3(1), dim3(1024), 0, st, lens_packed, lut, misc);
}

void launch_decode(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                   const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                   const int32_t* oval, uint32_t* ofirst, uint64_t n_out, double e2, float* out, int vec,
                   Misc* misc) {
    if (n_out) {
        uint64_t og = (n_out + 255) / 256;
        if (og > 4096) og = 4096;
        hipLaunchKernelGGL(k_outlier_index, dim3((uint32_t)og), dim3(256), 0, st, opos, n_out, g.nblocks, ofirst);
    }
    const uint32_t grid = (g.nblocks + 255) / 256;
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_decode<3>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut,
                           opos, oval, ofirst, n_out, e2, out, vec, misc);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_decode<2>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut,
                           opos, oval, ofirst, n_out, e2, out, vec, misc);
    else
        hipLaunchKernelGGL(k_decode<1>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut,
                           opos, oval, ofirst, n_out, e2, out, vec, misc);
}

void launch_map_unpack(hipStream_t st, const uint8_t* map, uint32_t nblocks, uint8_t* bpred, Misc* misc) {
    hipLaunchKernelGGL(k_map_unpack, dim3((nblocks + 255) / 256), dim3(256), 0, st, map, nblocks, bpred, misc);
}

void launch_decode_pred(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                        const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                        const int32_t* oval, uint32_t* ofirst, uint64_t n_out, int32_t* res, int fixed_pred,
                        const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coefs, uint64_t nreg, double e2,
                        float* out, int vec, Misc* misc) {
    if (n_out) {
        uint64_t og = (n_out + 255) / 256;
        if (og > 4096) og = 4096;
        hipLaunchKernelGGL(k_outlier_index, dim3((uint32_t)og), dim3(256), 0, st, opos, n_out, g.nblocks, ofirst);
    }
    const uint32_t grid = (g.nblocks + 255) / 256;
#define FZ_DRES(NDV)                                                                                              \
    hipLaunchKernelGGL(k_decode_res<NDV>, dim3(grid), dim3(256), 0, st, g, stream, stream_words, off, chunks, lut, \
                       opos, oval, ofirst, n_out, res, misc);                                                      \
    hipLaunchKernelGGL(k_inverse<NDV>, dim3(g.nblocks), dim3(64), 0, st, g, res, fixed_pred, bpred, reg_idx, coefs, \
                       nreg, e2, out, vec, misc)
    if (g.ndim == 3) {
        FZ_DRES(3);
    } else if (g.ndim == 2) {
        FZ_DRES(2);
    } else {
        FZ_DRES(1);
    }
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
