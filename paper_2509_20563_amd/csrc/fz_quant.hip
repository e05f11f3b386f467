// Compression front end: scratch reset, value-range reduction and the fused
// prequantisation + block-local Lorenzo + post-quantisation + histogram +
// outlier/patch gather kernel (FZModules Sec. 3.1 dual quantisation and
// outliers; Sec. 3.2 relative error bound and code histogram).
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// --------------------------------------------------------------- reset
// Clears the per-call scratch: Misc, the global histogram and the look-back
// descriptors (a fill kernel rather than a memset node, so the sequence can
// be captured in a graph).
__global__ void k_reset(Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2, uint32_t n2,
                        uint64_t* d3, uint32_t n3, uint64_t off_chunks, uint64_t off_stream, uint64_t nreg) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) reset_misc(misc, off_chunks, off_stream, nreg);
    clear_scratch(gid, gridDim.x * blockDim.x, hist, d1, n1, d2, n2, d3, n3);
}

// -------------------------------------------------------------- min/max
// One pass over the field: min and max (exact, order-preserving atomics)
// and a non-finite check.  Needed only for the value-range relative bound.
__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, uint64_t N, int vec, Misc* misc) {
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    bool bad = false;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t tail = 0;
    if (vec) {
        // four independent 16-byte loads in flight per thread and iteration
        const f32x4* x4 = reinterpret_cast<const f32x4*>(x);
        const uint64_t n4 = N / 4;
        uint64_t i = gid;
        for (; i + 3 * stride < n4; i += 4 * stride) {
            f32x4 v[4];
#pragma unroll
            for (int k = 0; k < 4; k++) v[k] = __builtin_nontemporal_load(&x4[i + k * stride]);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                bad |= !(__builtin_isfinite(v[k].x) && __builtin_isfinite(v[k].y) && __builtin_isfinite(v[k].z) &&
                         __builtin_isfinite(v[k].w));
                lo = fminf(lo, fminf(fminf(v[k].x, v[k].y), fminf(v[k].z, v[k].w)));
                hi = fmaxf(hi, fmaxf(fmaxf(v[k].x, v[k].y), fmaxf(v[k].z, v[k].w)));
            }
        }
        for (; i < n4; i += stride) {
            f32x4 v = __builtin_nontemporal_load(&x4[i]);
            bad |= !(__builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z) &&
                     __builtin_isfinite(v.w));
            lo = fminf(lo, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
            hi = fmaxf(hi, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
        }
        tail = n4 * 4;
    }
    for (uint64_t i = tail + gid; i < N; i += stride) {
        float v = x[i];
        bad |= !__builtin_isfinite(v);
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, 64));
        hi = fmaxf(hi, __shfl_xor(hi, d, 64));
    }
    __shared__ float slo[4], shi[4];
    __shared__ int sbad;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    if (bad) sbad = 1;
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            lo = fminf(lo, slo[w]);
            hi = fmaxf(hi, shi[w]);
        }
        if (lo <= hi) {
            atomicMin(&misc->mm_lo, ord_f32(lo));
            atomicMax(&misc->mm_hi, ord_f32(hi));
        }
        if (sbad) atomicOr(&misc->flags, F_NONFINITE);
    }
}

// Load-phase thread mapping: which (block-in-tile, segment) a thread loads,
// chosen so that consecutive lanes read consecutive addresses.
template <int ND>
__device__ __forceinline__ void load_map(uint32_t t, uint32_t& bi, uint32_t& s) {
    if (ND == 3) { bi = t & 3; s = t >> 2; }                              // 4 blocks x 32 B per row
    else if (ND == 2) { bi = (t >> 2) & 3; s = (t & 3) | ((t >> 4) << 2); }  // 512 B per row
    else { bi = t >> 6; s = t & 63; }                                     // contiguous
}

// ------------------------------------------- fused Lorenzo quantisation
// One workgroup (256 threads) handles a tile of 4 consecutive blocks per
// iteration (tiles assigned statically, grid-strided).
//   phase A (load mapping): 8 values per thread -> q, patch mask -> LDS
//   phase B (wave = block, lane = segment): Lorenzo residual from LDS rows
//     (neighbours outside the block read a zero row), codes (block-major,
//     u16), histogram, outlier/patch bookkeeping (only in waves that have
//     any).  Outliers and patches go to the tile's own staging slots with a
//     per-tile count; the container sections are compacted in order after
//     a scan of those counts.
template <int ND>
__device__ __forceinline__ void read_row(const int32_t* Q, uint32_t off, int32_t r[8]) {
    const int4* p = reinterpret_cast<const int4*>(&Q[off]);
    const int4 a = p[0], c = p[1];
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w;
    r[4] = c.x; r[5] = c.y; r[6] = c.z; r[7] = c.w;
}

// Halo of the 3D interpolation quantiser: the grid values outside a tile
// that its predictions read, at the positions the stride-s classes need
// (for a block with origin (X0, Y0, Z0), i, ly, lz its local coordinates;
// sh = log2 s):
//   per block (kIHB values), for s = 1, 2, 4 the three y rows and z planes
//   outside the block that stride-s points reach, Y0 - 2s, Y0 + 8,
//   Y0 + 8 + 2s (row k = 0, 1, 2), at the points of that stride:
//     y rows: i a multiple of 2s, lz of s (32, 8, 2 values per row)
//     z planes: i and ly multiples of 2s (16, 4, 1 values per plane)
//     then the anchor's (X0 - 8, Y0 - 8, Z0), (X0 - 8, Y0, Z0 - 8),
//     (X0 - 8, Y0 - 8, Z0 - 8), (X0, Y0 - 8, Z0 - 8)
//   per tile (kIHX values), x columns of every (ly, lz) row taking them
//     left of the first block: X0 - 2 (all 64 rows), X0 - 4 (even ly and
//     lz), X0 - 8 (ly, lz in {0, 4})
//     right of the last block: X0 + 8, X0 + 10 (all rows), X0 + 12 (even
//     ly and lz), X0 + 16 (ly, lz in {0, 4})
// The indices are arithmetic in (r, i, ly, lz, sh) so that the lookups
// compile without branches.
constexpr int kIHY = 126, kIHZ = 63, kIHB = kIHY + kIHZ + 4, kIHX = 232, kIHAnchor = kIHY + kIHZ;
// y row at local ly = r (outside 0..7, reached by stride 1 << sh) of x = i, plane lz
__device__ __forceinline__ int interp_halo_y(int r, int i, int lz, int sh) {
    const int k = (r > 0 ? 1 : 0) + (r > 8 ? 1 : 0);
    return (sh > 0 ? 96 : 0) + (sh > 1 ? 24 : 0) + k * (32 >> (2 * sh)) + (i >> (sh + 1)) + (lz >> sh) * (4 >> sh);
}
// z plane at local lz = r (outside 0..7, reached by stride 1 << sh) of x = i, row ly
__device__ __forceinline__ int interp_halo_z(int r, int i, int ly, int sh) {
    const int k = (r > 0 ? 1 : 0) + (r > 8 ? 1 : 0);
    return kIHY + (sh > 0 ? 48 : 0) + (sh > 1 ? 12 : 0) + k * (16 >> (2 * sh)) + (i >> (sh + 1)) +
           (ly >> (sh + 1)) * (4 >> sh);
}
// x column j = -2, -4, -8 left of the tile's first block, row (ly, lz)
__device__ __forceinline__ int interp_halo_left(int j, int ly, int lz) {
    if (j == -2) return ly + 8 * lz;
    if (j == -4) return 64 + (ly >> 1) + 4 * (lz >> 1);
    return 80 + (ly >> 2) + 2 * (lz >> 2);
}
// x column j = 8, 10, 12, 16 from the origin of the tile's last block
__device__ __forceinline__ int interp_halo_right(int j, int ly, int lz) {
    const int a = (j == 8 ? 84 : 148) + ly + 8 * lz;
    const int b = j == 12 ? 212 + (ly >> 1) + 4 * (lz >> 1) : 228 + (ly >> 2) + 2 * (lz >> 2);
    return j <= 10 ? a : b;
}
// Entry e of the halo: the block of the tile it is relative to and its
// offset from that block's origin.
__device__ __forceinline__ void interp_halo_at(uint32_t e, uint32_t& bi, int& dx, int& dy, int& dz) {
    if (e >= (uint32_t)(kTileBlocks * kIHB)) {
        int k = (int)(e - kTileBlocks * kIHB);
        if (k < 84) {
            bi = 0;
            if (k < 64) { dx = -2; dy = k & 7; dz = k >> 3; }
            else if (k < 80) { k -= 64; dx = -4; dy = 2 * (k & 3); dz = 2 * (k >> 2); }
            else { k -= 80; dx = -8; dy = 4 * (k & 1); dz = 4 * (k >> 1); }
        } else {
            bi = kTileBlocks - 1;
            k -= 84;
            if (k < 64) { dx = 8; dy = k & 7; dz = k >> 3; }
            else if (k < 128) { k -= 64; dx = 10; dy = k & 7; dz = k >> 3; }
            else if (k < 144) { k -= 128; dx = 12; dy = 2 * (k & 3); dz = 2 * (k >> 2); }
            else { k -= 144; dx = 16; dy = 4 * (k & 1); dz = 4 * (k >> 1); }
        }
        return;
    }
    bi = e / kIHB;
    int k = (int)(e - bi * kIHB);
    if (k < kIHY) {
        // y rows: s = 1 (0..95), 2 (96..119), 4 (120..125); 32 >> 2 sh
        // points per row, 4 >> sh of them along x
        const int sh = k < 96 ? 0 : (k < 120 ? 1 : 2);
        const int m0 = k - (sh == 0 ? 0 : (sh == 1 ? 96 : 120));
        const int r = m0 >> (5 - 2 * sh), m = m0 & ((32 >> (2 * sh)) - 1);
        const int sv = 1 << sh;
        dy = r == 0 ? -2 * sv : (r == 1 ? 8 : 8 + 2 * sv);
        dx = (m & ((4 >> sh) - 1)) * 2 * sv;
        dz = (m >> (2 - sh)) * sv;
    } else if (k < kIHY + kIHZ) {
        // z planes: s = 1 (0..47), 2 (48..59), 4 (60..62); 16 >> 2 sh
        // points per plane, 4 >> sh of them along x
        const int kk = k - kIHY;
        const int sh = kk < 48 ? 0 : (kk < 60 ? 1 : 2);
        const int m0 = kk - (sh == 0 ? 0 : (sh == 1 ? 48 : 60));
        const int r = m0 >> (4 - 2 * sh), m = m0 & ((16 >> (2 * sh)) - 1);
        const int sv = 1 << sh;
        dz = r == 0 ? -2 * sv : (r == 1 ? 8 : 8 + 2 * sv);
        dx = (m & ((4 >> sh) - 1)) * 2 * sv;
        dy = (m >> (2 - sh)) * 2 * sv;
    } else {
        const int a = k - kIHAnchor;  // (x-8, y-8), (x-8, z-8), (x-8, y-8, z-8), (y-8, z-8)
        dx = a == 3 ? 0 : -8;
        dy = (a == 0 || a >= 2) ? -8 : 0;
        dz = a >= 1 ? -8 : 0;
    }
}

// Halo of the 3D global Lorenzo quantiser: entry e of a tile, the block of
// the tile it is relative to and its offset from that block's origin.  Per
// block (136 entries) the plane below (x, y in 0..7, z = -1), the row below
// for every z (x, z in 0..7, y = -1) and their shared row (x in 0..7, y = z =
// -1); then the column left of the tile's first block (x = -1, y and z in
// -1..7, 81 entries).
__device__ __forceinline__ void global_halo_at(uint32_t e, uint32_t& bi, int& dx, int& dy, int& dz) {
    constexpr uint32_t kPerBlock = 136;
    if (e >= (uint32_t)kTileBlocks * kPerBlock) {
        const int k = (int)(e - (uint32_t)kTileBlocks * kPerBlock);
        bi = 0;
        dx = -1;
        dy = k % 9 - 1;
        dz = k / 9 - 1;
        return;
    }
    bi = e / kPerBlock;
    const int k = (int)(e - bi * kPerBlock);
    if (k < 64) {
        dx = k & 7; dy = k >> 3; dz = -1;
    } else if (k < 128) {
        dx = k & 7; dy = -1; dz = (k - 64) >> 3;
    } else {
        dx = k - 128; dy = -1; dz = -1;
    }
}

// MODE: kQuantP0 (first-order Lorenzo everywhere), kQuantPred (predictor
// per block: fixed_pred >= 0 for every block, else bpred[b]), kQuantTrial
// (no codes: per-block cost of each predictor under a reference code,
// cheapest predictor -> choice[b], the three costs -> costs[3 b + p]).
// kQuantInterp: the interpolation predictor over the whole field, and a
// top-3 histogram (the codes of residuals -1, 0, 1 counted by ballots: the
// interpolation residuals pile up there).  3D: every neighbour from LDS
// (the tile's blocks and a halo staged in phase A); 1D/2D: from LDS, or
// prequantised from the field outside the tile.
// kQuantGlobal: first-order Lorenzo over the whole field (neighbours in
// other blocks read as in kQuantInterp).
// kQuantShuffle: first-order Lorenzo for the bit-shuffle codec: no codes
// and no histogram; each block's plane words (shuffle_words) go to its
// staging slot in `codes` (kShufSlot words: the 5 mask words, then the
// kept words in order).
constexpr int kQuantP0 = 0, kQuantPred = 1, kQuantTrial = 2, kQuantInterp = 3, kQuantGlobal = 4, kQuantShuffle = 5;

template <int ND, int MODE>
__global__ __launch_bounds__(256) void k_quant(const float* __restrict__ x, Geom g, uint32_t mode, double eb,
                                               int vec, Misc* misc, uint32_t* __restrict__ hist_g,
                                               uint16_t* __restrict__ codes, uint32_t ntiles,
                                               uint32_t* __restrict__ tile_cnt, uint2* __restrict__ ostage,
                                               uint2* __restrict__ pstage, int fixed_pred,
                                               const uint8_t* __restrict__ bpred, int32_t* __restrict__ coef,
                                               const uint32_t* __restrict__ cw_ref, uint8_t* __restrict__ choice,
                                               uint32_t* __restrict__ costs) {
    constexpr bool PRED = MODE != kQuantP0 && MODE != kQuantShuffle;
    // bit-shuffle: one block's plane words per wave
    __shared__ uint32_t SW[MODE == kQuantShuffle ? 4 * kShufWords : 1];
    // q per block, regions padded by 8 words so the load-mapped writes of
    // four blocks do not fall into the same banks; one extra zero row
    constexpr int kQStride = kBlockElems + 8;
    constexpr uint32_t kZero = kTileBlocks * kQStride;
    // (the 3D interpolation predictor keeps its halo after the zero row,
    // HI, so that one LDS index reaches the tile's values or the halo)
    constexpr int kHI = MODE == kQuantInterp && ND == 3 ? kTileBlocks * kIHB + kIHX : 0;
    __shared__ int32_t Q[kTileBlocks * kQStride + 8 + kHI];
    int32_t* const HI = &Q[kTileBlocks * kQStride + 8];
    __shared__ uint8_t PM[kTileBlocks * kSegs];
    __shared__ uint32_t H[kBins];
    __shared__ uint32_t wsum[4];
    __shared__ uint8_t LREF[kBins];
    // global Lorenzo: grid values just outside each block's lower faces (3D:
    // the plane below in z, the row below in y for every z, their shared
    // row; 2D: the row below), then the column left of the tile's first
    // block (3D: its 9 x 9 (y, z) from -1; 2D: 17 y from -1; 1D: one value);
    // zero outside the field
    constexpr int kHB = ND == 3 ? 136 : (ND == 2 ? 32 : 0);
    constexpr int kHL = ND == 3 ? 81 : (ND == 2 ? 17 : 1);
    __shared__ int32_t HG[MODE == kQuantGlobal ? kTileBlocks * kHB + kHL : 1];
    // selector network, hidden-layer weights transposed (lane = unit)

    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(t >> 6));
    double eb_abs;
    if (!resolve_eb(mode, eb, misc->mm_lo, misc->mm_hi, &eb_abs)) {
        if (blockIdx.x == 0 && t == 0) atomicOr(&misc->flags, F_EB);
        return;
    }
    const double e2 = 2.0 * eb_abs;
    const double inv = 1.0 / e2;
    // under the value-range bound the min/max pass has already flagged
    // non-finite input; the absolute bound has no such pass
    const bool check_finite = mode != 1;
    // per-block choice whose map the map scan dropped (too few blocks off
    // first-order Lorenzo): every block first-order
    const bool map_off = MODE == kQuantPred && fixed_pred < 0 && misc->map_off != 0;
    for (uint32_t i = t; i < (uint32_t)kBins; i += 256) H[i] = 0;
    if (MODE == kQuantTrial) {
        // reference code lengths; an unused code counts as kLmax + 1 bits
        for (uint32_t i = t; i < (uint32_t)kBins; i += 256) {
            const uint32_t l = cw_ref[i] >> 16;
            LREF[i] = (uint8_t)(l ? l : kLmax + 1);
        }
    }
    if (t < 8) Q[kZero + t] = 0;

    // load-phase lane constants (the same for every tile): block in tile,
    // segment, segment coordinates and the segment's row-major offset from
    // its block origin (indices fit in 32 bits: N <= 2^32)
    uint32_t la_bi, la_s, la_lx0, la_ly, la_lz;
    load_map<ND>(t, la_bi, la_s);
    seg_coords<ND>(la_s, la_lx0, la_ly, la_lz);
    const uint32_t la_rowoff = la_lx0 + g.n[0] * (la_ly + g.n[1] * la_lz);
    // 3D interpolation and 3D global Lorenzo: this thread's halo entries
    // t + 256 k, decoded once (block of the tile in bits 0-1, dx + 8, dy + 8,
    // dz + 8 in 5 bits each)
    constexpr bool kHalo3 = (MODE == kQuantInterp || MODE == kQuantGlobal) && ND == 3;
    constexpr int kHaloN = MODE == kQuantInterp ? kTileBlocks * kIHB + kIHX : kTileBlocks * kHB + kHL;
    constexpr int kIHPerThread = kHalo3 ? (kHaloN + 255) / 256 : 1;
    uint32_t ih_code[kIHPerThread];
    if (kHalo3) {
#pragma unroll
        for (int k = 0; k < kIHPerThread; k++) {
            uint32_t bi = 0;
            int dx = 0, dy = 0, dz = 0;
            const uint32_t e = t + 256u * k;
            if (e < (uint32_t)kHaloN) {
                if (MODE == kQuantInterp) interp_halo_at(e, bi, dx, dy, dz);
                else global_halo_at(e, bi, dx, dy, dz);
            }
            ih_code[k] = bi | (uint32_t)(dx + 8) << 2 | (uint32_t)(dy + 8) << 7 | (uint32_t)(dz + 8) << 12;
        }
    }
    // 3D interpolation, phase B: the LDS byte offsets of the neighbours
    // this lane's predictions read (lane = row (ly, lz) of block `wave`).
    // The axis and stride of the point at x = X0 + i of the row follow from
    // i | ly | lz alone (block origins are multiples of 8), so the offsets
    // are the same for every tile: per even i the four neighbours at -3s,
    // -s, +s, +3s along its axis (slots 2 k, 2 k + 1 for i = 2 k; the
    // anchor's slots unused), per odd i the columns x = -2, 8, 10 (the
    // others are in the row's registers); two 16-bit offsets per word.
    // icls: per even i (4 bits from bit 4 k) the axis (0 x, 1 y, 2 z) and
    // log2 of the stride.
    constexpr int kIOff = MODE == kQuantInterp && ND == 3 ? 10 : 1;
    uint32_t ioff[kIOff];
    uint32_t icls = 0;
    if (MODE == kQuantInterp && ND == 3) {
        const int ly = (int)(lane & 7u), lz = (int)(lane >> 3);
        const int w = (int)wave;
        const int rowQ = w * kQStride + (int)lane * 8;
        const int hb = kTileBlocks * kQStride + 8 + w * kIHB;
        const int hx = kTileBlocks * kQStride + 8 + kTileBlocks * kIHB;
        // index of x = X0 + j on this row: the row, a block of the tile,
        // or the tile's x halo (left of its first block, right of its last)
        auto ix = [&](int j) -> int {
            if (j >= 0 && j < 8) return rowQ + j;
            const int ob = (j + 16) / 8 - 2;  // block offset along x (j >= -16)
            const int wb = w + ob;
            if (wb >= 0 && wb < kTileBlocks) return rowQ + ob * kQStride + (j - 8 * ob);
            return hx + (j < 0 ? interp_halo_left(j, ly, lz)
                               : interp_halo_right(w * 8 - 8 * (kTileBlocks - 1) + j, ly, lz));
        };
        uint32_t o[20];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = 2 * k;
            const int orc = i | ly | lz;
            const int sh = (orc & 1) ? 0 : ((orc & 2) ? 1 : 2);
            const int sv = 1 << sh;
            const int ax = orc == 0 ? 0 : ((i & sv) ? 0 : ((ly & sv) ? 1 : 2));
            icls |= (uint32_t)(ax | sh << 2) << (4 * k);
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const int dd = (m == 0 ? -3 : (m == 1 ? -1 : (m == 2 ? 1 : 3))) * sv;
                int idx;
                if (orc == 0) {
                    idx = rowQ;  // the anchor: predicted on the anchor grid
                } else if (ax == 0) {
                    idx = ix(i + dd);
                } else if (ax == 1) {
                    const int l = ly + dd;
                    idx = (l >= 0 && l < 8) ? rowQ + i + 8 * dd : hb + interp_halo_y(l, i, lz, sh);
                } else {
                    const int l = lz + dd;
                    idx = (l >= 0 && l < 8) ? rowQ + i + 64 * dd : hb + interp_halo_z(l, i, ly, sh);
                }
                o[4 * k + m] = 4u * (uint32_t)idx;
            }
        }
        o[16] = 4u * (uint32_t)ix(-2);
        o[17] = 4u * (uint32_t)ix(8);
        o[18] = 4u * (uint32_t)ix(10);
        o[19] = 0;
#pragma unroll
        for (int k = 0; k < kIOff; k++) ioff[k] = o[2 * k] | o[2 * k + 1] << 16;
    } else {
        ioff[0] = 0;
    }
    // phase-B lane (segment = lane) offset, for reloading patched values
    uint32_t lb_lx0, lb_ly, lb_lz;
    seg_coords<ND>(lane, lb_lx0, lb_ly, lb_lz);
    const uint32_t lb_rowoff = lb_lx0 + g.n[0] * (lb_ly + g.n[1] * lb_lz);

    // phase-A source of a tile for this lane: first index and real values
    auto tile_src = [&](uint32_t tile, uint32_t& base, uint32_t& nv) {
        const uint32_t bk = tile * kTileBlocks + la_bi;
        const bool ok = bk < g.nblocks;
        const BlockInfo ik = block_info(g, ok ? bk : 0);
        nv = (ok && la_ly < ik.ey && la_lz < ik.ez && la_lx0 < ik.ex) ? min(8u, ik.ex - la_lx0) : 0u;
        base = ik.bx * g.bs[0] + g.n[0] * (ik.by * g.bs[1] + g.n[1] * (ik.bz * g.bs[2])) + la_rowoff;
    };
    auto tile_load = [&](uint32_t base, uint32_t nv, float v[8]) {
        if (nv == 8 && vec) {
            const f32x4* p = reinterpret_cast<const f32x4*>(x + base);
            const f32x4 a = __builtin_nontemporal_load(p);
            const f32x4 c = __builtin_nontemporal_load(p + 1);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] = (i < (int)nv) ? x[base + i] : 0.0f;
        }
    };
    // the values of the workgroup's next tile are loaded one tile ahead:
    // issued right after phase A's barrier, consumed by the next phase A,
    // so their latency overlaps phase B (issued earlier, the waits for the
    // current values would also cover them)
    uint32_t pf_nv = 0;
    float pf[8];
    // 3D interpolation and global Lorenzo: this thread's halo entries of the
    // next tile, loaded with its values (raw; bit k of hpm: entry k inside
    // the field); the origins of the tile's blocks are wave-uniform
    float hpf[kIHPerThread];
    uint32_t hpm = 0;
    auto halo_load = [&](uint32_t tl) {
        if (!kHalo3) return;
        uint32_t ox[kTileBlocks], oy[kTileBlocks], oz[kTileBlocks], valid = 0;
#pragma unroll
        for (int k = 0; k < kTileBlocks; k++) {
            const uint32_t bk = tl * kTileBlocks + k;
            const BlockInfo ik = block_info(g, bk < g.nblocks ? bk : 0);
            ox[k] = ik.bx * 8;
            oy[k] = ik.by * 8;
            oz[k] = ik.bz * 8;
            valid |= (tl < ntiles && bk < g.nblocks ? 1u : 0u) << k;
        }
        hpm = 0;
#pragma unroll
        for (int k = 0; k < kIHPerThread; k++) {
            hpf[k] = 0.0f;
            const uint32_t e = t + 256u * k;
            if (e >= (uint32_t)kHaloN) break;
            const uint32_t hv = ih_code[k];
            const uint32_t bi = hv & 3u;
            const uint32_t X0 = bi == 0 ? ox[0] : (bi == 1 ? ox[1] : (bi == 2 ? ox[2] : ox[3]));
            const uint32_t Y0 = bi == 0 ? oy[0] : (bi == 1 ? oy[1] : (bi == 2 ? oy[2] : oy[3]));
            const uint32_t Z0 = bi == 0 ? oz[0] : (bi == 1 ? oz[1] : (bi == 2 ? oz[2] : oz[3]));
            const int64_t xx = (int64_t)X0 + ((int)((hv >> 2) & 31u) - 8),
                          yy = (int64_t)Y0 + ((int)((hv >> 7) & 31u) - 8),
                          zz = (int64_t)Z0 + ((int)((hv >> 12) & 31u) - 8);
            if (((valid >> bi) & 1u) && xx >= 0 && yy >= 0 && zz >= 0 && xx < (int64_t)g.n[0] &&
                yy < (int64_t)g.n[1] && zz < (int64_t)g.n[2]) {
                hpf[k] = x[(uint64_t)xx + (uint64_t)g.n[0] * ((uint64_t)yy + (uint64_t)g.n[1] * (uint64_t)zz)];
                hpm |= 1u << k;
            }
        }
    };
    // first tile: workgroup w, or for the 3D interpolation predictor (whose
    // halo reads the neighbouring tiles) the tiles of one round spread so
    // that the workgroups of one XCD (w mod 8, dispatch order) take one
    // contiguous eighth of them
    uint32_t tile0 = blockIdx.x;
    if (MODE == kQuantInterp && ND == 3 && (gridDim.x & 7u) == 0)
        tile0 = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    {
        uint32_t base = 0;
        if (tile0 < ntiles) tile_src(tile0, base, pf_nv);
        tile_load(base, tile0 < ntiles ? pf_nv : 0u, pf);
        halo_load(tile0);
    }

    for (uint32_t tile = tile0; tile < ntiles; tile += gridDim.x) {
        // ---------------- phase A: prequantise (values loaded a tile ago)
        {
            const uint32_t nv = pf_nv;
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] = pf[i];
            int32_t q[8];
            uint32_t pm = 0;
            bool bad = false;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                bool p;
                const int32_t qi = prequant1(v[i], e2, inv, eb_abs, p);
                const bool valid = i < (int)nv;
                bad |= check_finite && valid && !__builtin_isfinite(v[i]);
                q[i] = valid ? qi : 0;
                pm |= (valid && p ? 1u : 0u) << i;
            }
            if (bad) atomicOr(&misc->flags, F_NONFINITE);
            int4* dst = reinterpret_cast<int4*>(&Q[la_bi * kQStride + la_s * 8]);
            dst[0] = make_int4(q[0], q[1], q[2], q[3]);
            dst[1] = make_int4(q[4], q[5], q[6], q[7]);
            PM[la_bi * kSegs + la_s] = (uint8_t)pm;
        }
        if (MODE == kQuantInterp && ND == 3) {
            // interpolation (3D): the grid values outside the blocks that
            // the stride-s predictions of the tile read (loaded a tile ago)
#pragma unroll
            for (int k = 0; k < kIHPerThread; k++) {
                const uint32_t e = t + 256u * k;
                if (e >= (uint32_t)(kTileBlocks * kIHB + kIHX)) break;
                bool pq;
                const int32_t v = prequant1(hpf[k], e2, inv, eb_abs, pq);
                HI[e] = ((hpm >> k) & 1u) ? v : 0;
            }
        }
        if (MODE == kQuantGlobal && ND == 3) {
            // global Lorenzo (3D): the grid values just outside the tile's
            // blocks (global_halo_at), loaded a tile ago
#pragma unroll
            for (int k = 0; k < kIHPerThread; k++) {
                const uint32_t e = t + 256u * k;
                if (e >= (uint32_t)kHaloN) break;
                bool pq;
                const int32_t v = prequant1(hpf[k], e2, inv, eb_abs, pq);
                HG[e] = ((hpm >> k) & 1u) ? v : 0;
            }
        } else if (MODE == kQuantGlobal) {
            for (uint32_t e = t; e < (uint32_t)(kTileBlocks * kHB + kHL); e += 256) {
                const bool left = e >= (uint32_t)(kTileBlocks * kHB);
                const uint32_t bi = left ? 0u : e / (uint32_t)(kHB ? kHB : 1);
                const uint32_t k = left ? e - kTileBlocks * kHB : e % (uint32_t)(kHB ? kHB : 1);
                const uint32_t bk = tile * kTileBlocks + bi;
                int32_t v = 0;
                if (bk < g.nblocks) {
                    const BlockInfo ik = block_info(g, bk);
                    const int32_t X0 = (int32_t)(ik.bx * g.bs[0]), Y0 = (int32_t)(ik.by * g.bs[1]),
                                  Z0 = (int32_t)(ik.bz * g.bs[2]);
                    int32_t xx = X0, yy = Y0, zz = Z0;
                    if (left) {
                        xx = X0 - 1;
                        if (ND == 3) {
                            yy = Y0 + (int32_t)(k % 9) - 1;
                            zz = Z0 + (int32_t)(k / 9) - 1;
                        } else if (ND == 2) {
                            yy = Y0 + (int32_t)k - 1;
                        }
                    } else if (ND == 3) {
                        if (k < 64) {
                            xx = X0 + (int32_t)(k & 7);
                            yy = Y0 + (int32_t)(k >> 3);
                            zz = Z0 - 1;
                        } else if (k < 128) {
                            xx = X0 + (int32_t)(k & 7);
                            yy = Y0 - 1;
                            zz = Z0 + (int32_t)((k - 64) >> 3);
                        } else {
                            xx = X0 + (int32_t)(k - 128);
                            yy = Y0 - 1;
                            zz = Z0 - 1;
                        }
                    } else {
                        xx = X0 + (int32_t)k;
                        yy = Y0 - 1;
                    }
                    if (xx >= 0 && yy >= 0 && zz >= 0 && (uint32_t)xx < g.n[0] && (uint32_t)yy < g.n[1] &&
                        (uint32_t)zz < g.n[2]) {
                        bool pq;
                        v = prequant1(x[(uint64_t)xx + (uint64_t)g.n[0] * ((uint64_t)yy + (uint64_t)g.n[1] * zz)], e2,
                                      inv, eb_abs, pq);
                    }
                }
                HG[e] = v;
            }
        }
        __syncthreads();
        {
            const uint32_t nt = tile + gridDim.x;
            uint32_t base = 0;
            if (nt < ntiles) tile_src(nt, base, pf_nv);
            else pf_nv = 0;
            tile_load(base, pf_nv, pf);
            halo_load(nt);
        }

        // ---------------- phase B: wave = block, lane = segment
        const uint32_t s = lane;
        const uint32_t b = tile * kTileBlocks + wave;  // wave-uniform
        const bool blk = b < g.nblocks;
        const uint32_t Qb = wave * kQStride;
        uint32_t nv = 0;  // real values in this segment
        int32_t d[8];
        {
            const BlockInfo info = block_info(g, blk ? b : 0);
            uint32_t lx0, ly, lz;
            seg_coords<ND>(s, lx0, ly, lz);
            nv = (blk && ly < info.ey && lz < info.ez && lx0 < info.ex) ? min(8u, info.ex - lx0) : 0u;
            // whole-field predictors (interpolation, global Lorenzo): the
            // grid value anywhere in the field, from LDS where it falls in
            // this tile's blocks, else the value prequantised here (the same
            // arithmetic as phase A, so the same grid value)
            const uint32_t b0 = tile * kTileBlocks;
            auto q_at = [&](uint32_t xx, uint32_t yy, uint32_t zz) -> int32_t {
                uint32_t bb, loc;
                if (ND == 3) {
                    bb = (xx >> 3) + g.nb[0] * ((yy >> 3) + g.nb[1] * (zz >> 3));
                    loc = (xx & 7u) + 8u * ((yy & 7u) + 8u * (zz & 7u));
                } else if (ND == 2) {
                    bb = (xx >> 5) + g.nb[0] * (yy >> 4);
                    loc = (xx & 31u) + 32u * (yy & 15u);
                } else {
                    bb = xx >> 9;
                    loc = xx & 511u;
                }
                const uint32_t rel = bb - b0;
                if (rel < (uint32_t)kTileBlocks) return Q[rel * kQStride + loc];
                bool pq;
                return prequant1(x[(uint64_t)xx + (uint64_t)g.n[0] * ((uint64_t)yy + (uint64_t)g.n[1] * zz)], e2,
                                 inv, eb_abs, pq);
            };
            auto residual = [&](const uint32_t pr) {
            if (MODE == kQuantInterp && ND == 3) {
                // 3D: lane = row (ly, lz) of the block, values at x = X0 + i;
                // every neighbour in this row's registers or at an LDS
                // offset taken once per kernel (ioff, icls).  Grid values
                // are at most 2^24 in magnitude, so the cubic and linear
                // rules are exact in 32-bit integers.
                int32_t r0[8];
                read_row<ND>(Q, Qb + s * 8, r0);
                const uint32_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
                const uint32_t X0 = info.bx * 8, Y = info.by * 8 + ly, Z = info.bz * 8 + lz;
                const int32_t* Hb = &Q[kTileBlocks * kQStride + 8 + (int)wave * kIHB];
                // the value at the LDS byte offset in half h of word w
                auto at = [&](uint32_t w, int h) -> int32_t {
                    const uint32_t off = h ? (w >> 16) : (w & 0xffffu);
                    return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(Q) + off);
                };
                auto pick = [](bool m3, bool p1, bool p3, int32_t vm3, int32_t vm1, int32_t vp1, int32_t vp3) {
                    const int32_t cub = (-vm3 + 9 * vm1 + 9 * vp1 - vp3 + 8) >> 4;
                    const int32_t lin = (vm1 + vp1 + 1) >> 1;
                    return (m3 && p3) ? cub : (p1 ? lin : vm1);
                };
                // x = X0 + j of this row for the odd points (j = -2 .. 10)
                auto vx = [&](int j) -> int32_t {
                    if (j >= 0 && j < 8) return r0[j];
                    return j == -2 ? at(ioff[8], 0) : (j == 8 ? at(ioff[8], 1) : at(ioff[9], 0));
                };
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const uint32_t xx = X0 + i;
                    int32_t pq;
                    if (i & 1) {
                        pq = pick(xx >= 3, xx + 1 < n0, xx + 3 < n0, vx(i - 3), vx(i - 1), vx(i + 1), vx(i + 3));
                    } else {
                        const int k = i / 2;
                        const uint32_t c = icls >> (4 * k);
                        const uint32_t ax = c & 3u, sv = 1u << ((c >> 2) & 3u);
                        const uint32_t ca = ax == 0 ? xx : (ax == 1 ? Y : Z);
                        const uint32_t na = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
                        pq = pick(ca >= 3 * sv, ca + sv < na, ca + 3 * sv < na, at(ioff[2 * k], 0),
                                  at(ioff[2 * k], 1), at(ioff[2 * k + 1], 0), at(ioff[2 * k + 1], 1));
                        if (i == 0) {
                            // the block's anchor (ly = lz = 0): Lorenzo on the
                            // anchor grid, the neighbours 8 below in x, y, z
                            // (x - 8 is that row's stride-4 neighbour of i = 4)
                            const bool ix = X0 >= 8, iy = Y >= 8, iz = Z >= 8;
                            int32_t pa = 0;
                            pa += ix ? at(ioff[4], 0) : 0;
                            pa += iy ? Hb[interp_halo_y(-8, 0, 0, 2)] : 0;
                            pa += iz ? Hb[interp_halo_z(-8, 0, 0, 2)] : 0;
                            pa -= (ix && iy) ? Hb[kIHAnchor + 0] : 0;
                            pa -= (ix && iz) ? Hb[kIHAnchor + 1] : 0;
                            pa -= (iy && iz) ? Hb[kIHAnchor + 3] : 0;
                            pa += (ix && iy && iz) ? Hb[kIHAnchor + 2] : 0;
                            pq = ((Y | Z) & 7u) == 0 ? pa : pq;
                        }
                    }
                    d[i] = i < (int)nv ? (int32_t)((uint32_t)r0[i] - (uint32_t)pq) : 0;
                }
            } else if (MODE == kQuantInterp) {
                int32_t r0[8];
                read_row<ND>(Q, Qb + s * 8, r0);
                const uint32_t n3[3] = {g.n[0], g.n[1], g.n[2]};
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const uint32_t c[3] = {info.bx * g.bs[0] + lx0 + i, info.by * g.bs[1] + ly,
                                           info.bz * g.bs[2] + lz};
                    const int32_t pq = i < (int)nv ? interp_predict(c, n3, ND, q_at) : 0;
                    d[i] = (int32_t)((uint32_t)r0[i] - (uint32_t)pq);
                }
            } else if (MODE == kQuantGlobal) {
                // first-order Lorenzo over the whole field, every neighbour
                // from LDS: this block's rows, the halo rows below its lower
                // faces, and left of the segment the previous segment, the
                // previous block of the tile or the tile's left column
                const uint32_t bi = wave;
                const int32_t* Hb = &HG[bi * kHB];
                // row (y - dy, z - dz) of the lane's segment into r[1..8], the
                // value left of it into r[0]
                auto row9 = [&](uint32_t dy, uint32_t dz, int32_t r[9]) {
                    const bool iny = dy <= ly, inz = dz <= lz;
                    if (ND == 3) {
                        const int32_t* src = (iny && inz) ? &Q[Qb + (s - dy - 8 * dz) * 8]
                                             : (inz ? &Hb[64 + 8 * (lz - dz)]
                                                    : (iny ? &Hb[8 * (ly - dy)] : &Hb[128]));
#pragma unroll
                        for (int i = 0; i < 8; i++) r[1 + i] = src[i];
                        if (info.bx == 0) {
                            r[0] = 0;
                        } else if (bi > 0) {
                            const uint32_t Qp = (bi - 1) * kQStride;
                            const int32_t* Hp = &HG[(bi - 1) * kHB];
                            r[0] = (iny && inz) ? Q[Qp + (s - dy - 8 * dz) * 8 + 7]
                                                : (inz ? Hp[64 + 8 * (lz - dz) + 7]
                                                       : (iny ? Hp[8 * (ly - dy) + 7] : Hp[135]));
                        } else {
                            r[0] = HG[kTileBlocks * kHB + (ly + 1 - dy) + 9 * (lz + 1 - dz)];
                        }
                    } else if (ND == 2) {
                        const uint32_t sx = s & 3;
                        const int32_t* src = iny ? &Q[Qb + (s - 4 * dy) * 8] : &Hb[8 * sx];
#pragma unroll
                        for (int i = 0; i < 8; i++) r[1 + i] = src[i];
                        if (sx > 0) {
                            r[0] = iny ? Q[Qb + (s - 4 * dy - 1) * 8 + 7] : Hb[8 * sx - 1];
                        } else if (info.bx == 0) {
                            r[0] = 0;
                        } else if (bi > 0) {
                            r[0] = iny ? Q[(bi - 1) * kQStride + (3 + 4 * (ly - dy)) * 8 + 7] : HG[(bi - 1) * kHB + 31];
                        } else {
                            r[0] = HG[kTileBlocks * kHB + (ly + 1 - dy)];
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; i++) r[1 + i] = Q[Qb + s * 8 + i];
                        if (s > 0) r[0] = Q[Qb + (s - 1) * 8 + 7];
                        else if (info.bx == 0) r[0] = 0;
                        else if (bi > 0) r[0] = Q[(bi - 1) * kQStride + 63 * 8 + 7];
                        else r[0] = HG[0];
                    }
                };
                int32_t A[9];
                row9(0, 0, A);
                if (ND >= 2) {
                    int32_t ry[9];
                    row9(1, 0, ry);
#pragma unroll
                    for (int i = 0; i < 9; i++) A[i] -= ry[i];
                }
                if (ND == 3) {
                    int32_t rz[9], ryz[9];
                    row9(0, 1, rz);
                    row9(1, 1, ryz);
#pragma unroll
                    for (int i = 0; i < 9; i++) A[i] = A[i] - rz[i] + ryz[i];
                }
#pragma unroll
                for (int i = 0; i < 8; i++) d[i] = A[i + 1] - A[i];
            } else if (pr == 0) {
                // first-order Lorenzo: A = residual along y/z of the rows,
                // then the backward difference along x
                int32_t r0[8], A[8];
                int32_t am1 = 0;  // A[-1]: the left neighbour term along x
                read_row<ND>(Q, Qb + s * 8, r0);
                if (ND == 3) {
                    int32_t ry[8], rz[8], ryz[8];
                    read_row<ND>(Q, ly ? Qb + (s - 1) * 8 : kZero, ry);
                    read_row<ND>(Q, lz ? Qb + (s - 8) * 8 : kZero, rz);
                    read_row<ND>(Q, (ly && lz) ? Qb + (s - 9) * 8 : kZero, ryz);
#pragma unroll
                    for (int i = 0; i < 8; i++) A[i] = (r0[i] - ry[i]) - (rz[i] - ryz[i]);
                } else if (ND == 2) {
                    const uint32_t sx = s & 3;
                    int32_t up[8];
                    read_row<ND>(Q, ly ? Qb + (s - 4) * 8 : kZero, up);
                    const int32_t left = Q[sx ? Qb + (s - 1) * 8 + 7 : kZero];
                    const int32_t upleft = Q[(sx && ly) ? Qb + (s - 5) * 8 + 7 : kZero];
                    am1 = left - upleft;
#pragma unroll
                    for (int i = 0; i < 8; i++) A[i] = r0[i] - up[i];
                } else {
                    am1 = Q[s ? Qb + (s - 1) * 8 + 7 : kZero];
#pragma unroll
                    for (int i = 0; i < 8; i++) A[i] = r0[i];
                }
#pragma unroll
                for (int i = 7; i >= 0; i--) d[i] = A[i] - (i ? A[i - 1] : am1);
            } else if (PRED && pr == 1) {
                // second-order Lorenzo: weights (1, -2, 1) per axis; rows
                // combined first (R), then the second difference along x
                int32_t R[8], rr[8];
                int32_t rm1 = 0, rm2 = 0;  // R[-1], R[-2]
#pragma unroll
                for (int i = 0; i < 8; i++) R[i] = 0;
                if (ND == 3) {
#pragma unroll
                    for (int c = 0; c < 3; c++)
#pragma unroll
                        for (int a = 0; a < 3; a++) {
                            const int32_t w = (a == 1 ? -2 : 1) * (c == 1 ? -2 : 1);
                            read_row<ND>(Q, (ly >= (uint32_t)a && lz >= (uint32_t)c) ? Qb + (s - a - 8 * c) * 8 : kZero,
                                         rr);
#pragma unroll
                            for (int i = 0; i < 8; i++) R[i] += w * rr[i];
                        }
                } else if (ND == 2) {
                    const uint32_t sx = s & 3;
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const int32_t w = a == 1 ? -2 : 1;
                        const bool in = ly >= (uint32_t)a;
                        read_row<ND>(Q, in ? Qb + (s - 4 * a) * 8 : kZero, rr);
#pragma unroll
                        for (int i = 0; i < 8; i++) R[i] += w * rr[i];
                        const uint32_t lo = (sx && in) ? Qb + (s - 4 * a - 1) * 8 : kZero;
                        rm2 += w * Q[lo + (lo == kZero ? 0 : 6)];
                        rm1 += w * Q[lo + (lo == kZero ? 0 : 7)];
                    }
                } else {
                    read_row<ND>(Q, Qb + s * 8, R);
                    rm2 = Q[s ? Qb + (s - 1) * 8 + 6 : kZero];
                    rm1 = Q[s ? Qb + (s - 1) * 8 + 7 : kZero];
                }
#pragma unroll
                for (int i = 7; i >= 0; i--) {
                    const int32_t p1 = i >= 1 ? R[i - 1] : rm1;
                    const int32_t p2 = i >= 2 ? R[i - 2] : (i == 1 ? rm1 : rm2);
                    d[i] = R[i] - 2 * p1 + p2;
                }
            } else if (PRED) {
                // linear regression: wave-reduced sums over the block's real
                // values with centred coordinates, fixed point (8 bits)
                int32_t r0[8];
                read_row<ND>(Q, Qb + s * 8, r0);
                const int32_t v = 2 * (int32_t)ly - ((int32_t)info.ey - 1);
                const int32_t w = 2 * (int32_t)lz - ((int32_t)info.ez - 1);
                int64_t s0 = 0, su = 0;
#pragma unroll
                for (int i = 0; i < 8; i++)
                    if (i < (int)nv) {
                        const int32_t u = 2 * (int32_t)(lx0 + i) - ((int32_t)info.ex - 1);
                        s0 += r0[i];
                        su += (int64_t)u * r0[i];
                    }
                const int64_t sv = s0 * v, sw = s0 * w;
                auto wsum64 = [&](int64_t a) -> int64_t {
                    const uint64_t r = wave_incl_scan64((uint64_t)a, [](uint64_t x, uint64_t y) { return x + y; });
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r, 63);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(r >> 32), 63);
                    return (int64_t)(((uint64_t)hi << 32) | lo);
                };
                const int64_t S0 = wsum64(s0), SU = wsum64(su), SV = wsum64(sv), SW = wsum64(sw);
                const int64_t n = (int64_t)info.ex * info.ey * info.ez;
                auto rdiv = [](int64_t a, int64_t q) -> int64_t {
                    return a >= 0 ? (a + q / 2) / q : -((-a + q / 2) / q);
                };
                auto clamp32 = [](int64_t a) -> int32_t {
                    return a > INT32_MAX ? INT32_MAX : (a < INT32_MIN ? INT32_MIN : (int32_t)a);
                };
                auto dsum = [&](int64_t e) -> int64_t { return e * (e * e - 1) / 3 * (n / e); };
                const int64_t dx = dsum(info.ex), dy = dsum(info.ey), dz = dsum(info.ez);
                const int32_t cA = clamp32(rdiv(S0 * 256, n));
                const int32_t cX = dx > 0 ? clamp32(rdiv(SU * 256, dx)) : 0;
                const int32_t cY = (ND >= 2 && dy > 0) ? clamp32(rdiv(SV * 256, dy)) : 0;
                const int32_t cZ = (ND >= 3 && dz > 0) ? clamp32(rdiv(SW * 256, dz)) : 0;
                if (MODE == kQuantPred && lane == 0 && blk) {
                    int4* cp = reinterpret_cast<int4*>(coef + 4 * (uint64_t)b);
                    *cp = make_int4(cA, cX, cY, cZ);
                }
                const int64_t base = (int64_t)cA + (int64_t)cY * v + (int64_t)cZ * w + 128;
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const int32_t u = 2 * (int32_t)(lx0 + i) - ((int32_t)info.ex - 1);
                    const int32_t pred = (int32_t)((base + (int64_t)cX * u) >> 8);
                    d[i] = r0[i] - pred;
                }
            }
            };
            if (MODE == kQuantTrial) {
                // cost of each predictor: reference code bits + 64 per
                // outlier (+ 128 bits of coefficients for the regression)
                uint32_t cst[3];
#pragma unroll
                for (uint32_t pr = 0; pr < 3; pr++) {
                    residual(pr);
                    uint32_t c = 0;
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        const uint32_t u = (uint32_t)(d[i] + (kRadius - 1));
                        const uint32_t cd = u < (uint32_t)(2 * kRadius - 1) ? u + 1 : 0u;
                        c += (i < (int)nv) ? (uint32_t)LREF[cd] + (cd ? 0u : 64u) : 0u;
                    }
                    cst[pr] = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(c), 63) + (pr == 2 ? 128u : 0u);
                }
                if (lane == 0 && blk) {
                    uint32_t best = 0;
                    if (cst[1] < cst[best]) best = 1;
                    if (cst[2] < cst[best]) best = 2;
                    choice[b] = (uint8_t)best;
                    if (costs) {
                        costs[3 * (uint64_t)b] = cst[0];
                        costs[3 * (uint64_t)b + 1] = cst[1];
                        costs[3 * (uint64_t)b + 2] = cst[2];
                    }
                }
            } else {
                // a map dropped by the map scan (too few blocks off
                // first-order Lorenzo) codes every block first-order
                residual(PRED ? (fixed_pred >= 0 ? (uint32_t)fixed_pred
                                                 : ((blk && !map_off) ? (uint32_t)bpred[b] : 0u))
                              : 0u);
            }
        }
        if (MODE == kQuantTrial) {
            __syncthreads();
            continue;
        }
        // codes: residuals in (-512, 512) -> residual + 512, otherwise 0
        uint32_t code[8];
        uint32_t cmin = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t u = (uint32_t)(d[i] + (kRadius - 1));
            code[i] = u < (uint32_t)(2 * kRadius - 1) ? u + 1 : 0u;
            if (i < (int)nv) cmin = min(cmin, code[i]);
        }
        if (MODE == kQuantShuffle && blk) {
            // lane = slots 8 s .. 8 s + 7 of the block (the segment): the
            // block's plane words, its masks and kept words to its slot
            uint32_t sym[8];
#pragma unroll
            for (int i = 0; i < 8; i++) sym[i] = i < (int)nv ? fold_code(code[i]) : 0u;
            uint32_t w[3];
            shuffle_words(sym, lane, &SW[wave * kShufWords], w);
            const uint64_t m0 = __ballot(w[0] != 0), m1 = __ballot(w[1] != 0), m2 = __ballot(w[2] != 0);
            uint32_t* S = reinterpret_cast<uint32_t*>(codes) + (uint64_t)kShufSlot * b;
            if (lane < kMaskWords)
                S[lane] = lane == 0 ? (uint32_t)m0
                        : lane == 1 ? (uint32_t)(m0 >> 32)
                        : lane == 2 ? (uint32_t)m1
                        : lane == 3 ? (uint32_t)(m1 >> 32)
                                    : (uint32_t)m2;
            const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
            const uint32_t c0 = (uint32_t)__popcll(m0), c1 = (uint32_t)__popcll(m1);
            if (w[0]) S[kMaskWords + __popcll(m0 & below)] = w[0];
            if (w[1]) S[kMaskWords + c0 + __popcll(m1 & below)] = w[1];
            if (w[2]) S[kMaskWords + c0 + c1 + __popcll(m2 & below)] = w[2];
        } else if (blk) {
            uint4 pk;
            pk.x = code[0] | (code[1] << 16);
            pk.y = code[2] | (code[3] << 16);
            pk.z = code[4] | (code[5] << 16);
            pk.w = code[6] | (code[7] << 16);
            *reinterpret_cast<uint4*>(&codes[(uint64_t)b * kBlockElems + s * 8]) = pk;
        }
        // histogram: the zero residual's code (the most frequent one in
        // smooth and in flat regions) is counted by ballots and added once
        // per wave; every other valid code is added by its lane.  (A
        // candidate taken from the block's corner, whose residual is the
        // grid value itself, left most lanes of flat blocks adding to one
        // bin in the same instruction: 64-way serialised LDS atomics, 2.8 ms
        // instead of 1.9 on the 1024^3 fronts/spikes field.)
        if (MODE == kQuantShuffle) {
            // no histogram: the bit-shuffle codec needs none
        } else if (blk && MODE != kQuantInterp) {
            const uint32_t ca = (uint32_t)kRadius;
            uint32_t na = 0;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const bool valid = i < (int)nv;
                const bool ma = valid && code[i] == ca;
                na += (uint32_t)__popcll(__ballot(ma));
                if (valid && !ma) atomicAdd(&H[code[i]], 1u);
            }
            if (lane == 0 && na) atomicAdd(&H[ca], na);
        } else if (blk) {
            // top-3: residuals -1, 0, 1 by ballots, one add each per wave
            uint32_t nk[3] = {0, 0, 0};
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const bool valid = i < (int)nv;
                const uint32_t k = code[i] - (uint32_t)(kRadius - 1);  // 0, 1, 2 for codes 511..513
#pragma unroll
                for (uint32_t j = 0; j < 3; j++) nk[j] += (uint32_t)__popcll(__ballot(valid && k == j));
                if (valid && k > 2u) atomicAdd(&H[code[i]], 1u);
            }
            if (lane < 3 && nk[lane]) atomicAdd(&H[kRadius - 1 + lane], nk[lane]);
        }

        // ---------------- outliers and patches (block order inside the tile)
        const uint32_t pm_lane = PM[t] & ((1u << nv) - 1u);
        const bool has = (cmin == 0) || pm_lane;
        uint32_t packed = 0, incl = 0;
        if (__ballot(has)) {
            uint32_t omask = 0;
#pragma unroll
            for (int i = 0; i < 8; i++)
                if (i < (int)nv && code[i] == 0) omask |= 1u << i;
            packed = __popc(omask) | (__popc(pm_lane) << 16);
            incl = wave_incl_scan(packed);
            if (lane == 63) wsum[wave] = incl;
            if (omask | pm_lane) {
                // positions go to this tile's staging slots after the barrier
                code[0] = omask;  // keep the masks; codes are no longer needed
            }
        } else if (lane == 0) {
            wsum[wave] = 0;
        }
        __syncthreads();
        uint32_t wpre = 0, tot = 0;
#pragma unroll
        for (uint32_t w = 0; w < 4; w++) {
            const uint32_t v = wsum[w];
            wpre += (w < wave) ? v : 0u;
            tot += v;
        }
        if (t == 0) tile_cnt[tile] = tot;
        if (packed) {
            const uint32_t omask = code[0];
            const uint32_t excl_local = wpre + incl - packed;
            const uint64_t slot = (uint64_t)tile * kTileBlocks * kBlockElems;
            uint2* op = ostage + slot + (excl_local & 0xFFFFu);
            uint2* pp = pstage + slot + (excl_local >> 16);
            const uint32_t pos0 = b * kBlockElems + s * 8;
            const BlockInfo ib = block_info(g, b);
            const uint32_t base = ib.bx * g.bs[0] + g.n[0] * (ib.by * g.bs[1] + g.n[1] * (ib.bz * g.bs[2])) +
                                  lb_rowoff;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                if (omask & (1u << i)) *op++ = make_uint2(pos0 + i, (uint32_t)d[i]);
                if (pm_lane & (1u << i)) *pp++ = make_uint2(pos0 + i, __float_as_uint(x[base + i]));
            }
        }
        __syncthreads();
    }
    if (MODE == kQuantTrial) return;
    __syncthreads();
    for (uint32_t i = t; i < (uint32_t)kBins; i += 256)
        if (H[i]) atomicAdd(&hist_g[(blockIdx.x % kHistCopies) * kBins + i], H[i]);
}

// ------------------------------------------------------------ launchers
void launch_reset(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2,
                  uint32_t n2, uint64_t* d3, uint32_t n3, uint64_t off_chunks, uint64_t off_stream, uint64_t nreg) {
    uint32_t n = n1 > n2 ? n1 : n2;
    if (n3 > n) n = n3;
    uint32_t grid = (n + 255) / 256;
    if (grid < 4) grid = 4;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, st, misc, hist, d1, n1, d2, n2, d3, n3, off_chunks,
                       off_stream, nreg);
}

void launch_minmax(hipStream_t st, const float* x, uint64_t N, int vec, Misc* misc, int grid) {
    hipLaunchKernelGGL(k_minmax, dim3(grid), dim3(256), 0, st, x, N, vec, misc);
}

#define FZ_QUANT(NDV, MV)                                                                                        \
    hipLaunchKernelGGL((k_quant<NDV, MV>), dim3(grid), dim3(256), 0, st, x, g, mode, eb, vec, misc, hist, codes, \
                       ntiles, tile_cnt, ostage, pstage, fixed_pred, bpred, coef, cw_ref, choice, costs)

void launch_quant(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                  Misc* misc, uint32_t* hist, uint16_t* codes, uint32_t ntiles, uint32_t* tile_cnt, uint2* ostage,
                  uint2* pstage, int fixed_pred, const uint8_t* bpred, int32_t* coef) {
    const uint32_t* cw_ref = nullptr;
    uint8_t* choice = nullptr;
    uint32_t* costs = nullptr;
    if (fixed_pred == (int)kPredInterp) {
        if (g.ndim == 3) FZ_QUANT(3, kQuantInterp);
        else if (g.ndim == 2) FZ_QUANT(2, kQuantInterp);
        else FZ_QUANT(1, kQuantInterp);
        return;
    }
    if (fixed_pred == (int)kPredGlobal) {
        if (g.ndim == 3) FZ_QUANT(3, kQuantGlobal);
        else if (g.ndim == 2) FZ_QUANT(2, kQuantGlobal);
        else FZ_QUANT(1, kQuantGlobal);
        return;
    }
    const bool pred = fixed_pred != 0;
    if (g.ndim == 3) {
        if (pred) FZ_QUANT(3, kQuantPred); else FZ_QUANT(3, kQuantP0);
    } else if (g.ndim == 2) {
        if (pred) FZ_QUANT(2, kQuantPred); else FZ_QUANT(2, kQuantP0);
    } else {
        if (pred) FZ_QUANT(1, kQuantPred); else FZ_QUANT(1, kQuantP0);
    }
}

void launch_quant_shuffle(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                          Misc* misc, uint32_t* hist, uint32_t* slots, uint32_t ntiles, uint32_t* tile_cnt,
                          uint2* ostage, uint2* pstage) {
    uint16_t* codes = reinterpret_cast<uint16_t*>(slots);
    const int fixed_pred = 0;
    const uint8_t* bpred = nullptr;
    int32_t* coef = nullptr;
    const uint32_t* cw_ref = nullptr;
    uint8_t* choice = nullptr;
    uint32_t* costs = nullptr;
    if (g.ndim == 3) FZ_QUANT(3, kQuantShuffle);
    else if (g.ndim == 2) FZ_QUANT(2, kQuantShuffle);
    else FZ_QUANT(1, kQuantShuffle);
}

void launch_trial(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                  Misc* misc, uint32_t ntiles, const uint32_t* cw_ref, uint8_t* choice, uint32_t* costs) {
    uint32_t* hist = nullptr;
    uint16_t* codes = nullptr;
    uint32_t* tile_cnt = nullptr;
    uint2 *ostage = nullptr, *pstage = nullptr;
    int32_t* coef = nullptr;
    const uint8_t* bpred = nullptr;
    const int fixed_pred = -1;
    if (g.ndim == 3) FZ_QUANT(3, kQuantTrial);
    else if (g.ndim == 2) FZ_QUANT(2, kQuantTrial);
    else FZ_QUANT(1, kQuantTrial);
}

#undef FZ_QUANT

__global__ void k_fill32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v) {
    uint64_t grid = (n + 255) / 256;
    if (grid > 1024) grid = 1024;
    if (grid) hipLaunchKernelGGL(k_fill32, dim3((uint32_t)grid), dim3(256), 0, st, p, n, v);
}

}  // namespace fz
