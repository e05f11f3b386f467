// Bit-shuffle codec: the lossless stage of the throughput-oriented pipeline
// (FZMod-Speed, Sec. 3.3: FZ-GPU's bit-shuffle and dictionary encoding in
// place of Huffman coding).  The same quantisation codes as the Huffman
// path (first-order Lorenzo, radius 512) become 10-bit symbols
//   code 0 (outlier) -> 1023,  code c -> zigzag(c - 512) (0, -1, 1 -> 0, 1, 2),
// a block's 512 symbol slots form 16 groups of 32, each group 10 plane words
// (word p: bit p of the group's symbols, symbol j in bit j), and only the
// non-zero words are kept, flagged in a 160-bit mask per block.
//   k_shuffle   - one wave per block: symbols by lane (slot 64 r + lane in
//                 round r), one ballot per plane and round gives two plane
//                 words; per-block masks and word counts; a workgroup of 32
//                 blocks finds its first kept word by decoupled look-back
//                 and writes its masks and kept words
//   k_unshuffle - one wave per block: lane = 8 consecutive slots (a row),
//                 the lane's group's kept words gathered by mask popcounts,
//                 symbols -> residuals (outliers from the list), the
//                 inverse Lorenzo as in-lane and cross-lane prefix sums,
//                 dequantisation, row stores
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

constexpr int kShufBlocks = 32;  // blocks per workgroup (8 per wave)

uint32_t shuffle_groups(uint32_t nblocks) { return (nblocks + kShufBlocks - 1) / kShufBlocks; }

// In-block coordinates of slot s.
template <int ND>
__device__ __forceinline__ void slot_coords(uint32_t s, uint32_t& lx, uint32_t& ly, uint32_t& lz) {
    if (ND == 3) { lx = s & 7; ly = (s >> 3) & 7; lz = s >> 6; }
    else if (ND == 2) { lx = s & 31; ly = s >> 5; lz = 0; }
    else { lx = s; ly = 0; lz = 0; }
}

// Symbol of a quantisation code.
__device__ __forceinline__ uint32_t fold_code(uint32_t code) {
    const int32_t d = (int32_t)code - kRadius;
    const uint32_t z = ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
    return code ? z : kSymOutlier;
}

// ------------------------------------------------------------- encoder
template <int ND>
__global__ __launch_bounds__(256) void k_shuffle(Geom g, const uint16_t* __restrict__ codes, uint8_t* __restrict__ out,
                                                 uint64_t limit, uint64_t* desc, uint32_t ngroups, Misc* misc) {
    __shared__ uint32_t s_group;
    __shared__ uint32_t s_cnt[kShufBlocks];
    __shared__ uint32_t s_pre[kShufBlocks];
    __shared__ uint64_t s_mask[kShufBlocks][3];
    __shared__ uint64_t s_base;
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) s_group = atomicAdd(&misc->xtile_ctr, 1u);
    __syncthreads();
    const uint32_t grp = s_group;
    if (grp >= ngroups) return;
    // the kept words of this wave's blocks, lane = word index mod 64
    uint32_t kw[8][3];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t b = grp * kShufBlocks + wave * 8 + i;
        uint32_t w0 = 0, w1 = 0, w2 = 0;
        if (b < g.nblocks) {
            const BlockInfo bi = block_info(g, b);
            const uint16_t* cb = codes + (uint64_t)b * kBlockElems;
            uint32_t s[8];
#pragma unroll
            for (int r = 0; r < 8; r++) {
                const uint32_t slot = 64 * r + lane;
                uint32_t lx, ly, lz;
                slot_coords<ND>(slot, lx, ly, lz);
                const bool valid = lx < bi.ex && ly < bi.ey && lz < bi.ez;
                s[r] = valid ? fold_code(cb[slot]) : 0u;
            }
            // planes above the block's highest symbol bit, and rounds whose
            // 64 symbols are all zero, hold only zero words (wave-uniform
            // skips)
            uint32_t orl = s[0] | s[1] | s[2] | s[3] | s[4] | s[5] | s[6] | s[7];
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) orl |= (uint32_t)__shfl_xor((int)orl, d, 64);
            const int P = 32 - __clz((int)orl);
            // round r covers groups 2r (low half of each ballot) and 2r + 1;
            // word k = 10 group + plane goes to lane k mod 64, slot k / 64
#pragma unroll
            for (int r = 0; r < 8; r++) {
                if (!__ballot(s[r] != 0)) continue;
#pragma unroll
                for (int p = 0; p < kPlanes; p++) {
                    if (p >= P) break;
                    const uint64_t bal = __ballot((s[r] >> p) & 1u);
                    const uint32_t k0 = (2 * r) * kPlanes + p, k1 = k0 + kPlanes;
                    const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
                    if (lane == (k0 & 63)) {
                        if ((k0 >> 6) == 0) w0 = lo;
                        else if ((k0 >> 6) == 1) w1 = lo;
                        else w2 = lo;
                    }
                    if (lane == (k1 & 63)) {
                        if ((k1 >> 6) == 0) w0 = hi;
                        else if ((k1 >> 6) == 1) w1 = hi;
                        else w2 = hi;
                    }
                }
            }
        }
        kw[i][0] = w0;
        kw[i][1] = w1;
        kw[i][2] = w2;
        const uint64_t m0 = __ballot(w0 != 0), m1 = __ballot(w1 != 0), m2 = __ballot(w2 != 0);
        if (lane == 0) {
            s_mask[wave * 8 + i][0] = m0;
            s_mask[wave * 8 + i][1] = m1;
            s_mask[wave * 8 + i][2] = m2;
            s_cnt[wave * 8 + i] = (uint32_t)(__popcll(m0) + __popcll(m1) + __popcll(m2));
        }
    }
    __syncthreads();
    // the group's block prefix and total; its first kept word by look-back
    if (wave == 0) {
        const uint32_t c = lane < kShufBlocks ? s_cnt[lane] : 0u;
        const uint32_t incl = wave_incl_scan(c);
        if (lane < kShufBlocks) s_pre[lane] = incl - c;
        const uint64_t T = __shfl(incl, 63, 64);
        const uint64_t ex = lookback(desc, grp, T, OpAdd(), &misc->flags);
        if (lane == 0) {
            s_base = ex;
            if (grp == ngroups - 1) misc->total_bits_enc = ex + T;
        }
    }
    __syncthreads();
    const uint64_t words_at = align16((uint64_t)kHdr + 4ull * kMaskWords * g.nblocks);
    uint32_t* outw = reinterpret_cast<uint32_t*>(out);
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t bl = wave * 8 + i;
        const uint32_t b = grp * kShufBlocks + bl;
        if (b >= g.nblocks) break;
        const uint64_t m0 = s_mask[bl][0], m1 = s_mask[bl][1], m2 = s_mask[bl][2];
        // the 5 mask words (bits 0..159)
        if (lane < kMaskWords) {
            const uint64_t at = (uint64_t)kHdr + 4ull * (kMaskWords * (uint64_t)b + lane);
            const uint32_t mv = lane == 0 ? (uint32_t)m0
                              : lane == 1 ? (uint32_t)(m0 >> 32)
                              : lane == 2 ? (uint32_t)m1
                              : lane == 3 ? (uint32_t)(m1 >> 32)
                                          : (uint32_t)m2;
            if (at + 4 <= limit) outw[at >> 2] = mv;
        }
        const uint64_t base = s_base + s_pre[bl];
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        const uint32_t c0 = (uint32_t)__popcll(m0), c1 = (uint32_t)__popcll(m1);
        const uint32_t wv[3] = {kw[i][0], kw[i][1], kw[i][2]};
        const uint64_t mm[3] = {m0, m1, m2};
        const uint32_t before[3] = {0u, c0, c0 + c1};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (wv[j]) {
                const uint64_t idx = base + before[j] + (uint32_t)__popcll(mm[j] & below);
                const uint64_t at = words_at + 4 * idx;
                if (at + 4 <= limit) outw[at >> 2] = wv[j];
            }
        }
    }
}

// ------------------------------------------------------------- decoder
template <int ND>
__global__ __launch_bounds__(256) void k_unshuffle(Geom g, const uint32_t* __restrict__ masks,
                                                   const uint32_t* __restrict__ kept, uint64_t nkept,
                                                   const uint64_t* __restrict__ off, const uint32_t* __restrict__ opos,
                                                   const int32_t* __restrict__ oval, const uint2* __restrict__ oidx,
                                                   uint64_t n_out, double e2, float* __restrict__ out, int vec,
                                                   Misc* misc) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * 4;
    bool bad = false;
    for (uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6); b < g.nblocks; b += nw) {
        const uint32_t* mb = masks + (uint64_t)kMaskWords * b;
        const uint32_t mw0 = mb[0], mw1 = mb[1], mw2 = mb[2], mw3 = mb[3], mw4 = mb[4];
        const uint64_t base = off[b];
        // this lane's group (lane / 4) and its 10 mask bits
        const uint32_t kbit = 10 * (lane >> 2);
        const uint32_t a = kbit >> 5, sh = kbit & 31;
        const uint32_t wa = a == 0 ? mw0 : a == 1 ? mw1 : a == 2 ? mw2 : a == 3 ? mw3 : mw4;
        const uint32_t wb = a == 0 ? mw1 : a == 1 ? mw2 : a == 2 ? mw3 : a == 3 ? mw4 : 0u;
        const uint32_t field = (uint32_t)((((uint64_t)wb << 32) | wa) >> sh) & 0x3FFu;
        // kept words before the group: whole mask words below a, then the
        // bits of word a below sh
        uint32_t before = (uint32_t)__popc(wa & ((1u << sh) - 1u));
        before += (a > 0 ? __popc(mw0) : 0) + (a > 1 ? __popc(mw1) : 0) + (a > 2 ? __popc(mw2) : 0) +
                  (a > 3 ? __popc(mw3) : 0);
        // planes no group of the block keeps are zero for every lane
        uint32_t orf = field;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) orf |= (uint32_t)__shfl_xor((int)orf, d, 64);
        const int P = 32 - __clz((int)orf);
        const uint32_t bo = 8 * (lane & 3);
        uint32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (P) {
            uint32_t pb[kPlanes];  // this lane's 8 bits of each plane word
#pragma unroll
            for (int p = 0; p < kPlanes; p++) {
                pb[p] = 0;
                if (p >= P) continue;
                const uint64_t idx = base + before + (uint32_t)__popc(field & ((1u << p) - 1u));
                const bool has = (field >> p) & 1u;
                const bool inb = idx < nkept;
                bad |= has && !inb;
                pb[p] = (has && inb) ? (kept[idx] >> bo) & 0xFFu : 0u;
            }
#pragma unroll
            for (int p = 0; p < kPlanes; p++) {
                if (p >= P) break;
#pragma unroll
                for (int i = 0; i < 8; i++) s[i] |= ((pb[p] >> i) & 1u) << p;
            }
        }
        const BlockInfo bi = block_info(g, b);
        uint32_t nvalid;
        const uint64_t row = seg_index<ND>(g, bi, lane, nvalid);
        int32_t d[8];
        uint32_t nol = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t sv = s[i];
            d[i] = (int32_t)((sv >> 1) ^ (0u - (sv & 1u)));
            nol += ((uint32_t)i < nvalid && sv == kSymOutlier) ? 1u : 0u;
        }
        const uint32_t oincl = wave_incl_scan(nol);
        const uint32_t ototal = __shfl(oincl, 63, 64);
        const uint2 span = (n_out && ototal) ? oidx[b] : make_uint2(0, 0);
        if (ototal) {
            // outliers of the block in slot order: rank = earlier lanes'
            // outliers + earlier ones in this lane
            bad |= (span.y - span.x) != ototal;
            uint32_t r = span.x + oincl - nol;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                if ((uint32_t)i < nvalid && s[i] == kSymOutlier) {
                    const bool ok = r < span.y && (uint64_t)r < n_out &&
                                    opos[r] == (uint32_t)(b * kBlockElems + 8 * lane + i);
                    bad |= !ok;
                    d[i] = ok ? oval[r] : 0;
                    r++;
                }
            }
        } else if (n_out) {
            // a listed outlier that no symbol claims
            const uint2 sp = oidx[b];
            bad |= sp.y != sp.x;
        }
        block_prefix<ND>(d, lane);
        if (nvalid) {
            float f[8];
#pragma unroll
            for (int i = 0; i < 8; i++) f[i] = (float)((double)d[i] * e2);
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

// ------------------------------------------------------------ launchers
void launch_shuffle(hipStream_t st, const Geom& g, const uint16_t* codes, uint8_t* out, uint64_t limit,
                    uint64_t* desc, Misc* misc) {
    const uint32_t ng = shuffle_groups(g.nblocks);
    if (!ng) return;
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_shuffle<3>, dim3(ng), dim3(256), 0, st, g, codes, out, limit, desc, ng, misc);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_shuffle<2>, dim3(ng), dim3(256), 0, st, g, codes, out, limit, desc, ng, misc);
    else
        hipLaunchKernelGGL(k_shuffle<1>, dim3(ng), dim3(256), 0, st, g, codes, out, limit, desc, ng, misc);
}

void launch_unshuffle(hipStream_t st, const Geom& g, const uint32_t* masks, const uint32_t* kept, uint64_t nkept,
                      const uint64_t* off, const uint32_t* opos, const int32_t* oval, const uint2* oidx,
                      uint64_t n_out, double e2, float* out, Misc* misc) {
    uint32_t grid = (g.nblocks + 3) / 4;
    if (grid > 8192) grid = 8192;
    if (!grid) return;
    const int vec = ((uintptr_t)out & 15) == 0 && (g.ndim == 1 || (g.n[0] & 3) == 0);
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_unshuffle<3>, dim3(grid), dim3(256), 0, st, g, masks, kept, nkept, off, opos, oval,
                           oidx, n_out, e2, out, vec, misc);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_unshuffle<2>, dim3(grid), dim3(256), 0, st, g, masks, kept, nkept, off, opos, oval,
                           oidx, n_out, e2, out, vec, misc);
    else
        hipLaunchKernelGGL(k_unshuffle<1>, dim3(grid), dim3(256), 0, st, g, masks, kept, nkept, off, opos, oval,
                           oidx, n_out, e2, out, vec, misc);
}

}  // namespace fz
