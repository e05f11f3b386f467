// Bit-shuffle codec: the lossless stage of the throughput-oriented pipeline
// (FZMod-Speed, Sec. 3.3: FZ-GPU's bit-shuffle and dictionary encoding in
// place of Huffman coding).  The same quantisation codes as the Huffman
// path (first-order Lorenzo, radius 512) become 10-bit symbols
//   code 0 (outlier) -> 1023,  code c -> zigzag(c - 512) (0, -1, 1 -> 0, 1, 2),
// a block's 512 symbol slots form 16 groups of 32, each group 10 plane words
// (word p: bit p of the group's symbols, symbol j in bit j), and only the
// non-zero words are kept, flagged in a 160-bit mask per block.
//   k_shuffle   - one wave per block: lane = 8 consecutive slots (one
//                 16-byte code load), their symbols' bits transposed (8 x 8
//                 delta swaps) to one byte per plane, the quad's bytes
//                 transposed across lanes to the group's plane words;
//                 per-block masks and word counts; a workgroup of 32
//                 blocks finds its first kept word by decoupled look-back
//                 and writes its masks and kept words
//   k_unshuffle - one wave per block: lane = 8 consecutive slots (a row),
//                 the lane's group's kept words gathered by mask popcounts,
//                 its byte of each plane transposed back to 8 symbols,
//                 symbols -> residuals (outliers from the list), the
//                 inverse Lorenzo as in-lane and cross-lane prefix sums,
//                 dequantisation, row stores
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

constexpr int kShufBlocks = 32;  // blocks per workgroup (8 per wave)
constexpr int kGroups = kBlockElems / 32;  // 32-symbol groups per block

uint32_t shuffle_groups(uint32_t nblocks) { return (nblocks + kShufBlocks - 1) / kShufBlocks; }

// In-block coordinates of slot s.
template <int ND>
__device__ __forceinline__ void slot_coords(uint32_t s, uint32_t& lx, uint32_t& ly, uint32_t& lz) {
    if (ND == 3) { lx = s & 7; ly = (s >> 3) & 7; lz = s >> 6; }
    else if (ND == 2) { lx = s & 31; ly = s >> 5; lz = 0; }
    else { lx = s; ly = 0; lz = 0; }
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
    // the plane words of this wave's blocks through LDS (one block at a
    // time), read back with lane = word index mod 64
    __shared__ uint32_t s_words[4][kGroups * kPlanes];
    uint32_t* W = s_words[wave];
    // quad byte transpose selectors (v_perm): step 1 pairs lanes k, k ^ 1
    // (bytes), step 2 pairs k, k ^ 2 (16-bit halves)
    const uint32_t k4 = lane & 3;
    const uint32_t sel1 = (k4 & 1) ? 0x03070105u : 0x06020400u;
    const uint32_t sel2 = (k4 & 2) ? 0x03020706u : 0x05040100u;
    auto quad_t = [&](uint32_t v) {
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // lane ^ 1
        const uint32_t t1 = __builtin_amdgcn_perm(p1, v, sel1);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)t1, 0x4E, 0xF, 0xF, false);  // lane ^ 2
        return __builtin_amdgcn_perm(p2, t1, sel2);
    };
    // the kept words of this wave's blocks, lane = word index mod 64
    uint32_t kw[8][3];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t b = grp * kShufBlocks + wave * 8 + i;
        uint32_t w0 = 0, w1 = 0, w2 = 0;
        if (b < g.nblocks) {  // uniform over the wave
            const BlockInfo bi = block_info(g, b);
            // lane = 8 consecutive slots 8 lane + j of group lane / 4,
            // symbol 8 (lane & 3) + j of its plane words
            const uint4 cv = *reinterpret_cast<const uint4*>(codes + (uint64_t)b * kBlockElems + 8 * lane);
            const uint32_t c8[8] = {cv.x & 0xFFFFu, cv.x >> 16, cv.y & 0xFFFFu, cv.y >> 16,
                                    cv.z & 0xFFFFu, cv.z >> 16, cv.w & 0xFFFFu, cv.w >> 16};
            uint64_t lo = 0, hi = 0;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                uint32_t lx, ly, lz;
                slot_coords<ND>(8 * lane + j, lx, ly, lz);
                const bool valid = lx < bi.ex && ly < bi.ey && lz < bi.ez;
                const uint32_t sv = valid ? fold_code(c8[j]) : 0u;
                lo |= (uint64_t)(sv & 0xFFu) << (8 * j);
                hi |= (uint64_t)(sv >> 8) << (8 * j);
            }
            // transposed: byte p = plane p's 8 bits of this lane's slots
            const uint64_t tl = transpose8(lo), th = transpose8(hi);
            // across the quad: lane 4 g + k gets the words of planes k,
            // 4 + k (and 8 + k for k < 2) of group g
            const uint32_t wa = quad_t((uint32_t)tl), wb = quad_t((uint32_t)(tl >> 32)), wc = quad_t((uint32_t)th);
            const uint32_t g0 = (lane >> 2) * kPlanes;
            W[g0 + k4] = wa;
            W[g0 + 4 + k4] = wb;
            if (k4 < 2) W[g0 + 8 + k4] = wc;
            __builtin_amdgcn_wave_barrier();
            w0 = W[lane];
            w1 = W[64 + lane];
            w2 = lane < kGroups * kPlanes - 128 ? W[128 + lane] : 0u;
            __builtin_amdgcn_wave_barrier();
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
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    for (uint32_t b = b0; b < g.nblocks; b += nw) {  // wave-uniform: masks and offset by scalar loads
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
        const uint32_t bo = 8 * (lane & 3);
        uint32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        // a block whose groups keep no word has only zero symbols; else the
        // ten plane loads are issued together (a plane the group does not
        // keep reads word 0 and is masked), so their latencies overlap
        if (__ballot(field != 0) && nkept) {
            uint32_t pb[kPlanes];  // this lane's 8 bits of each plane word
            uint64_t idx = base + before;
#pragma unroll
            for (int p = 0; p < kPlanes; p++) {
                const uint32_t has = (field >> p) & 1u;
                const bool use = has && idx < nkept;
                bad |= has && !use;
                const uint32_t v = kept[use ? idx : 0];
                pb[p] = use ? (v >> bo) & 0xFFu : 0u;
                idx += has;
            }
            // planes 0-7 as the rows of an 8 x 8 bit matrix: transposed,
            // byte i holds bits 0-7 of symbol i; planes 8-9 likewise
            const uint64_t lo8 = (uint64_t)(pb[0] | pb[1] << 8 | pb[2] << 16 | pb[3] << 24) |
                                 (uint64_t)(pb[4] | pb[5] << 8 | pb[6] << 16 | pb[7] << 24) << 32;
            const uint64_t tl = transpose8(lo8);
#pragma unroll
            for (int i = 0; i < 8; i++) s[i] = (uint32_t)(tl >> (8 * i)) & 0xFFu;
            if (__ballot((field >> 8) != 0)) {
                const uint64_t th = transpose8((uint64_t)(pb[8] | pb[9] << 8));
#pragma unroll
                for (int i = 0; i < 8; i++) s[i] |= ((uint32_t)(th >> (8 * i)) & 3u) << 8;
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
