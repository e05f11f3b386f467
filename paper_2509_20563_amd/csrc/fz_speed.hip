// Bit-shuffle codec: the lossless stage of the throughput-oriented pipeline
// (FZMod-Speed, Sec. 3.3: FZ-GPU's bit-shuffle and dictionary encoding in
// place of Huffman coding).  The same quantisation codes as the Huffman
// path (first-order Lorenzo, radius 512) become 10-bit symbols
//   code 0 (outlier) -> 1023,  code c -> zigzag(c - 512) (0, -1, 1 -> 0, 1, 2),
// a block's 512 symbol slots form 16 groups of 32, each group 10 plane words
// (word p: bit p of the group's symbols, symbol j in bit j), and only the
// non-zero words are kept, flagged in a 160-bit mask per block.
//   (encoder)   - the quantiser builds each block's plane words (lane = 8
//                 consecutive slots, bits transposed by 8 x 8 delta swaps,
//                 the quad's bytes across lanes) and keeps the non-zero
//                 ones with the block's 160-bit mask in a staging slot; a
//                 scan of the masks' popcounts gives each block's first
//                 kept word, and k_shuffle_copy writes masks and words
//   k_unshuffle - one wave per block: lane = 8 consecutive slots (a row),
//                 the lane's group's kept words gathered by mask popcounts,
//                 its byte of each plane transposed back to 8 symbols,
//                 symbols -> residuals (outliers from the list), the
//                 inverse Lorenzo as in-lane and cross-lane prefix sums,
//                 dequantisation, row stores
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {



// In-block coordinates of slot s.
template <int ND>
__device__ __forceinline__ void slot_coords(uint32_t s, uint32_t& lx, uint32_t& ly, uint32_t& lz) {
    if (ND == 3) { lx = s & 7; ly = (s >> 3) & 7; lz = s >> 6; }
    else if (ND == 2) { lx = s & 31; ly = s >> 5; lz = 0; }
    else { lx = s; ly = 0; lz = 0; }
}

// ------------------------------------------------------------- encoder
// The plane words, masks and kept words of each block come from the
// quantiser (k_quant<ND, kQuantShuffle>) in the block's staging slot, and
// the slot scan (SCAN_SLOTS) gives the offset of its first kept word.  A
// wave takes 64 consecutive blocks (lane = block): their mask words go
// after the header, and their kept words, one contiguous run of the
// stream, are written in order: with fewer than 32 kept words per block on
// average lane = output word, its block found by a binary search over the
// wave's word prefix in LDS, else block by block.  Nothing beyond limit
// (the verbatim size: such a container is written verbatim by k_finalize).
__global__ __launch_bounds__(256) void k_shuffle_copy(Geom g, const uint32_t* __restrict__ slots,
                                                      const uint64_t* __restrict__ off, uint8_t* __restrict__ out,
                                                      uint64_t limit) {
    __shared__ uint32_t s_pre[4][64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * 4;
    const uint64_t words_at = align16((uint64_t)kHdr + 4ull * kMaskWords * g.nblocks);
    uint32_t* outw = reinterpret_cast<uint32_t*>(out);
    uint32_t* P = s_pre[wave];
    for (uint64_t c0 = ((uint64_t)blockIdx.x * 4 + wave) * 64; c0 < g.nblocks; c0 += nw * 64) {
        const uint64_t b = c0 + lane;
        const bool in = b < g.nblocks;
        const uint32_t* S = slots + (uint64_t)kShufSlot * (in ? b : c0);
        uint32_t m[kMaskWords];
#pragma unroll
        for (int k = 0; k < kMaskWords; k++) m[k] = in ? S[k] : 0u;
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < kMaskWords; k++) {
            cnt += (uint32_t)__popc(m[k]);
            const uint64_t at = (uint64_t)kHdr + 4ull * (kMaskWords * b + k);
            if (in && at + 4 <= limit) outw[at >> 2] = m[k];
        }
        const uint32_t incl = wave_incl_scan(cnt);
        P[lane] = incl - cnt;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        const uint64_t base = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)off[c0]) |
                               ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(off[c0] >> 32))
                                << 32));
        __builtin_amdgcn_wave_barrier();
        if (total >= 64u * 32u) {
            // dense (32 or more kept words per block on average): block by
            // block, lane = word of the block
            // four blocks at a time, every load issued before the stores
            for (uint32_t k0 = 0; k0 < 64; k0 += 4) {
                uint32_t v[4][3];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)cnt, (int)(k0 + u));
                    const uint32_t* src = slots + (uint64_t)kShufSlot * (c0 + k0 + u) + kMaskWords;
#pragma unroll
                    for (int r = 0; r < 3; r++) {
                        const uint32_t j = lane + 64 * r;
                        v[u][r] = j < ck ? src[j] : 0u;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)cnt, (int)(k0 + u));
                    const uint32_t pk = P[k0 + u];
#pragma unroll
                    for (int r = 0; r < 3; r++) {
                        const uint32_t j = lane + 64 * r;
                        const uint64_t at = words_at + 4 * (base + pk + j);
                        if (j < ck && at + 4 <= limit) outw[at >> 2] = v[u][r];
                    }
                }
            }
        } else {
            for (uint32_t q = lane; q < total; q += 64) {
                // the last block whose first word is at or before q
                uint32_t k = 0;
#pragma unroll
                for (uint32_t st = 32; st > 0; st >>= 1)
                    if (P[k + st] <= q) k += st;
                const uint64_t at = words_at + 4 * (base + q);
                if (at + 4 <= limit) outw[at >> 2] = slots[(uint64_t)kShufSlot * (c0 + k) + kMaskWords + (q - P[k])];
            }
        }
        __builtin_amdgcn_wave_barrier();
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
void launch_shuffle_copy(hipStream_t st, const Geom& g, const uint32_t* slots, const uint64_t* off, uint8_t* out,
                         uint64_t limit) {
    // 64 blocks per wave, 4 waves per workgroup
    uint32_t grid = (uint32_t)((g.nblocks + 255) / 256);
    if (grid > 8192) grid = 8192;
    if (!grid) return;
    hipLaunchKernelGGL(k_shuffle_copy, dim3(grid), dim3(256), 0, st, g, slots, off, out, limit);
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
