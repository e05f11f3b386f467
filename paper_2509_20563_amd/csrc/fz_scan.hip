// Exclusive prefix scans over per-tile or per-block counts, single pass
// with decoupled look-back (one workgroup per 1024 entries, so a 512^3 field
// needs 64 workgroups and one counter atomic each):
//   SCAN_COUNTS - packed (outliers | patches << 16) per quantisation tile ->
//                 packed prefix (outliers: 31 bits, patches: 31 bits above)
//   SCAN_CHUNKS - u16 bit count per block (container) -> bit offset per block
//   SCAN_PMAP   - per-block predictor (u8) -> index of each regression block
//                 among the regression blocks; sets the section offsets
//   SCAN_MASKS  - per-block plane-word mask (5 u32, bit-shuffle codec) ->
//                 offset of the block's first kept word
//   SCAN_SLOTS  - the same from the encoder's staging slots (the mask at the
//                 start of each kShufSlot-word slot); the total kept words
//                 go to misc->total_bits_enc
#include <type_traits>

#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

constexpr int kScanTile = 1024;  // entries per workgroup (256 threads x 4)

template <int KIND>
__global__ __launch_bounds__(256) void k_scan(const void* __restrict__ in, uint32_t n, uint64_t* __restrict__ out,
                                              uint64_t* desc, uint32_t* ctr, uint32_t ntiles, Misc* misc,
                                              uint64_t expect) {
    // packed pairs: (outliers, patches); for the map (regression blocks,
    // blocks off first-order Lorenzo)
    constexpr bool PAIR = KIND == SCAN_COUNTS || KIND == SCAN_PMAP;
    using Op = typename std::conditional<PAIR, OpPair31, OpAdd>::type;
    const Op op;
    __shared__ uint64_t wsum[4];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) s_tile = atomicAdd(ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;
    const uint64_t base = (uint64_t)tile * kScanTile + 4 * t;
    uint64_t v[4];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint64_t e = 0;
        if (base + k < n) {
            if (KIND == SCAN_COUNTS) {
                const uint32_t c = static_cast<const uint32_t*>(in)[base + k];
                e = (uint64_t)(c & 0xFFFFu) | ((uint64_t)(c >> 16) << 31);
            } else if (KIND == SCAN_PMAP) {
                const uint8_t pr = static_cast<const uint8_t*>(in)[base + k];
                e = (pr == 2 ? 1ull : 0ull) | ((pr != 0 ? 1ull : 0ull) << 31);
            } else if (KIND == SCAN_MASKS || KIND == SCAN_SLOTS) {
                const uint32_t* m =
                    static_cast<const uint32_t*>(in) + (KIND == SCAN_SLOTS ? kShufSlot : kMaskWords) * (base + k);
                e = __popc(m[0]) + __popc(m[1]) + __popc(m[2]) + __popc(m[3]) + __popc(m[4]);
            } else {
                e = static_cast<const uint16_t*>(in)[base + k];
            }
        }
        v[k] = e;
        sum = op(sum, e);
    }
    const uint64_t incl = wave_incl_scan64(sum, op);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t wpre = 0, T = 0;
    for (uint32_t w = 0; w < 4; w++) {
        if (w < wave) wpre = op(wpre, wsum[w]);
        T = op(T, wsum[w]);
    }
    if (wave == 0) {
        const uint64_t ex = lookback(desc, tile, T, op, &misc->flags);
        if (lane == 0) {
            s_excl = ex;
            if (tile == ntiles - 1) {
                const uint64_t total = op(ex, T);
                if (KIND == SCAN_COUNTS) {
                    const uint64_t m = (1ull << 31) - 1;
                    misc->n_out = total & m;
                    misc->n_pat = total >> 31;
                    if ((total & m) == m || (total >> 31) == m) atomicOr(&misc->flags, F_OVERFLOW);
                } else if (KIND == SCAN_PMAP) {
                    // regression blocks decide where the chunk table starts;
                    // the map (a quarter byte per block) is kept only when at
                    // least one block in 64 leaves first-order Lorenzo, else
                    // every block is coded first-order and there is no map
                    const uint64_t m = (1ull << 31) - 1;
                    const bool map = 64 * (total >> 31) >= (uint64_t)n;
                    const uint64_t nreg = map ? (total & m) : 0;
                    const Layout L = make_layout(n, map, nreg, 0, 0, 0);
                    misc->nreg = nreg;
                    misc->map_off = map ? 0u : 1u;
                    misc->off_chunks = L.chunks;
                    misc->off_stream = L.stream;
                } else if (KIND == SCAN_SLOTS) {
                    misc->total_bits_enc = total;
                } else if (total != expect) {
                    atomicOr(&misc->flags, F_CORRUPT);
                }
            }
        }
    }
    __syncthreads();
    // exclusive prefix of this thread's first entry: the wave-exclusive part
    // (exact: no field saturates inside one tile), earlier waves, the tile
    uint64_t excl_wave;
    if (PAIR) {
        const uint64_t m = (1ull << 31) - 1;
        excl_wave = ((incl & m) - (sum & m)) | (((incl >> 31) - (sum >> 31)) << 31);
    } else {
        excl_wave = incl - sum;
    }
    uint64_t p = op(op(s_excl, wpre), excl_wave);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        // the map's output is the regression-block index alone
        if (base + k < n) out[base + k] = KIND == SCAN_PMAP ? (p & ((1ull << 31) - 1)) : p;
        p = op(p, v[k]);
    }
}

void launch_scan(hipStream_t st, int kind, const void* in, uint32_t n, uint64_t* out, uint64_t* desc, uint32_t* ctr,
                 Misc* misc, uint64_t expect) {
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles == 0) return;
    if (kind == SCAN_COUNTS)
        hipLaunchKernelGGL(k_scan<SCAN_COUNTS>, dim3(ntiles), dim3(256), 0, st, in, n, out, desc, ctr, ntiles, misc,
                           expect);
    else if (kind == SCAN_PMAP)
        hipLaunchKernelGGL(k_scan<SCAN_PMAP>, dim3(ntiles), dim3(256), 0, st, in, n, out, desc, ctr, ntiles, misc,
                           expect);
    else if (kind == SCAN_MASKS)
        hipLaunchKernelGGL(k_scan<SCAN_MASKS>, dim3(ntiles), dim3(256), 0, st, in, n, out, desc, ctr, ntiles, misc,
                           expect);
    else if (kind == SCAN_SLOTS)
        hipLaunchKernelGGL(k_scan<SCAN_SLOTS>, dim3(ntiles), dim3(256), 0, st, in, n, out, desc, ctr, ntiles, misc,
                           expect);
    else
        hipLaunchKernelGGL(k_scan<SCAN_CHUNKS>, dim3(ntiles), dim3(256), 0, st, in, n, out, desc, ctr, ntiles, misc,
                           expect);
}

uint32_t scan_tiles(uint32_t n) { return (n + kScanTile - 1) / kScanTile; }

}  // namespace fz
