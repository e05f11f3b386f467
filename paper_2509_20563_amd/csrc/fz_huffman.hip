// Huffman stages of compression (FZModules Sec. 3.2: the Huffman encoder
// builds its code from the histogram of quantisation codes; FZMod-Default
// runs this on the CPU, here it runs on the GPU):
//   k_codebook - length-limited minimum-redundancy code lengths by
//                package-merge in one workgroup, canonical codewords;
//   k_encode   - chunked encoding (chunk = block) in one pass over the
//                codes, stream offsets by a look-back over tile groups,
//                words assembled in LDS;
//   k_finalize - tile-boundary words, outlier/patch sections, header, or
//                the verbatim container.
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// ------------------------------------------------------------ codebook
// Package-merge (Larmore & Hirschberg): leaves = used symbols sorted by
// (count, symbol); list[kLmax] = leaves; list[l] = merge(leaves,
// packages of list[l+1]) with equal weights putting the leaf first; select
// the first 2n-2 items of list[1], each selected package standing for the
// next two items one level deeper.  A symbol's length is the number of
// levels at which it is selected.  Leaves keep their sorted order in every
// list, so a level is summarised by a bitmask of leaf positions.
__global__ __launch_bounds__(1024) void k_codebook(uint32_t* __restrict__ hist, uint8_t* __restrict__ out_lens,
                                                   uint32_t* __restrict__ cw, Misc* misc) {
    __shared__ uint64_t key[kBins];
    __shared__ uint64_t la[2 * kBins], lb[2 * kBins];
    __shared__ uint32_t mask[kLmax + 1][64];
    __shared__ uint32_t klev[kLmax + 2];
    __shared__ uint8_t slen[kBins];
    __shared__ uint32_t s_first_unused;
    __shared__ uint64_t red[16];
    __shared__ CanonShared cs;

    const uint32_t t = threadIdx.x;
    // sum the histogram copies; copy 0 keeps the total, the others are
    // cleared
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < kHistCopies; k++) h += hist[k * kBins + t];
    hist[t] = h;
#pragma unroll
    for (int k = 1; k < kHistCopies; k++) hist[k * kBins + t] = 0;
    slen[t] = 0;
    key[t] = h ? (((uint64_t)h << 10) | t) : ~0ull;
    if (t == 0) s_first_unused = kBins;
    const int n = __syncthreads_count(h > 0);

    if (n == 1) {
        if (h == 0) atomicMin(&s_first_unused, t);
        __syncthreads();
        if (h > 0) slen[t] = 1;
        if (t == s_first_unused) slen[t] = 1;
    } else if (n >= 2) {
        // bitonic sort of (count << 10 | symbol), unused symbols last; a
        // thread keeps its key in a register: partners closer than 64 are
        // exchanged inside the wave, farther ones through two alternating
        // LDS buffers (one barrier per such stage)
        uint64_t v = key[t];
        int buf = 0;
        for (uint32_t k = 2; k <= (uint32_t)kBins; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                uint64_t o;
                if (j >= 64) {
                    uint64_t* kb = buf ? lb : la;
                    kb[t] = v;
                    __syncthreads();
                    o = kb[t ^ j];
                    buf ^= 1;
                } else {
                    o = __shfl_xor(v, (int)j, 64);
                }
                const bool keep_min = ((t & j) == 0) == ((t & k) == 0);
                v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
            }
        }
        key[t] = v;
        for (int l = 0; l <= kLmax; l++)
            if (t < 64) mask[l][t] = 0;
        __syncthreads();
        const uint64_t wleaf = (t < (uint32_t)n) ? (key[t] >> 10) : 0;
        if (t < (uint32_t)n) {
            la[t] = wleaf;
            atomicOr(&mask[kLmax][t >> 5], 1u << (t & 31));
        }
        uint64_t* cur = la;
        uint64_t* nxt = lb;
        uint32_t len_cur = n;
        __syncthreads();
        for (int l = kLmax - 1; l >= 1; l--) {
            const uint32_t np = len_cur / 2;
            if (t < (uint32_t)n) {
                // packages strictly lighter than this leaf come before it
                uint32_t lo = 0, hi = np;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (cur[2 * mid] + cur[2 * mid + 1] < wleaf) lo = mid + 1;
                    else hi = mid;
                }
                const uint32_t r = t + lo;
                nxt[r] = wleaf;
                atomicOr(&mask[l][r >> 5], 1u << (r & 31));
            }
            if (t < np) {
                const uint64_t pw = cur[2 * t] + cur[2 * t + 1];
                // leaves not heavier than this package come before it
                uint32_t lo = 0, hi = (uint32_t)n;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if ((key[mid] >> 10) <= pw) lo = mid + 1;
                    else hi = mid;
                }
                nxt[t + lo] = pw;
            }
            __syncthreads();
            uint64_t* tmp = cur;
            cur = nxt;
            nxt = tmp;
            len_cur = (uint32_t)n + np;
        }
        if (t < 64) {
            // leaves among the first `take` items of each level: lane =
            // 32-item word of the level's bitmask, popcounts summed over
            // the wave
            uint32_t take = 2 * (uint32_t)n - 2;
            for (int l = 1; l <= kLmax; l++) {
                if (take > 2 * kBins - 1) take = 2 * kBins - 1;
                const uint32_t w0 = 32 * t;
                const uint32_t w = mask[l][t];
                uint32_t k = take <= w0 ? 0u : (uint32_t)__popc(take - w0 >= 32 ? w : (w & ((1u << (take - w0)) - 1u)));
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) k += __shfl_xor(k, d, 64);
                if (t == 0) klev[l] = k;
                take = 2 * (take - k);
            }
        }
        __syncthreads();
        if (t < (uint32_t)n) {
            uint32_t L = 0;
            for (int l = 1; l <= kLmax; l++) L += (t < klev[l]) ? 1u : 0u;
            slen[key[t] & 1023] = (uint8_t)L;
        }
    }
    __syncthreads();
    const uint32_t len = slen[t];
    const uint32_t code = canonical_code(len, cs);
    cw[t] = code | (len << 16);
    // total stream bits = sum count * length
    uint64_t v = (uint64_t)h * len;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    if (t < 512) out_lens[t] = (uint8_t)(slen[2 * t] | (slen[2 * t + 1] << 4));
    __syncthreads();
    if (t == 0) {
        uint64_t s = 0;
        for (int w = 0; w < 16; w++) s += red[w];
        misc->total_bits_cb = s;
    }
}

// --------------------------------------------------------------- encode
// (hi, lo) |= v << sh as 128-bit values, sh in [0, 127], the result fits.
__device__ __forceinline__ void or_shl128(uint64_t& hi, uint64_t& lo, uint64_t v, uint32_t sh) {
    const bool upper = sh >= 64;
    const uint32_t s = sh & 63;
    hi |= upper ? (v << s) : (s ? (v >> ((64 - s) & 63)) : 0ull);
    lo |= upper ? 0ull : (v << s);
}

// words of one tile at most (every value at kLmax bits)
constexpr int kEncTileWords = kTileBlocks * kBlockElems * kLmax / 32;

// A lane's 8 codes of block b, segment s (from the start of the codes when
// the block or segment holds no values, so the load is unconditional and
// can be issued a tile ahead), and the number of real values among them.
template <int ND>
__device__ __forceinline__ uint4 load_codes(const uint16_t* __restrict__ codes, const Geom& g, uint32_t b,
                                            uint32_t s, uint32_t& nv) {
    nv = 0;
    if (b < g.nblocks) {
        BlockInfo info = block_info(g, b);
        seg_index<ND>(g, info, s, nv);
    }
    const uint64_t at = nv ? (uint64_t)b * kBlockElems + s * 8 : 0;
    return *reinterpret_cast<const uint4*>(&codes[at]);
}

// The (codeword | length << 16) entries of the 8 codes (0 past the real
// values) and their bit count.
__device__ __forceinline__ uint32_t code_entries(const uint4& pk, uint32_t nv, const uint32_t* CW, uint32_t e8[8]) {
    const uint32_t c8[8] = {pk.x & 0xFFFFu, pk.x >> 16, pk.y & 0xFFFFu, pk.y >> 16,
                            pk.z & 0xFFFFu, pk.z >> 16, pk.w & 0xFFFFu, pk.w >> 16};
    uint32_t nb = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t e = CW[c8[i] & (kBins - 1)];
        e8[i] = i < (int)nv ? e : 0u;
        nb += e8[i] >> 16;
    }
    return nb;
}

// Single pass over the codes.  A workgroup takes kEncTiles consecutive
// 4-block tiles: it reads their codes once (all loads issued together, kept
// packed in registers), writes the
// chunk table, publishes the group's bit count and obtains the group's
// stream offset by a decoupled look-back over groups, then writes the bits
// tile by tile.  A group publishes its count before it waits, and waits
// only on groups with lower workgroup index (dispatched before it), so the
// chain never waits on a workgroup that is not running; the wait is bounded
// anyway (F_TIMEOUT).
// tiles per group: 12 measured fastest at 1024^3 (0.88 ms; 4: 1.21, 8:
// 0.93, 16: 0.92); the bits are written in passes of kEncPass tiles
constexpr uint32_t kEncTiles = 12;
constexpr uint32_t kEncPass = 6;
constexpr int kEncWords = (int)kEncPass * kEncTileWords + 8;  // one pass (+ bit offset and window overrun)

template <int ND>
__global__ __launch_bounds__(256) void k_encode(const uint16_t* __restrict__ codes, Geom g,
                                                const uint32_t* __restrict__ cw_g, uint32_t ntiles, Misc* misc,
                                                uint8_t* __restrict__ out, uint64_t* desc,
                                                uint64_t* __restrict__ tile_start, uint32_t* __restrict__ tfirst,
                                                uint32_t* __restrict__ tlast) {
    __shared__ uint32_t CW[kBins];
    __shared__ uint32_t W[kEncWords];  // one pass of tiles
    __shared__ uint32_t s_carry[2];    // a pass's partial last word, for the next pass (by pass parity)
    __shared__ uint32_t wsum[kEncTiles][4];
    __shared__ uint64_t s_excl;
    uint16_t* chunks = reinterpret_cast<uint16_t*>(out + misc->off_chunks);
    uint32_t* stream = reinterpret_cast<uint32_t*>(out + misc->off_stream);
    const uint32_t t = threadIdx.x, lane = t & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(t >> 6));
    for (uint32_t i = t; i < (uint32_t)kBins; i += 256) CW[i] = cw_g[i];
    for (uint32_t i = t; i < (uint32_t)kEncWords; i += 256) W[i] = 0;
    __syncthreads();
    const uint32_t grp = blockIdx.x;
    const uint32_t tile0 = grp * kEncTiles;
    // pass over the group's codes: every tile's codes loaded at once
    // (packed, 4 registers per tile, so the loads' latencies overlap), then
    // the tiles' bit counts and totals; the codeword entries are looked up
    // again when the bits are written
    uint4 pk[kEncTiles];
    uint32_t nvk[kEncTiles];
#pragma unroll
    for (uint32_t k = 0; k < kEncTiles; k++) {
        const uint32_t b = (tile0 + k) * kTileBlocks + wave;
        pk[k] = load_codes<ND>(codes, g, tile0 + k < ntiles ? b : g.nblocks, lane, nvk[k]);
    }
#pragma unroll
    for (uint32_t k = 0; k < kEncTiles; k++) {
        uint32_t e8[8];
        const uint32_t nb = tile0 + k < ntiles ? code_entries(pk[k], nvk[k], CW, e8) : 0u;
        const uint32_t incl = wave_incl_scan(nb);
        if (lane == 63) wsum[k][wave] = incl;
    }
    __syncthreads();
    // chunk table (block bit counts) from the tile totals: no store among
    // the phase's loads, whose waits would otherwise also cover it
    if (t < kEncTiles * 4) {
        const uint32_t k = t >> 2, w = t & 3;
        const uint32_t b = (tile0 + k) * kTileBlocks + w;
        if (tile0 + k < ntiles && b < g.nblocks) chunks[b] = (uint16_t)wsum[k][w];
    }
    uint64_t gsum = 0;
    for (uint32_t k = 0; k < kEncTiles; k++) gsum += wsum[k][0] + wsum[k][1] + wsum[k][2] + wsum[k][3];
    if (wave == 0) {
        const uint64_t ex = lookback(desc, grp, gsum, OpAdd(), &misc->flags);
        if (lane == 0) {
            s_excl = ex;
            if (tile0 + kEncTiles >= ntiles) misc->total_bits_enc = ex + gsum;
        }
    }
    __syncthreads();
    // the bits, in passes of kEncPass tiles: each pass's tiles are OR-ed
    // into one LDS buffer (one barrier), then its words are stored as one
    // contiguous run.  The group's partial first and last words are shared
    // with the neighbouring groups and merged by k_finalize (tile_start of
    // the group's first tile; its other tiles start at 0, nothing to
    // merge); a pass's partial last word is carried into the next pass.
    const uint64_t G0 = s_excl;
    const uint32_t tend = min(tile0 + kEncTiles, ntiles);  // past the group's last tile
    if (t < kEncTiles && tile0 + t < ntiles) tile_start[tile0 + t] = t == 0 ? G0 : 0ull;
    uint64_t G = G0;
#pragma unroll
    for (uint32_t h = 0; h < kEncTiles / kEncPass; h++) {
        const uint32_t k0 = h * kEncPass;
        if (tile0 + k0 >= ntiles) break;  // uniform
        const uint32_t shp = (uint32_t)(G & 31);
        uint32_t rel = 0;  // bits of the pass's earlier tiles
#pragma unroll
        for (uint32_t kk = 0; kk < kEncPass; kk++) {
            const uint32_t k = k0 + kk;
            const uint32_t tile = tile0 + k;
            if (tile >= ntiles) break;  // uniform
            uint32_t wpre = 0, T = 0;
            for (uint32_t w = 0; w < 4; w++) {
                if (w < wave) wpre += wsum[k][w];
                T += wsum[k][w];
            }
            if (t == 0 && tile != ntiles - 1 && T < 32) atomicOr(&misc->flags, F_INTERNAL);
            // the lane's bit string as two shift-or chains of 4 codewords
            // (at most 48 bits each)
            uint32_t e8[8];
            code_entries(pk[k], nvk[k], CW, e8);
            uint64_t a0 = 0, a1 = 0;
            uint32_t n0 = 0, n1 = 0;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t e = e8[i], l = e >> 16;
                a0 = (a0 << l) | (e & 0xFFFFu);
                n0 += l;
            }
#pragma unroll
            for (int i = 4; i < 8; i++) {
                const uint32_t e = e8[i], l = e >> 16;
                a1 = (a1 << l) | (e & 0xFFFFu);
                n1 += l;
            }
            const uint32_t nb = n0 + n1;
            // the scan runs with every lane active (lanes with no bits add 0)
            const uint32_t incl = wave_incl_scan(nb);
            if (nb) {
                // place the string at bit o of word w0 (from the pass's
                // first word), most significant first: 128-bit window
                // (hi, lo) = words w0 .. w0 + 3 (o + nb <= 127)
                const uint32_t p = shp + rel + wpre + incl - nb;
                const uint32_t o = p & 31, w0 = p >> 5;
                uint64_t hi = 0, lo = 0;
                or_shl128(hi, lo, a0, (128 - o - n0) & 127);  // a0 = 0 when n0 = 0
                or_shl128(hi, lo, a1, 128 - o - nb);
                const uint32_t o0 = (uint32_t)(hi >> 32), o1 = (uint32_t)hi, o2 = (uint32_t)(lo >> 32),
                               o3 = (uint32_t)lo;
                if (o0) atomicOr(&W[w0], o0);
                if (o1) atomicOr(&W[w0 + 1], o1);
                if (o2) atomicOr(&W[w0 + 2], o2);
                if (o3) atomicOr(&W[w0 + 3], o3);
            }
            rel += T;
        }
        __syncthreads();
        // the pass's words: the first one shares bits with the previous
        // pass (carried) or group (parked in tfirst), the last one with the
        // next pass (carried) or group (parked in tlast of the group's last
        // tile); the field's very last word is stored
        const bool last_pass = tile0 + k0 + kEncPass >= tend;
        const uint32_t nwords = (shp + rel + 31) >> 5;
        const bool end_part = ((shp + rel) & 31) != 0;
        const uint64_t wbase = G >> 5;
        // pass h reads the slot pass h - 1 wrote and writes the other one:
        // the writer of this pass's carry may run before every thread has
        // read the previous one
        const uint32_t carry_in = s_carry[(h + 1) & 1];
        for (uint32_t w = t; w < nwords; w += 256) {
            uint32_t v = W[w];
            W[w] = 0;
            const bool first = w == 0 && shp != 0, last = w == nwords - 1 && end_part;
            if (first && h > 0) v |= carry_in;
            if (first && h == 0) tfirst[tile0] = v;
            else if (last && !last_pass) s_carry[h & 1] = v;
            else if (last && tend != ntiles) tlast[tend - 1] = v;
            else stream[wbase + w] = v;
        }
        G += rel;
        __syncthreads();
    }
}

// -------------------------------------------------------------- verbatim
// The verbatim container: header (flag bit 0) and the raw floats, written by
// the whole finalize grid.
__device__ void write_verbatim(const Geom& g, uint32_t mode, double eb, uint32_t pred, uint32_t hflags,
                               const Misc* misc, const float* __restrict__ x, uint8_t* __restrict__ out, int vec,
                               uint64_t gid, uint64_t stride) {
    if (gid == 0) {
        double eb_abs;
        resolve_eb(mode, eb, misc->mm_lo, misc->mm_hi, &eb_abs);
        uint8_t h[kHdr];
        for (int k = 0; k < kHdr; k++) h[k] = 0;
        auto st32 = [&](int o, uint32_t v) { for (int k = 0; k < 4; k++) h[o + k] = (uint8_t)(v >> (8 * k)); };
        auto st64 = [&](int o, uint64_t v) { for (int k = 0; k < 8; k++) h[o + k] = (uint8_t)(v >> (8 * k)); };
        st32(0, kMagic);
        h[4] = (uint8_t)kVersion;
        h[5] = (uint8_t)(kVersion >> 8);
        h[6] = (uint8_t)hflags;
        st32(8, g.ndim);
        st32(12, pred);
        st64(16, g.n[0]);
        st64(24, g.n[1]);
        st64(32, g.n[2]);
        st32(40, mode);
        st32(44, kRadius);
        st64(48, __double_as_longlong(eb));
        st64(56, __double_as_longlong(eb_abs));
        st64(64, (uint64_t)kHdr + 4 * g.N);
        uint4* dst = reinterpret_cast<uint4*>(out);
        const uint4* src = reinterpret_cast<const uint4*>(h);
        for (int k = 0; k < kHdr / 16; k++) dst[k] = src[k];
    }
    float* o = reinterpret_cast<float*>(out + kHdr);
    if (vec) {
        const f32x4* x4 = reinterpret_cast<const f32x4*>(x);
        f32x4* o4 = reinterpret_cast<f32x4*>(o);
        for (uint64_t i = gid; i < g.N / 4; i += stride) o4[i] = x4[i];
        for (uint64_t i = (g.N & ~3ull) + gid; i < g.N; i += stride) o[i] = x[i];
    } else {
        for (uint64_t i = gid; i < g.N; i += stride) o[i] = x[i];
    }
}

// ------------------------------------------------------------- finalize
// Layout from the device-side counts; boundary words shared by two tiles;
// outlier and patch sections compacted from the per-tile staging slots in
// tile order (= position order); zero padding; header.  When the packed
// container would not be smaller than the raw floats only the verbatim
// decision is recorded for the host.
__global__ __launch_bounds__(256) void k_finalize(Geom g, uint32_t mode, double eb, uint32_t pred, Misc* misc,
                                                  uint8_t* out, uint32_t ntiles, const uint64_t* __restrict__ tile_start,
                                                  const uint32_t* __restrict__ tfirst,
                                                  const uint32_t* __restrict__ tlast,
                                                  const uint32_t* __restrict__ tile_cnt,
                                                  const uint64_t* __restrict__ tile_off,
                                                  const uint2* __restrict__ ostage, const uint2* __restrict__ pstage,
                                                  const uint8_t* __restrict__ bpred,
                                                  const uint64_t* __restrict__ reg_idx,
                                                  const int32_t* __restrict__ coef, const float* __restrict__ x,
                                                  int xvec, uint32_t codec) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t flags = misc->flags;
    const bool shuffle = codec != 0;
    // Huffman: stream bits; bit-shuffle: kept words (no bit count)
    const uint64_t bits = shuffle ? 0 : misc->total_bits_enc;
    const uint64_t words = shuffle ? misc->total_bits_enc : (bits + 31) / 32;
    const uint64_t nout = misc->n_out, npat = misc->n_pat, nreg = misc->nreg;
    // a per-block choice of first-order Lorenzo everywhere is written as a
    // first-order container (no map)
    if (pred_has_map(pred) && misc->map_off) pred = 0;
    const bool has_map = pred_has_map(pred);
    const Layout L = shuffle ? make_speed_layout(g.nblocks, words, nout, npat)
                             : make_layout(g.nblocks, has_map, nreg, words, nout, npat);
    const bool verbatim = (flags & F_OVERFLOW) || L.total >= (uint64_t)kHdr + 4 * g.N;
    if (gid == 0) {
        if (!shuffle && (bits != misc->total_bits_cb || L.chunks != misc->off_chunks))
            atomicOr(&misc->flags, F_INTERNAL);
        misc->verbatim = verbatim ? 1 : 0;
        misc->total_bytes = verbatim ? (uint64_t)kHdr + 4 * g.N : L.total;
    }
    if (flags & (F_NONFINITE | F_EB | F_INTERNAL | F_TIMEOUT)) return;
    if (verbatim) {
        write_verbatim(g, mode, eb, pred, shuffle ? 1u | kFlagShuffle : 1u, misc, x, out, xvec, gid, stride);
        return;
    }

    // predictor map (2 bits per block) and regression coefficients
    if (has_map)
        for (uint64_t i = gid; i < ((uint64_t)g.nblocks + 3) / 4; i += stride) {
            uint8_t v = 0;
            for (int k = 0; k < 4; k++) {
                const uint64_t b = 4 * i + k;
                if (b < g.nblocks) v |= (uint8_t)((bpred[b] & 3) << (2 * k));
            }
            out[L.map + i] = v;
        }
    if (nreg)
        for (uint64_t b = gid; b < g.nblocks; b += stride) {
            const bool reg = pred == 2 || (has_map && bpred[b] == 2);
            if (!reg) continue;
            const uint64_t r = pred == 2 ? b : reg_idx[b];
            reinterpret_cast<int4*>(out + L.coef)[r] = reinterpret_cast<const int4*>(coef)[b];
        }
    uint32_t* stream = reinterpret_cast<uint32_t*>(out + L.stream);
    for (uint64_t i = gid + 1; !shuffle && i < ntiles; i += stride) {
        const uint64_t G = tile_start[i];
        if (G & 31) stream[G >> 5] = tlast[i - 1] | tfirst[i];
    }
    uint32_t* o_pos = reinterpret_cast<uint32_t*>(out + L.opos);
    int32_t* o_val = reinterpret_cast<int32_t*>(out + L.oval);
    uint32_t* p_pos = reinterpret_cast<uint32_t*>(out + L.ppos);
    uint32_t* p_bits = reinterpret_cast<uint32_t*>(out + L.pbits);
    if (nout | npat) {
        const uint32_t lane = threadIdx.x & 63;
        const uint64_t wid = gid >> 6, nw = stride >> 6;
        const uint64_t m31 = (1ull << 31) - 1;
        for (uint64_t tile = wid; tile < ntiles; tile += nw) {
            const uint32_t c = tile_cnt[tile];
            if (!c) continue;
            const uint64_t off = tile_off[tile];
            const uint64_t slot = tile * (uint64_t)(kTileBlocks * kBlockElems);
            const uint32_t co = c & 0xFFFFu, cp = c >> 16;
            // four entries per lane and pass, all loads issued before the
            // stores (the copy is latency-bound otherwise)
            for (uint32_t j0 = 0; j0 < co; j0 += 256) {
                uint2 a[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t j = j0 + lane + 64 * k;
                    a[k] = j < co ? ostage[slot + j] : make_uint2(0, 0);
                }
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t j = j0 + lane + 64 * k;
                    if (j < co) {
                        o_pos[(off & m31) + j] = a[k].x;
                        o_val[(off & m31) + j] = (int32_t)a[k].y;
                    }
                }
            }
            for (uint32_t j0 = 0; j0 < cp; j0 += 256) {
                uint2 a[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t j = j0 + lane + 64 * k;
                    a[k] = j < cp ? pstage[slot + j] : make_uint2(0, 0);
                }
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t j = j0 + lane + 64 * k;
                    if (j < cp) {
                        p_pos[(off >> 31) + j] = a[k].x;
                        p_bits[(off >> 31) + j] = a[k].y;
                    }
                }
            }
        }
    }
    if (gid == 0) {
        // zero padding between and after sections
        const uint64_t ends[8] = {L.map + (has_map ? ((uint64_t)g.nblocks + 3) / 4 : 0), L.coef + 16 * nreg,
                                  L.chunks + (shuffle ? 4 * kMaskWords : 2) * (uint64_t)g.nblocks,
                                  L.stream + 4 * words, L.opos + 4 * nout, L.oval + 4 * nout, L.ppos + 4 * npat,
                                  L.pbits + 4 * npat};
        const uint64_t starts[8] = {L.coef, L.chunks, L.stream, L.opos, L.oval, L.ppos, L.pbits, L.total};
        for (int k = shuffle ? 2 : 0; k < 8; k++)
            for (uint64_t a = ends[k]; a < starts[k]; a++) out[a] = 0;
        // header
        double eb_abs;
        resolve_eb(mode, eb, misc->mm_lo, misc->mm_hi, &eb_abs);
        uint8_t h[kHdr];
        for (int k = 0; k < kHdr; k++) h[k] = 0;
        auto st32 = [&](int o, uint32_t v) { for (int k = 0; k < 4; k++) h[o + k] = (uint8_t)(v >> (8 * k)); };
        auto st64 = [&](int o, uint64_t v) { for (int k = 0; k < 8; k++) h[o + k] = (uint8_t)(v >> (8 * k)); };
        st32(0, kMagic);
        h[4] = (uint8_t)kVersion;
        h[5] = (uint8_t)(kVersion >> 8);
        h[6] = shuffle ? (uint8_t)kFlagShuffle : 0;
        st32(8, g.ndim);
        st32(12, pred);
        st64(16, g.n[0]);
        st64(24, g.n[1]);
        st64(32, g.n[2]);
        st32(40, mode);
        st32(44, kRadius);
        st64(48, __double_as_longlong(eb));
        st64(56, __double_as_longlong(eb_abs));
        st64(64, L.total);
        st32(72, g.nblocks);
        st32(76, (uint32_t)nout);
        st32(80, (uint32_t)npat);
        st32(84, (uint32_t)words);
        st64(88, bits);
        st32(96, (uint32_t)nreg);
        uint4* dst = reinterpret_cast<uint4*>(out);
        const uint4* src = reinterpret_cast<const uint4*>(h);
        for (int k = 0; k < kHdr / 16; k++) dst[k] = src[k];
    }
}

// ------------------------------------------------------------ launchers
void launch_codebook(hipStream_t st, uint32_t* hist, uint8_t* out_lens, uint32_t* cw, Misc* misc) {
    hipLaunchKernelGGL(k_codebook, dim3(1), dim3(1024), 0, st, hist, out_lens, cw, misc);
}

void launch_encode(hipStream_t st, int grid, const uint16_t* codes, const Geom& g, const uint32_t* cw, Misc* misc,
                   uint32_t ntiles, uint8_t* out, uint64_t* desc, uint64_t* tile_start, uint32_t* tfirst,
                   uint32_t* tlast) {
    (void)grid;  // one workgroup per group of tiles
    const uint32_t groups = (ntiles + kEncTiles - 1) / kEncTiles;
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_encode<3>, dim3(groups), dim3(256), 0, st, codes, g, cw, ntiles, misc, out, desc,
                           tile_start, tfirst, tlast);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_encode<2>, dim3(groups), dim3(256), 0, st, codes, g, cw, ntiles, misc, out, desc,
                           tile_start, tfirst, tlast);
    else
        hipLaunchKernelGGL(k_encode<1>, dim3(groups), dim3(256), 0, st, codes, g, cw, ntiles, misc, out, desc,
                           tile_start, tfirst, tlast);
}

uint32_t encode_groups(uint32_t ntiles) { return (ntiles + kEncTiles - 1) / kEncTiles; }

void launch_finalize(hipStream_t st, const Geom& g, uint32_t mode, double eb, uint32_t pred, Misc* misc,
                     uint8_t* out, uint32_t ntiles, const uint64_t* tile_start, const uint32_t* tfirst,
                     const uint32_t* tlast, const uint32_t* tile_cnt, const uint64_t* tile_off, const uint2* ostage,
                     const uint2* pstage, const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coef,
                     const float* x, uint32_t codec) {
    // about four tiles per wave for the outlier/patch compaction
    uint32_t grid = (ntiles + 15) / 16;
    if (grid < 1024) grid = 1024;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, st, g, mode, eb, pred, misc, out, ntiles, tile_start,
                       tfirst, tlast, tile_cnt, tile_off, ostage, pstage, bpred, reg_idx, coef, x,
                       (int)(((uintptr_t)x & 15) == 0), codec);
}

}  // namespace fz
