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
__global__ void k_reset(Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2, uint32_t n2) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (gid == 0) {
        Misc m = {};
        m.mm_lo = 0xFFFFFFFFu;
        m.mm_hi = 0u;
        *misc = m;
    }
    for (uint32_t i = gid; i < (uint32_t)kBins; i += stride) hist[i] = 0;
    for (uint32_t i = gid; i < n1; i += stride) d1[i] = 0;
    for (uint32_t i = gid; i < n2; i += stride) d2[i] = 0;
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

// ------------------------------------------------ prequantisation helper
// q = rint(x / 2eb) via x * (1 / 2eb) in double, round half to even.
// Patch when |t| >= 2^24 (q = 0) or when float(q * 2eb) misses the bound.
__device__ __forceinline__ int32_t prequant1(float xv, double e2, double inv, double eb_abs, bool& patch) {
    const double xd = (double)xv;
    const double t = xd * inv;
    const bool big = fabs(t) >= 16777216.0;
    const double r = __builtin_rint(big ? 0.0 : t);  // branch-free: q = 0 when out of range
    const float xh = (float)(r * e2);
    patch = big || (fabs(xd - (double)xh) > eb_abs);
    return (int32_t)r;
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

template <int ND>
__global__ __launch_bounds__(256) void k_quant(const float* __restrict__ x, Geom g, uint32_t mode, double eb,
                                               int vec, Misc* misc, uint32_t* __restrict__ hist_g,
                                               uint16_t* __restrict__ codes, uint32_t ntiles,
                                               uint32_t* __restrict__ tile_cnt, uint32_t* __restrict__ opos,
                                               int32_t* __restrict__ oval, uint32_t* __restrict__ ppos,
                                               uint32_t* __restrict__ pbits) {
    // q per block, regions padded by 8 words so the load-mapped writes of
    // four blocks do not fall into the same banks; one extra zero row
    constexpr int kQStride = kBlockElems + 8;
    constexpr uint32_t kZero = kTileBlocks * kQStride;
    __shared__ int32_t Q[kTileBlocks * kQStride + 8];
    __shared__ uint8_t PM[kTileBlocks * kSegs];
    __shared__ uint32_t H[kBins];
    __shared__ uint32_t wsum[4];

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
    for (uint32_t i = t; i < (uint32_t)kBins; i += 256) H[i] = 0;
    if (t < 8) Q[kZero + t] = 0;

    // load-phase lane constants (the same for every tile): block in tile,
    // segment, segment coordinates and the segment's row-major offset from
    // its block origin (indices fit in 32 bits: N <= 2^32)
    uint32_t la_bi, la_s, la_lx0, la_ly, la_lz;
    load_map<ND>(t, la_bi, la_s);
    seg_coords<ND>(la_s, la_lx0, la_ly, la_lz);
    const uint32_t la_rowoff = la_lx0 + g.n[0] * (la_ly + g.n[1] * la_lz);
    // phase-B lane (segment = lane) offset, for reloading patched values
    uint32_t lb_lx0, lb_ly, lb_lz;
    seg_coords<ND>(lane, lb_lx0, lb_ly, lb_lz);
    const uint32_t lb_rowoff = lb_lx0 + g.n[0] * (lb_ly + g.n[1] * lb_lz);

    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // ---------------- phase A: load + prequantise
        {
            // the tile's four block origins and extents are wave-uniform
            // (scalar); each lane picks its block's entry
            uint32_t org[kTileBlocks], ex[kTileBlocks], ey[kTileBlocks], ez[kTileBlocks];
#pragma unroll
            for (int k = 0; k < kTileBlocks; k++) {
                const uint32_t bk = tile * kTileBlocks + k;
                const bool ok = bk < g.nblocks;
                const BlockInfo ik = block_info(g, ok ? bk : 0);
                org[k] = ik.bx * g.bs[0] + g.n[0] * (ik.by * g.bs[1] + g.n[1] * (ik.bz * g.bs[2]));
                ex[k] = ok ? ik.ex : 0u;
                ey[k] = ik.ey;
                ez[k] = ik.ez;
            }
            auto pick = [&](const uint32_t* a) {
                return la_bi == 0 ? a[0] : la_bi == 1 ? a[1] : la_bi == 2 ? a[2] : a[3];
            };
            const uint32_t bex = pick(ex), bey = pick(ey), bez = pick(ez);
            const uint32_t nv = (la_ly < bey && la_lz < bez && la_lx0 < bex) ? min(8u, bex - la_lx0) : 0u;
            const uint32_t base = pick(org) + la_rowoff;
            int32_t q[8];
            uint32_t pm = 0;
            bool bad = false;
            float v[8];
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
#pragma unroll
            for (int i = 0; i < 8; i++) {
                bool p;
                const int32_t qi = prequant1(v[i], e2, inv, eb_abs, p);
                const bool valid = i < (int)nv;
                bad |= valid && !__builtin_isfinite(v[i]);
                q[i] = valid ? qi : 0;
                pm |= (valid && p ? 1u : 0u) << i;
            }
            if (bad) atomicOr(&misc->flags, F_NONFINITE);
            int4* dst = reinterpret_cast<int4*>(&Q[la_bi * kQStride + la_s * 8]);
            dst[0] = make_int4(q[0], q[1], q[2], q[3]);
            dst[1] = make_int4(q[4], q[5], q[6], q[7]);
            PM[la_bi * kSegs + la_s] = (uint8_t)pm;
        }
        __syncthreads();

        // ---------------- phase B: wave = block, lane = segment
        const uint32_t s = lane;
        const uint32_t b = tile * kTileBlocks + wave;  // wave-uniform
        const bool blk = b < g.nblocks;
        const uint32_t Qb = wave * kQStride;
        uint32_t nv = 0;  // real values in this segment
        int32_t d[8];
        {
            const BlockInfo info = block_info(g, blk ? b : 0);
            int32_t r0[8], A[8];
            int32_t am1 = 0;  // A[-1]: the left neighbour term along x
            read_row<ND>(Q, Qb + s * 8, r0);
            if (ND == 3) {
                const uint32_t ly = s & 7, lz = s >> 3;
                nv = (blk && ly < info.ey && lz < info.ez) ? info.ex : 0u;
                int32_t ry[8], rz[8], ryz[8];
                read_row<ND>(Q, ly ? Qb + (s - 1) * 8 : kZero, ry);
                read_row<ND>(Q, lz ? Qb + (s - 8) * 8 : kZero, rz);
                read_row<ND>(Q, (ly && lz) ? Qb + (s - 9) * 8 : kZero, ryz);
#pragma unroll
                for (int i = 0; i < 8; i++) A[i] = (r0[i] - ry[i]) - (rz[i] - ryz[i]);
            } else if (ND == 2) {
                const uint32_t sx = s & 3, ly = s >> 2;
                nv = (blk && ly < info.ey && 8 * sx < info.ex) ? min(8u, info.ex - 8 * sx) : 0u;
                int32_t up[8];
                read_row<ND>(Q, ly ? Qb + (s - 4) * 8 : kZero, up);
                const int32_t left = Q[sx ? Qb + (s - 1) * 8 + 7 : kZero];
                const int32_t upleft = Q[(sx && ly) ? Qb + (s - 5) * 8 + 7 : kZero];
                am1 = left - upleft;
#pragma unroll
                for (int i = 0; i < 8; i++) A[i] = r0[i] - up[i];
            } else {
                nv = (blk && 8 * s < info.ex) ? min(8u, info.ex - 8 * s) : 0u;
                am1 = Q[s ? Qb + (s - 1) * 8 + 7 : kZero];
#pragma unroll
                for (int i = 0; i < 8; i++) A[i] = r0[i];
            }
#pragma unroll
            for (int i = 7; i >= 0; i--) d[i] = A[i] - (i ? A[i - 1] : am1);
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
        if (blk) {
            uint4 pk;
            pk.x = code[0] | (code[1] << 16);
            pk.y = code[2] | (code[3] << 16);
            pk.z = code[4] | (code[5] << 16);
            pk.w = code[6] | (code[7] << 16);
            *reinterpret_cast<uint4*>(&codes[(uint64_t)b * kBlockElems + s * 8]) = pk;
        }
        // histogram: lane 0's code is added once for every lane sharing it,
        // the other lanes add their own
        if (blk) {
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint32_t c = (i < (int)nv) ? code[i] : 0xFFFFu;
                const uint32_t cand = (uint32_t)__builtin_amdgcn_readfirstlane((int)c);
                const uint64_t m = __ballot(c == cand);
                if (lane == 0 && cand != 0xFFFFu) atomicAdd(&H[cand], (uint32_t)__popcll(m));
                if (c != cand && c != 0xFFFFu) atomicAdd(&H[c], 1u);
            }
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
            uint64_t oi = slot + (excl_local & 0xFFFFu);
            uint64_t pi = slot + (excl_local >> 16);
            const uint32_t pos0 = b * kBlockElems + s * 8;
            const BlockInfo ib = block_info(g, b);
            const uint32_t base = ib.bx * g.bs[0] + g.n[0] * (ib.by * g.bs[1] + g.n[1] * (ib.bz * g.bs[2])) +
                                  lb_rowoff;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                if (omask & (1u << i)) {
                    opos[oi] = pos0 + i;
                    oval[oi] = d[i];
                    oi++;
                }
                if (pm_lane & (1u << i)) {
                    ppos[pi] = pos0 + i;
                    pbits[pi] = __float_as_uint(x[base + i]);
                    pi++;
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (uint32_t i = t; i < (uint32_t)kBins; i += 256)
        if (H[i]) atomicAdd(&hist_g[i], H[i]);
}

// ------------------------------------------------------------ launchers
void launch_reset(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2,
                  uint32_t n2) {
    uint32_t n = n1 > n2 ? n1 : n2;
    uint32_t grid = (n + 255) / 256;
    if (grid < 4) grid = 4;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, st, misc, hist, d1, n1, d2, n2);
}

void launch_minmax(hipStream_t st, const float* x, uint64_t N, int vec, Misc* misc, int grid) {
    hipLaunchKernelGGL(k_minmax, dim3(grid), dim3(256), 0, st, x, N, vec, misc);
}

void launch_quant(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                  Misc* misc, uint32_t* hist, uint16_t* codes, uint32_t ntiles, uint32_t* tile_cnt, uint32_t* opos,
                  int32_t* oval, uint32_t* ppos, uint32_t* pbits) {
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_quant<3>, dim3(grid), dim3(256), 0, st, x, g, mode, eb, vec, misc, hist, codes, ntiles,
                           tile_cnt, opos, oval, ppos, pbits);
    else if (g.ndim == 2)
        hipLaunchKernelGGL(k_quant<2>, dim3(grid), dim3(256), 0, st, x, g, mode, eb, vec, misc, hist, codes, ntiles,
                           tile_cnt, opos, oval, ppos, pbits);
    else
        hipLaunchKernelGGL(k_quant<1>, dim3(grid), dim3(256), 0, st, x, g, mode, eb, vec, misc, hist, codes, ntiles,
                           tile_cnt, opos, oval, ppos, pbits);
}

}  // namespace fz
