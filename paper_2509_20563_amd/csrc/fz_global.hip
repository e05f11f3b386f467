// Decoding of the global (non-blocked) first-order Lorenzo predictor
// (Sec. 3.1's Lorenzo predictor with neighbours anywhere in the field).  The
// Huffman decoders leave every residual in the block-major residual field;
// the inverse is a prefix sum along each axis over the whole field, done
// here one axis per launch on that field, in place, each thread carrying
// the running sum of one line across the blocks:
//   3D  k_gl_y3 - line along y: lane = (lx, lz), 8 values per block
//       k_gl_z3 - line along z: lane = (lx, ly), 8 values per block
//       k_gl_x3_store - line along x: lane = (ly, lz) of a block row, two
//                 16-byte loads per block, dequantised values staged in
//                 LDS and stored as whole 256-byte pieces of the lines
//   2D  k_gl_x2 - line along x: lane = ly, 32 values per block
//       k_gl_y2 - line along y: lane = lx, dequantised stores
//   1D  k_gl_scan1 - one prefix sum over the field: tiles of 2048 values
//                 taken in order from a counter, tile sums chained by
//                 decoupled look-back, dequantised stores
// Values past the field's edge in edge blocks sit at the end of every line
// they are on, so whatever they hold reaches no value inside the field.
// Sums are modulo 2^32 (unsigned arithmetic).
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

__device__ __forceinline__ uint4 scan4(uint4 a, uint32_t& carry) {
    a.x += carry;
    a.y += a.x;
    a.z += a.y;
    a.w += a.z;
    carry = a.w;
    return a;
}

__global__ __launch_bounds__(256) void k_gl_y3(Geom g, uint32_t* __restrict__ R) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= 64u * g.nb[0] * g.nb[2]) return;
    const uint32_t seg = gid & 63u, bc = gid >> 6;
    const uint32_t lx = seg & 7u, lz = seg >> 3;
    const uint32_t bx = bc % g.nb[0], bz = bc / g.nb[0];
    uint32_t carry = 0;
    for (uint32_t by = 0; by < g.nb[1]; by++) {
        const uint64_t b = bx + (uint64_t)g.nb[0] * (by + (uint64_t)g.nb[1] * bz);
        uint32_t* p = R + b * kBlockElems + lx + 64u * lz;
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = p[8 * k];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            carry += v[k];
            p[8 * k] = carry;
        }
    }
}

__global__ __launch_bounds__(256) void k_gl_z3(Geom g, uint32_t* __restrict__ R) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= 64u * g.nb[0] * g.nb[1]) return;
    const uint32_t seg = gid & 63u, bc = gid >> 6;  // seg = lx + 8 ly
    uint32_t carry = 0;
    const uint64_t plane = (uint64_t)g.nb[0] * g.nb[1];
    uint32_t* p = R + (uint64_t)bc * kBlockElems + seg;
    for (uint32_t bz = 0; bz < g.nb[2]; bz++, p += plane * kBlockElems) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = p[64 * k];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            carry += v[k];
            p[64 * k] = carry;
        }
    }
}

// 3D, last pass: lines along x with dequantisation.  Wave = one block row
// (lane = (ly, lz)); every 8 blocks along x a lane has 64 values of its
// line, staged in LDS (64 lines x 64 values per wave) and stored as whole
// 256-byte line pieces: each store instruction writes four lines' pieces.
__global__ __launch_bounds__(256) void k_gl_x3_store(Geom g, const uint32_t* __restrict__ R, double e2,
                                                     float* __restrict__ out, int vec) {
    __shared__ float S[4][64 * 65];  // per wave, line l at l * 65 (padding against bank conflicts)
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t br = blockIdx.x * 4 + wave;  // block row: by + nb1 * bz
    const bool act = br < g.nb[1] * g.nb[2];
    const uint32_t by = act ? br % g.nb[1] : 0, bz = act ? br / g.nb[1] : 0;
    float* Sw = S[wave];
    uint32_t carry = 0;
    const uint4* p = reinterpret_cast<const uint4*>(R + (uint64_t)g.nb[0] * br * kBlockElems + lane * 8);
    for (uint32_t bx0 = 0; bx0 < g.nb[0]; bx0 += 8) {
        const uint32_t nbk = min(8u, g.nb[0] - bx0);
        if (act) {
            for (uint32_t j = 0; j < nbk; j++) {
                const uint4 a = p[0], c = p[1];
                p += kBlockElems / 4;
                const uint32_t q[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    carry += q[i];
                    Sw[lane * 65 + 8 * j + i] = (float)((double)(int32_t)carry * e2);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // store: 16 rounds, four lines per round (lane = line 4 r + lane / 16,
        // float4 index lane % 16 of the 64 values)
        if (act) {
            const uint32_t x0 = bx0 * 8;
            for (uint32_t r = 0; r < 16; r++) {
                const uint32_t l = 4 * r + lane / 16, f = lane % 16;  // line (ly + 8 lz), float4 in it
                const uint32_t y = by * 8 + (l & 7), z = bz * 8 + (l >> 3);
                const uint32_t x = x0 + 4 * f;
                if (y >= g.n[1] || z >= g.n[2] || x >= g.n[0]) continue;
                const float* src = &Sw[l * 65 + 4 * f];
                const uint64_t o = x + (uint64_t)g.n[0] * (y + (uint64_t)g.n[1] * z);
                if (vec && x + 4 <= g.n[0]) {
                    const f32x4 w = {src[0], src[1], src[2], src[3]};
                    __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(out + o));
                } else {
                    for (uint32_t m = 0; m < 4 && x + m < g.n[0]; m++) out[o + m] = src[m];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__global__ __launch_bounds__(256) void k_gl_x2(Geom g, uint32_t* __restrict__ R) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= 16u * g.nb[1]) return;
    const uint32_t ly = gid & 15u, by = gid >> 4;
    uint32_t carry = 0;
    for (uint32_t bx = 0; bx < g.nb[0]; bx++) {
        const uint64_t b = bx + (uint64_t)g.nb[0] * by;
        uint4* p = reinterpret_cast<uint4*>(R + b * kBlockElems + 32u * ly);
        uint4 v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = p[k];
#pragma unroll
        for (int k = 0; k < 8; k++) p[k] = scan4(v[k], carry);
    }
}

__global__ __launch_bounds__(256) void k_gl_y2(Geom g, const uint32_t* __restrict__ R, double e2,
                                               float* __restrict__ out) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= 32u * g.nb[0]) return;
    const uint32_t lx = gid & 31u, bx = gid >> 5;
    const uint32_t x = bx * 32 + lx;
    const bool in = x < g.n[0];
    uint32_t carry = 0;
    for (uint32_t by = 0; by < g.nb[1]; by++) {
        const uint32_t* p = R + (bx + (uint64_t)g.nb[0] * by) * kBlockElems + lx;
        uint32_t v[16];
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = p[32 * k];
#pragma unroll
        for (int k = 0; k < 16; k++) {
            carry += v[k];
            const uint32_t y = by * 16 + (uint32_t)k;
            if (in && y < g.n[1])
                __builtin_nontemporal_store((float)((double)(int32_t)carry * e2), out + x + (uint64_t)g.n[0] * y);
        }
    }
}

constexpr uint32_t kScan1 = 2048;  // values per tile of the 1D scan

__global__ __launch_bounds__(256) void k_gl_scan1(uint64_t N, const uint32_t* __restrict__ R, uint32_t ntiles,
                                                  uint64_t* desc, Misc* misc, double e2, float* __restrict__ out) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t s_excl;
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) s_tile = atomicAdd(&misc->mtile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;  // uniform: the grid is exactly ntiles
    const uint64_t i0 = (uint64_t)tile * kScan1 + 8ull * t;
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = i0 + k < N ? R[i0 + k] : 0u;
#pragma unroll
    for (int k = 1; k < 8; k++) v[k] += v[k - 1];
    const uint32_t incl = (uint32_t)wave_incl_scan(v[7]);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < 4; w++) {
        wpre += w < wave ? wsum[w] : 0u;
        total += wsum[w];
    }
    if (wave == 0) {
        const uint64_t ex = lookback(desc, tile, (uint64_t)total, OpAdd(), &misc->flags);
        if (lane == 0) s_excl = ex;
    }
    __syncthreads();
    const uint32_t base = (uint32_t)s_excl + wpre + incl - v[7];
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (i0 + k < N) __builtin_nontemporal_store((float)((double)(int32_t)(base + v[k]) * e2), out + i0 + k);
}

uint32_t global_scan_tiles(uint64_t N) { return (uint32_t)((N + kScan1 - 1) / kScan1); }

void launch_global_inverse(hipStream_t st, const Geom& g, int32_t* res, uint64_t* desc, Misc* misc, double e2,
                           float* out, int vec) {
    uint32_t* R = reinterpret_cast<uint32_t*>(res);
    auto grid = [](uint64_t threads) { return dim3((uint32_t)((threads + 255) / 256)); };
    if (g.ndim == 3) {
        // y and z in place, then x (the output's contiguous axis) with the
        // dequantised, staged row stores
        hipLaunchKernelGGL(k_gl_y3, grid(64ull * g.nb[0] * g.nb[2]), dim3(256), 0, st, g, R);
        hipLaunchKernelGGL(k_gl_z3, grid(64ull * g.nb[0] * g.nb[1]), dim3(256), 0, st, g, R);
        hipLaunchKernelGGL(k_gl_x3_store, dim3((g.nb[1] * g.nb[2] + 3) / 4), dim3(256), 0, st, g, R, e2, out, vec);
    } else if (g.ndim == 2) {
        hipLaunchKernelGGL(k_gl_x2, grid(16ull * g.nb[1]), dim3(256), 0, st, g, R);
        hipLaunchKernelGGL(k_gl_y2, grid(32ull * g.nb[0]), dim3(256), 0, st, g, R, e2, out);
    } else {
        const uint32_t nt = global_scan_tiles(g.N);
        launch_fill32(st, reinterpret_cast<uint32_t*>(desc), 2ull * nt, 0u);
        hipLaunchKernelGGL(k_gl_scan1, dim3(nt), dim3(256), 0, st, g.N, R, nt, desc, misc, e2, out);
    }
}

}  // namespace fz
