// Decoding of the global (non-blocked) first-order Lorenzo predictor
// (Sec. 3.1's Lorenzo predictor with neighbours anywhere in the field).  The
// Huffman decoders leave every residual in the row-major residual field;
// the inverse is a prefix sum along each axis over the whole field.  Large
// 3D fields (rows of at most 4096 values, enough planes):
//   k_gl_xy    - lines along x and y together, workgroup = plane, in place
//   k_gl_z_out - lines along z, dequantised stores
// otherwise one axis per launch, in place:
//   k_gl_y  - lines along y (2D/3D): thread = (x, z), carrying the sum
//   k_gl_z  - lines along z (3D): thread = (x, y)
//   k_gl_x  - lines along x, last: one wave per row, 256 values per step by
//             in-lane and cross-lane prefix sums, dequantised row stores
//   1D  k_gl_scan1 - one prefix sum over the field: tiles of 2048 values
//             taken in order from a counter, tile sums chained by decoupled
//             look-back, dequantised stores
// Sums are modulo 2^32 (unsigned arithmetic).
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// Line along y (2D/3D): thread = (x, z), consecutive threads on
// consecutive x, so every step reads and writes one contiguous run.
__global__ __launch_bounds__(256) void k_gl_y(Geom g, uint32_t* __restrict__ R) {
    const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (uint64_t)g.n[0] * g.n[2]) return;
    const uint64_t x = gid % g.n[0], z = gid / g.n[0];
    uint32_t* p = R + x + (uint64_t)g.n[0] * g.n[1] * z;
    const uint64_t st = g.n[0];
    uint32_t carry = 0;
    uint32_t y = 0;
    for (; y + 4 <= g.n[1]; y += 4) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = p[k * st];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            carry += v[k];
            p[k * st] = carry;
        }
        p += 4 * st;
    }
    for (; y < g.n[1]; y++, p += st) {
        carry += *p;
        *p = carry;
    }
}

// Line along z (3D): thread = (x, y).
__global__ __launch_bounds__(256) void k_gl_z(Geom g, uint32_t* __restrict__ R) {
    const uint64_t plane = (uint64_t)g.n[0] * g.n[1];
    const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= plane) return;
    uint32_t* p = R + gid;
    uint32_t carry = 0;
    uint32_t z = 0;
    for (; z + 4 <= g.n[2]; z += 4) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = p[k * plane];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            carry += v[k];
            p[k * plane] = carry;
        }
        p += 4 * plane;
    }
    for (; z < g.n[2]; z++, p += plane) {
        carry += *p;
        *p = carry;
    }
}

// Line along x (last pass, 2D/3D) with dequantisation: one wave per row,
// 256 values per step (4 per lane: a 16-byte load and store where the rows
// are aligned), in-lane and cross-lane prefix sums plus the row's carry.
__global__ __launch_bounds__(256) void k_gl_x(Geom g, const uint32_t* __restrict__ R, double e2,
                                              float* __restrict__ out, int vec) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (uint64_t)g.n[1] * g.n[2]) return;  // uniform per wave
    const uint64_t base = row * g.n[0];
    const uint32_t* src = R + base;
    float* dst = out + base;
    auto dq = [&](uint32_t q) { return (float)((double)(int32_t)q * e2); };
    uint32_t carry = 0;
    for (uint32_t x0 = 0; x0 < g.n[0]; x0 += 256) {
        const uint32_t x = x0 + 4 * lane;
        uint32_t v[4] = {0, 0, 0, 0};
        const bool full = vec && x + 4 <= g.n[0];
        if (full) {
            const uint4 a = *reinterpret_cast<const uint4*>(src + x);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (x + k < g.n[0]) v[k] = src[x + k];
        }
        v[1] += v[0];
        v[2] += v[1];
        v[3] += v[2];
        const uint32_t incl = (uint32_t)wave_incl_scan(v[3]);
        const uint32_t pre = carry + incl - v[3];
        carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (full) {
            const f32x4 w = {dq(pre + v[0]), dq(pre + v[1]), dq(pre + v[2]), dq(pre + v[3])};
            __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(dst + x));
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (x + k < g.n[0]) dst[x + k] = dq(pre + v[k]);
        }
    }
}

// Lines along x and y together (3D, rows of at most 4096 values):
// workgroup = one plane z, wave w = the x range [256 C w, 256 C (w + 1)) of
// every row; the waves walk the rows in order with the running sums along
// y in registers (the next D - 1 rows' loads in flight), and per row take
// the prefix along x of their range plus the row totals of the waves to
// their left (LDS, two slots alternating by row, one barrier per row).  In
// place; the z pass follows and writes the output.
template <int C>
__global__ __launch_bounds__(256) void k_gl_xy(Geom g, uint32_t* __restrict__ R, int vec) {
    constexpr int D = 4;  // rows in flight per wave (8 measured the same)
    __shared__ uint32_t tot[2][4];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
    const uint32_t n0 = g.n[0], n1 = g.n[1];
    uint32_t* P = R + (uint64_t)n0 * n1 * blockIdx.x;
    const uint32_t xb = 256u * C * w + 4 * lane;  // chunk c starts at xb + 256 c
    const bool v4 = vec && (n0 & 3) == 0;
    auto load = [&](uint32_t y, uint32_t (&v)[C][4]) {
        const uint32_t* row = P + (uint64_t)n0 * y;
#pragma unroll
        for (int c = 0; c < C; c++) {
            const uint32_t x = xb + 256u * c;
            if (v4 && x + 4 <= n0) {
                const uint4 a = *reinterpret_cast<const uint4*>(row + x);
                v[c][0] = a.x; v[c][1] = a.y; v[c][2] = a.z; v[c][3] = a.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) v[c][k] = x + k < n0 ? row[x + k] : 0u;
            }
        }
    };
    uint32_t cy[C][4];  // sums along y of the rows so far
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
        for (int k = 0; k < 4; k++) cy[c][k] = 0;
    uint32_t buf[D][C][4];
#pragma unroll
    for (int d = 0; d < D; d++)
        if ((uint32_t)d < n1) load(d, buf[d]);
    for (uint32_t y0 = 0; y0 < n1; y0 += D) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            const uint32_t y = y0 + d;  // uniform over the workgroup
            if (y >= n1) break;
            uint32_t a[C][4];
#pragma unroll
            for (int c = 0; c < C; c++)
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    cy[c][k] += buf[d][c][k];
                    a[c][k] = cy[c][k];
                }
            if (y + D < n1) load(y + D, buf[d]);
            uint32_t carry = 0;
#pragma unroll
            for (int c = 0; c < C; c++) {
                a[c][1] += a[c][0];
                a[c][2] += a[c][1];
                a[c][3] += a[c][2];
                const uint32_t incl = wave_incl_scan(a[c][3]);
                const uint32_t pre = carry + incl - a[c][3];
#pragma unroll
                for (int k = 0; k < 4; k++) a[c][k] += pre;
                carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            }
            if (lane == 0) tot[y & 1][w] = carry;
            __syncthreads();
            uint32_t left = 0;
            for (uint32_t u = 0; u < W; u++) left += u < w ? tot[y & 1][u] : 0u;
            uint32_t* row = P + (uint64_t)n0 * y;
#pragma unroll
            for (int c = 0; c < C; c++) {
                const uint32_t x = xb + 256u * c;
                if (v4 && x + 4 <= n0) {
                    *reinterpret_cast<uint4*>(row + x) =
                        make_uint4(a[c][0] + left, a[c][1] + left, a[c][2] + left, a[c][3] + left);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; k++)
                        if (x + k < n0) row[x + k] = a[c][k] + left;
                }
            }
        }
    }
}

// Line along z with dequantisation (3D, after k_gl_xy): thread = 4
// consecutive x of one (x, y) row segment, walking z.
__global__ __launch_bounds__(256) void k_gl_z_out(Geom g, const uint32_t* __restrict__ R, double e2,
                                                  float* __restrict__ out, int vec) {
    const uint64_t plane = (uint64_t)g.n[0] * g.n[1];
    const uint64_t i0 = 4 * ((uint64_t)blockIdx.x * 256 + threadIdx.x);
    if (i0 >= plane) return;
    auto dq = [&](uint32_t q) { return (float)((double)(int32_t)q * e2); };
    const bool v4 = vec && (plane & 3) == 0;  // then i0 + 4 <= plane
    uint32_t c[4] = {0, 0, 0, 0};
    for (uint32_t z = 0; z < g.n[2]; z++) {
        const uint64_t i = i0 + plane * z;
        if (v4) {
            const uint4 a = *reinterpret_cast<const uint4*>(R + i);
            c[0] += a.x; c[1] += a.y; c[2] += a.z; c[3] += a.w;
            const f32x4 o = {dq(c[0]), dq(c[1]), dq(c[2]), dq(c[3])};
            __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(out + i));
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (i0 + k < plane) {
                    c[k] += R[i + k];
                    out[i + k] = dq(c[k]);
                }
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

// The fused x/y pass walks each plane's rows in order, one workgroup per
// plane: it needs at least this many waves to keep HBM busy (1024^3: 4096
// waves, 4.9 -> 3.4 ms for the inverse; 512^3 has 1024 waves and runs the
// separate passes, 0.56 ms against 0.64 fused)
constexpr uint64_t kGlFusedWaves = 2048;

void launch_global_inverse(hipStream_t st, const Geom& g, int32_t* res, uint64_t* desc, Misc* misc, double e2,
                           float* out, int vec) {
    uint32_t* R = reinterpret_cast<uint32_t*>(res);
    auto grid = [](uint64_t threads) { return dim3((uint32_t)((threads + 255) / 256)); };
    const uint32_t C = g.n[0] <= 1024 ? 1u : (g.n[0] <= 2048 ? 2u : 4u);  // chunks of 256 per wave and row
    const uint32_t W = (g.n[0] + 256 * C - 1) / (256 * C);                 // waves per plane
    if (g.ndim == 3 && g.n[0] <= 4096 && (uint64_t)g.n[2] * W >= kGlFusedWaves) {
        // x and y together in place, then z with the dequantised stores
        if (C == 1) hipLaunchKernelGGL(k_gl_xy<1>, dim3(g.n[2]), dim3(64 * W), 0, st, g, R, vec);
        else if (C == 2) hipLaunchKernelGGL(k_gl_xy<2>, dim3(g.n[2]), dim3(64 * W), 0, st, g, R, vec);
        else hipLaunchKernelGGL(k_gl_xy<4>, dim3(g.n[2]), dim3(64 * W), 0, st, g, R, vec);
        const uint64_t plane = (uint64_t)g.n[0] * g.n[1];
        hipLaunchKernelGGL(k_gl_z_out, grid((plane + 3) / 4), dim3(256), 0, st, g, R, e2, out, vec);
    } else if (g.ndim >= 2) {
        // y (and z) in place, then x, the output's contiguous axis, with the
        // dequantised stores
        hipLaunchKernelGGL(k_gl_y, grid((uint64_t)g.n[0] * g.n[2]), dim3(256), 0, st, g, R);
        if (g.ndim == 3) hipLaunchKernelGGL(k_gl_z, grid((uint64_t)g.n[0] * g.n[1]), dim3(256), 0, st, g, R);
        const int xvec = vec && (g.n[0] & 3) == 0;
        hipLaunchKernelGGL(k_gl_x, grid(64ull * g.n[1] * g.n[2]), dim3(256), 0, st, g, R, e2, out, xvec);
    } else {
        const uint32_t nt = global_scan_tiles(g.N);
        launch_fill32(st, reinterpret_cast<uint32_t*>(desc), 2ull * nt, 0u);
        hipLaunchKernelGGL(k_gl_scan1, dim3(nt), dim3(256), 0, st, g.N, R, nt, desc, misc, e2, out);
    }
}

}  // namespace fz
