// Decoding of the interpolation predictor (FZMod-Quality pipeline, Sec. 3.3:
// the G-Interp interpolator in place of Lorenzo).  The Huffman decoders
// leave the residuals of every value in the row-major residual field;
// these kernels turn them into grid values in place, in the order the
// prediction needs (fz_common.h, interp_predict), one launch per stride and
// axis:
//   k_interp_anchor  - prefix sums along one axis of the anchor grid (every
//                      coordinate a multiple of 8), one thread per line
//   k_interp_level_z, k_interp_level_yx - strides 4 and 2 (2D/3D): the
//                      stride-1 passes below on the lattice of that stride,
//                      in place
//   k_interp_level   - strides 4 and 2 of a 1D field, one thread per point
//   k_interp_final_yx - stride 1 (2D/3D): the z pass of the odd planes
//                      (3D), the y pass and the x pass of a group of rows
//                      together, the even points exchanged in LDS for the
//                      odd points' x prediction, the pair dequantised to
//                      the output
//   k_interp_z       - stride 1, z pass of fields one row high: a thread per
//                      pair of points (2m, 2m + 1) of an even row through a
//                      group of 8 planes, so that stores cover whole lines
//   k_interp_final_x - stride 1, x pass alone (1D, and fields one row
//                      high)
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// Position of (x, y, z) in the row-major residual and grid-value fields.
template <int ND>
__device__ __forceinline__ uint64_t rm_index(const Geom& g, uint32_t x, uint32_t y, uint32_t z) {
    return (uint64_t)x + (uint64_t)g.n[0] * ((uint64_t)y + (uint64_t)g.n[1] * z);
}

// Number of coordinates c < n with c = first + step k.
__device__ __forceinline__ uint32_t n_coords(uint32_t n, uint32_t first, uint32_t step) {
    return n > first ? (n - first + step - 1) / step : 0u;
}

// Loads of one anchor line issued together (the line is read and written
// in place, so a load cannot move above an earlier store by itself)
constexpr int kAnchorBatch = 16;

template <int ND>
__global__ __launch_bounds__(64) void k_interp_anchor(Geom g, const int32_t* src, int32_t* dst, int axis) {
    // lines: the anchor coordinates of the other axes
    uint32_t cnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) cnt[a] = n_coords(g.n[a], 0, 8);
    uint32_t lc[3] = {cnt[0], cnt[1], cnt[2]};
    lc[axis] = 1;
    const uint64_t nlines = (uint64_t)lc[0] * lc[1] * lc[2];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t sa = 8 * (axis == 0 ? 1ull : (axis == 1 ? (uint64_t)g.n[0] : (uint64_t)g.n[0] * g.n[1]));
    const uint32_t len = cnt[axis];
    for (uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlines; l += stride) {
        uint32_t c[3] = {(uint32_t)(l % lc[0]) * 8, (uint32_t)((l / lc[0]) % lc[1]) * 8,
                         (uint32_t)(l / ((uint64_t)lc[0] * lc[1])) * 8};
        c[axis] = 0;
        const uint64_t i0 = rm_index<ND>(g, c[0], c[1], c[2]);
        int32_t acc = 0;
        for (uint32_t k0 = 0; k0 < len; k0 += kAnchorBatch) {
            int32_t v[kAnchorBatch];
#pragma unroll
            for (int j = 0; j < kAnchorBatch; j++) v[j] = k0 + j < len ? src[i0 + sa * (k0 + j)] : 0;
#pragma unroll
            for (int j = 0; j < kAnchorBatch; j++) {
                acc = (int32_t)((uint32_t)acc + (uint32_t)v[j]);
                if (k0 + j < len) dst[i0 + sa * (k0 + j)] = acc;
            }
        }
    }
}

// Prediction of a point at coordinate c along its axis (field extent n,
// stride s) from the neighbours at -3s, -s, +s, +3s (those outside the
// field are not used).
__device__ __forceinline__ int32_t pick_pred(uint32_t c, uint32_t n, uint32_t s, int32_t m3, int32_t m1, int32_t p1,
                                             int32_t p3) {
    if (c >= 3 * s && c + 3 * s < n) return (int32_t)((-(int64_t)m3 + 9 * (int64_t)m1 + 9 * (int64_t)p1 - (int64_t)p3 + 8) >> 4);
    if (c + s < n) return (int32_t)(((int64_t)m1 + (int64_t)p1 + 1) >> 1);
    return m1;
}

// The points of one stride s and axis AXIS (an odd multiple of s on that
// axis, even multiples (of 2s) on the axes before it in x, y, z order, any
// multiple of s on the axes after it), in place on the row-major grid
// values: thread = one point, blockIdx.x along x, rows of (y, z) over
// blockIdx.y; every neighbour along AXIS is a point rebuilt before.
template <int AXIS>
__global__ __launch_bounds__(256) void k_interp_level(Geom g, int32_t* __restrict__ q, uint32_t s, uint32_t f0,
                                                      uint32_t s0, uint32_t c0, uint32_t f1, uint32_t s1, uint32_t c1,
                                                      uint32_t f2, uint32_t s2, uint32_t nrows) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= c0) return;
    const uint32_t x = f0 + s0 * i;
    const uint64_t sa = AXIS == 0 ? 1ull : (AXIS == 1 ? (uint64_t)g.n[0] : (uint64_t)g.n[0] * g.n[1]);
    for (uint32_t r = blockIdx.y; r < nrows; r += gridDim.y) {
        const uint32_t j = r % c1, k = r / c1;
        const uint32_t y = f1 + s1 * j, z = f2 + s2 * k;
        const uint64_t idx = (uint64_t)x + (uint64_t)g.n[0] * ((uint64_t)y + (uint64_t)g.n[1] * z);
        const uint32_t ca = AXIS == 0 ? x : (AXIS == 1 ? y : z), na = g.n[AXIS];
        const uint64_t d1 = (uint64_t)s * sa, d3 = 3 * d1;
        const int32_t m1 = q[idx - d1];
        const int32_t p1 = ca + s < na ? q[idx + d1] : 0;
        const int32_t m3 = ca >= 3 * s ? q[idx - d3] : 0;
        const int32_t p3 = ca + 3 * s < na ? q[idx + d3] : 0;
        q[idx] = (int32_t)((uint32_t)q[idx] + (uint32_t)pick_pred(ca, na, s, m3, m1, p1, p3));
    }
}

// rows (planes) per workgroup group of the stride-1 passes
constexpr int kYXRows = 8;

// Stride 1, the z pass (3D): the points (x even, y even, z odd).  A
// thread takes the pair (2m, 2m + 1) of one even row y through a group of
// kYXRows planes (z0 = kYXRows j): it loads the even planes z0 - 2 ..
// z0 + 10 once (final grid values) and rewrites the pairs of the group's
// odd planes, the even point predicted along z, the odd one unchanged (so
// the stores cover whole lines), in place.
__global__ __launch_bounds__(256) void k_interp_z(Geom g, int32_t* __restrict__ q, uint32_t ngroups, uint32_t gpr) {
    const uint32_t n0 = g.n[0], n2 = g.n[2];
    const uint32_t x = 2 * (blockIdx.x * 256 + threadIdx.x);
    if (x >= n0) return;
    const bool two = x + 1 < n0;
    const bool v2 = two && (n0 & 1) == 0;
    const uint64_t sz = (uint64_t)n0 * g.n[1];
    for (uint32_t u = blockIdx.y; u < ngroups; u += gridDim.y) {
        const uint32_t zg = u / gpr, y = 2 * (u - zg * gpr), z0 = zg * kYXRows;
        const uint64_t rb = (uint64_t)n0 * y + x;  // (x, y) in plane 0
        // even points of planes z0 - 3 .. z0 + 10 (the even ones)
        int32_t ev[kYXRows + 6];
#pragma unroll
        for (int j = 0; j < kYXRows + 6; j += 2) {
            const int zz = (int)z0 - 3 + j + 1;  // even plane z0 - 2 + j
            ev[j] = 0;
            ev[j + 1] = (zz >= 0 && (uint32_t)zz < n2) ? q[rb + sz * (uint32_t)zz] : 0;
        }
#pragma unroll
        for (int k = 1; k < kYXRows; k += 2) {
            const uint32_t z = z0 + k;
            if (z >= n2) break;  // uniform
            const uint64_t i = rb + sz * z;
            const int32_t pr = pick_pred(z, n2, 1, z >= 3 ? ev[k] : 0, ev[k + 2], z + 1 < n2 ? ev[k + 4] : 0,
                                         z + 3 < n2 ? ev[k + 6] : 0);
            if (v2) {
                int2 v = *reinterpret_cast<const int2*>(q + i);
                v.x = (int32_t)((uint32_t)v.x + (uint32_t)pr);
                *reinterpret_cast<int2*>(q + i) = v;
            } else {
                q[i] = (int32_t)((uint32_t)q[i] + (uint32_t)pr);
            }
        }
    }
}

// Strides 4 and 2 on the lattice of stride s (coordinates s X, s Y, s Z,
// extents N = ceil(n / s)): there a level's z, y and x passes are the
// stride-1 passes (the edge rules of stride s at s X are those of stride 1
// at X), in place on the row-major grid values.
//
// The z pass (3D): the points (X even, Y even, Z odd).  A thread takes one
// even X of an even row Y through a group of kYXRows planes Z (Z0 =
// kYXRows j), loads the even planes Z0 - 2 .. Z0 + 10 once and updates the
// group's odd planes.
__global__ __launch_bounds__(256) void k_interp_level_z(Geom g, int32_t* __restrict__ q, uint32_t s, uint32_t N0,
                                                        uint32_t N2, uint32_t ngroups, uint32_t gpr) {
    const uint32_t X = 2 * (blockIdx.x * 256 + threadIdx.x);
    if (X >= N0) return;
    const uint64_t sz = (uint64_t)g.n[0] * g.n[1] * s;  // one lattice plane
    for (uint32_t u = blockIdx.y; u < ngroups; u += gridDim.y) {
        const uint32_t zg = u / gpr, Y = 2 * (u - zg * gpr), Z0 = zg * kYXRows;
        const uint64_t rb = (uint64_t)g.n[0] * s * Y + (uint64_t)s * X;  // (X, Y) in plane 0
        // planes Z0 - 3 .. Z0 + 10 (the even ones loaded)
        int32_t ev[kYXRows + 6];
#pragma unroll
        for (int j = 0; j < kYXRows + 6; j += 2) {
            const int zz = (int)Z0 - 2 + j;
            ev[j] = 0;
            ev[j + 1] = (zz >= 0 && (uint32_t)zz < N2) ? q[rb + sz * (uint32_t)zz] : 0;
        }
#pragma unroll
        for (int k = 1; k < kYXRows; k += 2) {
            const uint32_t Z = Z0 + k;
            if (Z >= N2) break;  // uniform
            const uint64_t i = rb + sz * Z;
            const int32_t pr = pick_pred(Z, N2, 1, Z >= 3 ? ev[k] : 0, ev[k + 2], Z + 1 < N2 ? ev[k + 4] : 0,
                                         Z + 3 < N2 ? ev[k + 6] : 0);
            q[i] = (int32_t)((uint32_t)q[i] + (uint32_t)pr);
        }
    }
}

// The y and x passes together (2D/3D, after the z pass): the points (X
// even, Y odd) predicted along y, then (X odd, any Y) along x.  Workgroup =
// kYXRows consecutive lattice rows of one lattice plane (Y0 = kYXRows j),
// the whole row length in chunks of 256 pairs (X = 2m, 2m + 1), so that no
// other workgroup writes the points this one reads: the even points of odd
// rows to the right of a chunk, rebuilt by lanes 1 and 2 from their
// residuals, are only overwritten by the same workgroup's next chunk, and
// those left of it are carried from the previous chunk by lane 255.  Per
// chunk a thread loads its pair of every row once and the even points of
// rows Y0 - 2, Y0 + 8, Y0 + 10 (never written here), so an odd row's y
// prediction reads registers; the even points then go through LDS to the
// odd points' x prediction.  Stores cover the points this pass rebuilds.
__global__ __launch_bounds__(256) void k_interp_level_yx(Geom g, int32_t* __restrict__ q, uint32_t s, uint32_t N0,
                                                         uint32_t N1, uint32_t ngroups, uint32_t gpp) {
    __shared__ int32_t E[kYXRows][256 + 3];  // even points of the pairs m0 - 1 .. m0 + 257, per row
    const uint32_t t = threadIdx.x;
    const uint64_t sy = (uint64_t)g.n[0] * s;         // one lattice row
    const uint64_t sp = (uint64_t)g.n[0] * g.n[1] * s;  // one lattice plane
    const uint32_t nch = (N0 + 511) / 512;
    for (uint32_t u = blockIdx.x; u < ngroups; u += gridDim.x) {
        const uint32_t Z = u / gpp, Y0 = (u - Z * gpp) * kYXRows;
        const uint64_t pb = sp * Z;
        // even point of lattice row YY at X: final (YY even) or rebuilt from
        // the rows YY -/+ 1, 3 (YY odd)
        auto even_at = [&](uint32_t XX, uint32_t YY) -> int32_t {
            const uint64_t i = pb + sy * YY + (uint64_t)s * XX;
            uint32_t v = (uint32_t)q[i];
            if (YY & 1) {
                const int32_t m1 = q[i - sy];
                const int32_t p1 = YY + 1 < N1 ? q[i + sy] : 0;
                const int32_t m3 = YY >= 3 ? q[i - 3 * sy] : 0;
                const int32_t p3 = YY + 3 < N1 ? q[i + 3 * sy] : 0;
                v += (uint32_t)pick_pred(YY, N1, 1, m3, m1, p1, p3);
            }
            return (int32_t)v;
        };
        int32_t prev[kYXRows];  // lane 255: the even points of the previous chunk
#pragma unroll
        for (int k = 0; k < kYXRows; k++) prev[k] = 0;
        for (uint32_t c = 0; c < nch; c++) {
            const uint32_t m0 = 256 * c;
            const uint32_t X = 2 * (m0 + t);
            const bool in = X < N0;
            const bool two = X + 1 < N0;
            const uint64_t xb = (uint64_t)s * X;
            const bool halo = t == 1 || t == 2;
            const uint32_t hX = 2 * (m0 + 255 + t);
            const bool hin = halo && hX < N0;
            int32_t ev[kYXRows + 6];  // even points of rows Y0 - 3 .. Y0 + 10 (odd rows outside unused)
            int32_t od[kYXRows];
#pragma unroll
            for (int k = 0; k < kYXRows + 6; k++) ev[k] = 0;
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                od[k] = 0;
                const uint32_t YY = Y0 + k;
                if (in && YY < N1) {
                    const uint64_t i = pb + sy * YY + xb;
                    ev[k + 3] = q[i];
                    if (two) od[k] = q[i + s];
                }
            }
            if (in) {
                if (Y0 >= 2) ev[1] = q[pb + sy * (Y0 - 2) + xb];
                if (Y0 + 8 < N1) ev[kYXRows + 3] = q[pb + sy * (Y0 + 8) + xb];
                if (Y0 + 10 < N1) ev[kYXRows + 5] = q[pb + sy * (Y0 + 10) + xb];
            }
            int32_t e[kYXRows];
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                const uint32_t YY = Y0 + k;
                e[k] = ev[k + 3];
                if (k & 1) {
                    const int32_t pr = pick_pred(YY, N1, 1, YY >= 3 ? ev[k] : 0, ev[k + 2],
                                                 YY + 1 < N1 ? ev[k + 4] : 0, YY + 3 < N1 ? ev[k + 6] : 0);
                    e[k] = (int32_t)((uint32_t)e[k] + (uint32_t)pr);
                }
                E[k][1 + t] = in ? e[k] : 0;
                if (t == 255) E[k][0] = prev[k];
                if (halo) E[k][256 + t] = (hin && YY < N1) ? even_at(hX, YY) : 0;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                const uint32_t YY = Y0 + k;
                prev[k] = e[k];
                if (YY >= N1) break;  // uniform
                int32_t o = od[k];
                if (two) {
                    const uint32_t ca = X + 1;
                    const int32_t p1 = ca + 1 < N0 ? E[k][t + 2] : 0;
                    const int32_t m3 = ca >= 3 ? E[k][t] : 0;
                    const int32_t p3 = ca + 3 < N0 ? E[k][t + 3] : 0;
                    o = (int32_t)((uint32_t)o + (uint32_t)pick_pred(ca, N0, 1, m3, e[k], p1, p3));
                }
                if (in) {
                    const uint64_t i = pb + sy * YY + xb;
                    if (k & 1) q[i] = e[k];
                    if (two) q[i + s] = o;
                }
            }
            __syncthreads();
        }
    }
}

// the x pass alone (the odd point of each pair) with dequantisation: the pair
// (even point final before this pass, odd point rebuilt here) goes to the
// output as two floats, so this pass writes the whole field
__global__ __launch_bounds__(256) void k_interp_final_x(Geom g, const int32_t* __restrict__ q, double e2,
                                                        float* __restrict__ out, uint32_t nrows) {
    const uint32_t m = blockIdx.x * 256 + threadIdx.x;
    const uint32_t x = 2 * m;
    if (x >= g.n[0]) return;
    const uint32_t n0 = g.n[0];
    const bool two = x + 1 < n0;
    const bool v2 = two && (n0 & 1) == 0;
    auto dq = [&](int32_t v) { return (float)((double)v * e2); };
    for (uint32_t r = blockIdx.y; r < nrows; r += gridDim.y) {
        const uint64_t idx = (uint64_t)x + (uint64_t)n0 * r;
        int32_t e0, o = 0;
        if (v2) {
            const int2 v = *reinterpret_cast<const int2*>(q + idx);
            e0 = v.x;
            o = v.y;
        } else {
            e0 = q[idx];
            if (two) o = q[idx + 1];
        }
        if (two) {
            const uint32_t ca = x + 1;
            const int32_t p1 = ca + 1 < n0 ? q[idx + 2] : 0;
            const int32_t m3 = ca >= 3 ? q[idx - 2] : 0;
            const int32_t p3 = ca + 3 < n0 ? q[idx + 4] : 0;
            o = (int32_t)((uint32_t)o + (uint32_t)pick_pred(ca, n0, 1, m3, e0, p1, p3));
        }
        if (v2) {
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            const f32x2 w = {dq(e0), dq(o)};
            __builtin_nontemporal_store(w, reinterpret_cast<f32x2*>(out + idx));
        } else {
            out[idx] = dq(e0);
            if (two) out[idx + 1] = dq(o);
        }
    }
}

// Stride 1, the y and x passes together (2D/3D) and, with ZF (3D), the
// z pass of the odd planes folded in: workgroup = kYXRows consecutive rows
// of one plane (y0 = kYXRows j) over their whole length, in chunks of 256
// pairs (x = 2m, 2m + 1).  Per chunk a thread loads its pair of every row
// once and the even points of the rows y0 - 2, y0 + 8 and y0 + 10; in an
// odd plane an even row's even point first takes its z prediction from the
// planes z -/+ 1, 3 (even planes, whose even rows' even points are final:
// this pass writes only the output), then an odd row's y prediction reads
// registers.  The even points go through an LDS ring of three chunks
// (slot = pair mod 768): chunk c + 1 is built before chunk c's odd points
// take their x prediction, so the pairs right of a chunk are there and
// those left of it still are.  Each pair is written dequantised.
template <bool ZF>
__global__ __launch_bounds__(256) void k_interp_final_yx(Geom g, const int32_t* __restrict__ q, double e2,
                                                         float* __restrict__ out, uint32_t ngroups, uint32_t gpp) {
    constexpr uint32_t kRing = 768;
    __shared__ int32_t S[kYXRows][kRing];
    const uint32_t t = threadIdx.x;
    const uint32_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const uint32_t nch = ((n0 + 1) / 2 + 255) / 256;
    const bool even_n0 = (n0 & 1) == 0;
    const uint64_t sy = n0, sz = (uint64_t)n0 * n1;
    auto dq = [&](int32_t v) { return (float)((double)v * e2); };
    for (uint32_t u = blockIdx.x; u < ngroups; u += gridDim.x) {
        const uint32_t z = u / gpp, y0 = (u - z * gpp) * kYXRows;
        const uint64_t pb = sz * z;  // the plane
        const bool zodd = ZF && (z & 1u);
        // z prediction at index i of this (odd) plane from the planes
        // z -/+ 1, 3
        auto zpred = [&](uint64_t i) -> uint32_t {
            const int32_t m1 = q[i - sz];
            const int32_t p1 = z + 1 < n2 ? q[i + sz] : 0;
            const int32_t m3 = z >= 3 ? q[i - 3 * sz] : 0;
            const int32_t p3 = z + 3 < n2 ? q[i + 3 * sz] : 0;
            return (uint32_t)pick_pred(z, n2, 1, m3, m1, p1, p3);
        };
        // chunk c of the group: this thread's even points after the z and
        // y passes (e, also into the ring) and odd residuals (od)
        auto build = [&](uint32_t c, int32_t* e, int32_t* od) {
            const uint32_t x = 2 * (256 * c + t);
            const bool in = x < n0;
            const bool two = x + 1 < n0;
            const bool v2 = two && even_n0;
            int32_t ev[kYXRows + 6];  // even points of rows y0 - 3 .. y0 + 10 (odd rows outside unused)
#pragma unroll
            for (int k = 0; k < kYXRows + 6; k++) ev[k] = 0;
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                od[k] = 0;
                const uint32_t yy = y0 + k;
                if (in && yy < n1) {
                    const uint64_t i = pb + sy * yy + x;
                    if (v2) {
                        const int2 v = *reinterpret_cast<const int2*>(q + i);
                        ev[k + 3] = v.x;
                        od[k] = v.y;
                    } else {
                        ev[k + 3] = q[i];
                        if (two) od[k] = q[i + 1];
                    }
                    if (zodd && !(k & 1)) ev[k + 3] = (int32_t)((uint32_t)ev[k + 3] + zpred(i));
                }
            }
            if (in) {
                auto halo_row = [&](uint32_t yy) -> int32_t {
                    const uint64_t i = pb + sy * yy + x;
                    uint32_t v = (uint32_t)q[i];
                    if (zodd) v += zpred(i);
                    return (int32_t)v;
                };
                if (y0 >= 2) ev[1] = halo_row(y0 - 2);
                if (y0 + 8 < n1) ev[kYXRows + 3] = halo_row(y0 + 8);
                if (y0 + 10 < n1) ev[kYXRows + 5] = halo_row(y0 + 10);
            }
            const uint32_t sl = (256 * c + t) % kRing;
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                const uint32_t yy = y0 + k;
                e[k] = ev[k + 3];
                if (k & 1) {
                    const int32_t pr = pick_pred(yy, n1, 1, yy >= 3 ? ev[k] : 0, ev[k + 2],
                                                 yy + 1 < n1 ? ev[k + 4] : 0, yy + 3 < n1 ? ev[k + 6] : 0);
                    e[k] = (int32_t)((uint32_t)e[k] + (uint32_t)pr);
                }
                S[k][sl] = in ? e[k] : 0;
            }
        };
        int32_t e0[kYXRows], o0[kYXRows], e1[kYXRows], o1[kYXRows];
        build(0, e0, o0);
        for (uint32_t c = 0; c < nch; c++) {
            if (c + 1 < nch) build(c + 1, e1, o1);  // uniform
            __syncthreads();
            // the x pass of chunk c: odd point of pair P from the even
            // points of pairs P - 1, P (registers), P + 1, P + 2
            const uint32_t P = 256 * c + t;
            const uint32_t x = 2 * P;
            const bool in = x < n0;
            const bool two = x + 1 < n0;
            const bool v2 = two && even_n0;
            const uint32_t sl = P % kRing;
            const uint32_t sm1 = sl == 0 ? kRing - 1 : sl - 1;
            const uint32_t sp1 = sl + 1 == kRing ? 0 : sl + 1;
            const uint32_t sp2 = sp1 + 1 == kRing ? 0 : sp1 + 1;
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                const uint32_t yy = y0 + k;
                if (yy >= n1) break;  // uniform
                int32_t o = o0[k];
                if (two) {
                    const uint32_t ca = x + 1;
                    const int32_t p1 = ca + 1 < n0 ? S[k][sp1] : 0;
                    const int32_t m3 = ca >= 3 ? S[k][sm1] : 0;
                    const int32_t p3 = ca + 3 < n0 ? S[k][sp2] : 0;
                    o = (int32_t)((uint32_t)o + (uint32_t)pick_pred(ca, n0, 1, m3, e0[k], p1, p3));
                }
                const uint64_t i = pb + sy * yy + x;
                if (v2) {
                    typedef float f32x2 __attribute__((ext_vector_type(2)));
                    const f32x2 w = {dq(e0[k]), dq(o)};
                    __builtin_nontemporal_store(w, reinterpret_cast<f32x2*>(out + i));
                } else if (in) {
                    out[i] = dq(e0[k]);
                    if (two) out[i + 1] = dq(o);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kYXRows; k++) {
                e0[k] = e1[k];
                o0[k] = o1[k];
            }
        }
    }
}

template <int ND>
static void interp_anchors(hipStream_t st, const Geom& g, const int32_t* src, int32_t* dst) {
    uint32_t acnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) acnt[a] = (g.n[a] + 7) / 8;
    for (int a = 0; a < ND; a++) {
        uint64_t lines = (uint64_t)acnt[0] * acnt[1] * acnt[2] / acnt[a];
        uint64_t gr = (lines + 63) / 64;
        if (gr > 32768) gr = 32768;
        hipLaunchKernelGGL(k_interp_anchor<ND>, dim3((uint32_t)gr), dim3(64), 0, st, g, a ? dst : src, dst, a);
    }
}

// 1D and 2D: one pass per stride and axis, in place on the residuals
template <int ND>
static void interp_inverse_passes(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out) {
    interp_anchors<ND>(st, g, q, q);
    auto cap = [](uint64_t r) { return (uint32_t)(r < 65535 ? r : 65535); };
    for (uint32_t s = 4; s >= 2; s >>= 1) {
        if (ND >= 2) {
            // the stride-1 passes on the lattice of stride s
            const uint32_t N0 = (g.n[0] + s - 1) / s, N1 = (g.n[1] + s - 1) / s;
            const uint32_t N2 = ND == 3 ? (g.n[2] + s - 1) / s : 1u;
            if (ND == 3 && N2 > 1) {
                const uint32_t gpr = (N1 + 1) / 2;
                const uint64_t ngroups = (uint64_t)gpr * ((N2 + kYXRows - 1) / kYXRows);
                const uint32_t nev = (N0 + 1) / 2;
                hipLaunchKernelGGL(k_interp_level_z, dim3((nev + 255) / 256, cap(ngroups)), dim3(256), 0, st, g, q, s,
                                   N0, N2, (uint32_t)ngroups, gpr);
            }
            const uint32_t gpp = (N1 + kYXRows - 1) / kYXRows;
            const uint64_t ngroups = (uint64_t)gpp * N2;
            const uint32_t grid = (uint32_t)(ngroups < (1u << 20) ? ngroups : (1u << 20));
            hipLaunchKernelGGL(k_interp_level_yx, dim3(grid), dim3(256), 0, st, g, q, s, N0, N1, (uint32_t)ngroups,
                               gpp);
            continue;
        }
        // 1D: the points of stride s along x, one thread per point
        const uint32_t c0 = g.n[0] > s ? (g.n[0] - s + 2 * s - 1) / (2 * s) : 0u;
        if (!c0) continue;
        hipLaunchKernelGGL(k_interp_level<0>, dim3((c0 + 255) / 256, 1), dim3(256), 0, st, g, q, s, s, 2 * s, c0, 0u,
                           1u, 1u, 0u, 1u, 1u);
    }
    // stride 1: the y and x passes together, with the z pass of the odd
    // planes folded in (3D), writing the output; fields one row high: the z
    // pass (pairs of points through groups of planes), then the x pass
    const uint32_t npairs = (g.n[0] + 1) / 2;
    if (ND >= 2 && g.n[1] > 1) {
        const uint32_t gpp = (g.n[1] + kYXRows - 1) / kYXRows;
        const uint64_t ngroups = (uint64_t)gpp * g.n[2];
        const uint32_t grid = (uint32_t)(ngroups < (1u << 20) ? ngroups : (1u << 20));
        if (ND == 3 && g.n[2] > 1)
            hipLaunchKernelGGL(k_interp_final_yx<true>, dim3(grid), dim3(256), 0, st, g, q, e2, out,
                               (uint32_t)ngroups, gpp);
        else
            hipLaunchKernelGGL(k_interp_final_yx<false>, dim3(grid), dim3(256), 0, st, g, q, e2, out,
                               (uint32_t)ngroups, gpp);
        return;
    }
    if (ND == 3 && g.n[2] > 1) {
        // even rows y through groups of kYXRows planes
        const uint32_t gpr = (g.n[1] + 1) / 2;
        const uint64_t ngroups = (uint64_t)gpr * ((g.n[2] + kYXRows - 1) / kYXRows);
        hipLaunchKernelGGL(k_interp_z, dim3((npairs + 255) / 256, cap(ngroups)), dim3(256), 0, st, g, q,
                           (uint32_t)ngroups, gpr);
    }
    const uint64_t rows = (uint64_t)g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_interp_final_x, dim3((npairs + 255) / 256, cap(rows)), dim3(256), 0, st, g, q, e2, out,
                       (uint32_t)rows);
}

void launch_interp_inverse(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out) {
    if (g.ndim == 3) interp_inverse_passes<3>(st, g, q, e2, out);
    else if (g.ndim == 2) interp_inverse_passes<2>(st, g, q, e2, out);
    else interp_inverse_passes<1>(st, g, q, e2, out);
}

}  // namespace fz
