// Decoding of the interpolation predictor (FZMod-Quality pipeline, Sec. 3.3:
// the G-Interp interpolator in place of Lorenzo).  The Huffman decoders
// leave the residuals of every value in the row-major residual field;
// these kernels turn them into grid values in place, in the order the
// prediction needs (fz_common.h, interp_predict):
//   k_interp_anchor - prefix sums along one axis of the anchor grid (every
//                     coordinate a multiple of 8), one thread per line
//   k_interp_tile3  - 3D: one level (stride 4, 2 or 1) per launch, tiles of
//                     8^3 lattice points in LDS with the coarser values and
//                     the z- and y-pass points of a halo of 2 lattice steps
//   k_interp_level  - 1D/2D: the points of one stride and axis, one thread
//                     per point, in place
//   k_interp_store  - 1D/2D: dequantisation
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

template <int ND>
__global__ __launch_bounds__(256) void k_interp_anchor(Geom g, const int32_t* src, int32_t* dst, int axis) {
    // lines: the anchor coordinates of the other axes
    uint32_t cnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) cnt[a] = n_coords(g.n[a], 0, 8);
    uint32_t lc[3] = {cnt[0], cnt[1], cnt[2]};
    lc[axis] = 1;
    const uint64_t nlines = (uint64_t)lc[0] * lc[1] * lc[2];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlines; l += stride) {
        uint32_t c[3] = {(uint32_t)(l % lc[0]) * 8, (uint32_t)((l / lc[0]) % lc[1]) * 8,
                         (uint32_t)(l / ((uint64_t)lc[0] * lc[1])) * 8};
        int32_t acc = 0;
        for (uint32_t k = 0; k < cnt[axis]; k++) {
            c[axis] = 8 * k;
            const uint64_t i = rm_index<ND>(g, c[0], c[1], c[2]);
            acc = (int32_t)((uint32_t)acc + (uint32_t)src[i]);
            dst[i] = acc;
        }
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_interp_level(Geom g, int32_t* __restrict__ q, uint32_t s, int axis) {
    // points interpolated along `axis` at stride s: an odd multiple of s on
    // that axis, even multiples (of 2s) on the axes before it in x, y, z
    // order, any multiple of s on the axes after it
    uint32_t first[3] = {0, 0, 0}, step[3] = {1, 1, 1}, cnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) {
        first[a] = a == axis ? s : 0u;
        step[a] = a <= axis ? 2 * s : s;
        cnt[a] = n_coords(g.n[a], first[a], step[a]);
    }
    const uint64_t npts = (uint64_t)cnt[0] * cnt[1] * cnt[2];
    const uint32_t n3[3] = {g.n[0], g.n[1], g.n[2]};
    auto q_at = [&](uint32_t x, uint32_t y, uint32_t z) -> int32_t { return q[rm_index<ND>(g, x, y, z)]; };
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += stride) {
        const uint32_t c[3] = {first[0] + step[0] * (uint32_t)(p % cnt[0]),
                               first[1] + step[1] * (uint32_t)((p / cnt[0]) % cnt[1]),
                               first[2] + step[2] * (uint32_t)(p / ((uint64_t)cnt[0] * cnt[1]))};
        const int32_t pred = interp_predict(c, n3, ND, q_at);
        const uint64_t i = rm_index<ND>(g, c[0], c[1], c[2]);
        q[i] = (int32_t)((uint32_t)q[i] + (uint32_t)pred);
    }
}

// 3D: one level of stride S on tiles of 8x8x8 lattice points (spacing S,
// the box [X0, X0 + 8S) per axis), one workgroup per tile.  The level's
// points are those with an odd lattice coordinate; lattice points with all
// coordinates even are the coarser levels (final in V).  In LDS:
//   C  coarse values at even lattice coordinates -2..10 on every axis
//   Z  the z-pass points (i, j even in -2..10, k odd in 1..7), rebuilt here
//      also where they lie outside the tile (the y and x passes read them)
//   Y  the y-pass points (i even in -2..10, j odd in 1..7, k in 0..7)
// then the x-pass points of the tile.  Residuals come from R (read-only
// here, so rebuilding a neighbour tile's points races with nothing); the
// tile's own points go to V (S > 1) or, at S = 1, every value of the tile
// (one 8^3 block) is dequantised into row-major floats.
__device__ __forceinline__ int32_t pick_pred(uint32_t c, uint32_t n, uint32_t s, int32_t m3, int32_t m1, int32_t p1,
                                             int32_t p3) {
    if (c >= 3 * s && c + 3 * s < n) return (int32_t)((-(int64_t)m3 + 9 * (int64_t)m1 + 9 * (int64_t)p1 - (int64_t)p3 + 8) >> 4);
    if (c + s < n) return (int32_t)(((int64_t)m1 + (int64_t)p1 + 1) >> 1);
    return m1;
}

template <uint32_t S>
__global__ __launch_bounds__(256) void k_interp_tile3(Geom g, const int32_t* __restrict__ R, int32_t* __restrict__ V,
                                                      double e2, float* __restrict__ out, uint32_t ntx, uint32_t nty,
                                                      uint32_t ntiles, int vec) {
    __shared__ int32_t C[343];
    __shared__ int32_t Z[196];
    __shared__ int32_t Y[224];
    __shared__ int32_t T[S == 1 ? 512 : 1];
    const uint32_t t = threadIdx.x;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t tx = tile % ntx, r1 = tile / ntx, ty = r1 % nty, tz = r1 / nty;
        const int32_t X0 = (int32_t)(tx * 8 * S), Y0 = (int32_t)(ty * 8 * S), Z0 = (int32_t)(tz * 8 * S);
        auto inside = [&](int32_t x, int32_t y, int32_t z) {
            return x >= 0 && y >= 0 && z >= 0 && (uint32_t)x < g.n[0] && (uint32_t)y < g.n[1] && (uint32_t)z < g.n[2];
        };
        // coarse values
        for (uint32_t e = t; e < 343; e += 256) {
            const int32_t i = 2 * (int32_t)(e % 7) - 2, j = 2 * (int32_t)((e / 7) % 7) - 2, k = 2 * (int32_t)(e / 49) - 2;
            const int32_t x = X0 + (int32_t)S * i, y = Y0 + (int32_t)S * j, z = Z0 + (int32_t)S * k;
            C[e] = inside(x, y, z) ? V[rm_index<3>(g, x, y, z)] : 0;
        }
        __syncthreads();
        // z pass
        if (t < 196) {
            const uint32_t e = t;
            const int32_t i = 2 * (int32_t)(e % 7) - 2, j = 2 * (int32_t)((e / 7) % 7) - 2, k = 2 * (int32_t)(e / 49) + 1;
            const int32_t x = X0 + (int32_t)S * i, y = Y0 + (int32_t)S * j, z = Z0 + (int32_t)S * k;
            int32_t v = 0;
            if (inside(x, y, z)) {
                // planes k - 3, k - 1, k + 1, k + 3 are C planes ko .. ko + 3
                const uint32_t cc = e % 49, ko = e / 49;
                const int32_t m3 = C[ko * 49 + cc], m1 = C[(ko + 1) * 49 + cc], p1 = C[(ko + 2) * 49 + cc],
                              p3 = C[(ko + 3) * 49 + cc];
                v = (int32_t)((uint32_t)R[rm_index<3>(g, x, y, z)] +
                              (uint32_t)pick_pred((uint32_t)z, g.n[2], S, m3, m1, p1, p3));
            }
            Z[e] = v;
        }
        __syncthreads();
        // y pass
        if (t < 224) {
            const uint32_t e = t;
            const int32_t i = 2 * (int32_t)(e % 7) - 2, jo = (int32_t)((e / 7) % 4), k = (int32_t)(e / 28);
            const int32_t j = 2 * jo + 1;
            const int32_t x = X0 + (int32_t)S * i, y = Y0 + (int32_t)S * j, z = Z0 + (int32_t)S * k;
            int32_t v = 0;
            if (inside(x, y, z)) {
                const uint32_t ii = e % 7;
                // rows j - 3, j - 1, j + 1, j + 3 are even rows jo .. jo + 3
                // (numbered from -2)
                int32_t nb[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint32_t jj = (uint32_t)jo + (uint32_t)q;
                    nb[q] = (k & 1) ? Z[((uint32_t)(k - 1) / 2) * 49 + jj * 7 + ii] : C[((uint32_t)(k + 2) / 2) * 49 + jj * 7 + ii];
                }
                v = (int32_t)((uint32_t)R[rm_index<3>(g, x, y, z)] +
                              (uint32_t)pick_pred((uint32_t)y, g.n[1], S, nb[0], nb[1], nb[2], nb[3]));
            }
            Y[e] = v;
        }
        __syncthreads();
        // x pass: the tile's own points (i odd)
        {
            const uint32_t io = t % 4, j = (t / 4) % 8, k = t / 32;
            const int32_t i = 2 * (int32_t)io + 1;
            const int32_t x = X0 + (int32_t)S * i, y = Y0 + (int32_t)S * (int32_t)j, z = Z0 + (int32_t)S * (int32_t)k;
            if (inside(x, y, z)) {
                int32_t nb[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint32_t ii = io + (uint32_t)q;  // i - 3 + 2 q in the -2..10 numbering
                    if (j & 1) nb[q] = Y[k * 28 + ((j - 1) / 2) * 7 + ii];
                    else if (k & 1) nb[q] = Z[((k - 1) / 2) * 49 + ((j + 2) / 2) * 7 + ii];
                    else nb[q] = C[((k + 2) / 2) * 49 + ((j + 2) / 2) * 7 + ii];
                }
                const int32_t v = (int32_t)((uint32_t)R[rm_index<3>(g, x, y, z)] +
                                            (uint32_t)pick_pred((uint32_t)x, g.n[0], S, nb[0], nb[1], nb[2], nb[3]));
                if (S == 1) T[i + 8 * (j + 8 * k)] = v;
                else V[rm_index<3>(g, x, y, z)] = v;
            }
        }
        if (S == 1) {
            // the tile's coarse, z- and y-pass values into T
            if (t < 64) {
                const uint32_t i = 2 * (t % 4), j = 2 * ((t / 4) % 4), k = 2 * (t / 16);
                T[i + 8 * (j + 8 * k)] = C[((k + 2) / 2) * 49 + ((j + 2) / 2) * 7 + (i + 2) / 2];
            } else if (t < 128) {
                const uint32_t e = t - 64;
                const uint32_t i = 2 * (e % 4), j = 2 * ((e / 4) % 4), k = 2 * (e / 16) + 1;
                T[i + 8 * (j + 8 * k)] = Z[((k - 1) / 2) * 49 + ((j + 2) / 2) * 7 + (i + 2) / 2];
            } else {
                const uint32_t e = t - 128;  // 128 y-pass points of the tile
                const uint32_t i = 2 * (e % 4), j = 2 * ((e / 4) % 4) + 1, k = e / 16;
                T[i + 8 * (j + 8 * k)] = Y[k * 28 + ((j - 1) / 2) * 7 + (i + 2) / 2];
            }
            __syncthreads();
            // rows of 8 floats: thread = half row
            if (t < 128) {
                const uint32_t row = t / 2, h = t % 2;
                const uint32_t y = (uint32_t)Y0 + row % 8, z = (uint32_t)Z0 + row / 8;
                const uint32_t x = (uint32_t)X0 + 4 * h;
                if (y < g.n[1] && z < g.n[2] && x < g.n[0]) {
                    const int32_t* src = &T[4 * h + 8 * row];
                    const uint64_t o = (uint64_t)x + (uint64_t)g.n[0] * ((uint64_t)y + (uint64_t)g.n[1] * z);
                    auto dq = [&](int32_t q) { return (float)((double)q * e2); };
                    if (vec && x + 4 <= g.n[0]) {
                        const f32x4 w = {dq(src[0]), dq(src[1]), dq(src[2]), dq(src[3])};
                        __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(out + o));
                    } else {
                        for (uint32_t m = 0; m < 4 && x + m < g.n[0]; m++) out[o + m] = dq(src[m]);
                    }
                }
            }
        } else {
            // the tile's own z- and y-pass points to V
            if (t < 64) {
                const uint32_t i = 2 * (t % 4), j = 2 * ((t / 4) % 4), k = 2 * (t / 16) + 1;
                const int32_t x = X0 + (int32_t)(S * i), y = Y0 + (int32_t)(S * j), z = Z0 + (int32_t)(S * k);
                if (inside(x, y, z)) V[rm_index<3>(g, x, y, z)] = Z[((k - 1) / 2) * 49 + ((j + 2) / 2) * 7 + (i + 2) / 2];
            } else if (t < 192) {
                const uint32_t e = t - 64;
                const uint32_t i = 2 * (e % 4), j = 2 * ((e / 4) % 4) + 1, k = e / 16;
                const int32_t x = X0 + (int32_t)(S * i), y = Y0 + (int32_t)(S * j), z = Z0 + (int32_t)(S * k);
                if (inside(x, y, z)) V[rm_index<3>(g, x, y, z)] = Y[k * 28 + ((j - 1) / 2) * 7 + (i + 2) / 2];
            }
        }
        __syncthreads();
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_interp_store(Geom g, const int32_t* __restrict__ q, double e2,
                                                      float* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        out[i] = (float)((double)q[i] * e2);
    }
}

static uint32_t grid_for(uint64_t n) {
    uint64_t gr = (n + 255) / 256;
    if (gr < 1) gr = 1;
    if (gr > 8192) gr = 8192;
    return (uint32_t)gr;
}

template <int ND>
static void interp_anchors(hipStream_t st, const Geom& g, const int32_t* src, int32_t* dst) {
    uint32_t acnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) acnt[a] = (g.n[a] + 7) / 8;
    for (int a = 0; a < ND; a++) {
        uint64_t lines = (uint64_t)acnt[0] * acnt[1] * acnt[2] / acnt[a];
        hipLaunchKernelGGL(k_interp_anchor<ND>, dim3(grid_for(lines)), dim3(256), 0, st, g, a ? dst : src, dst, a);
    }
}

// 1D and 2D: one pass per stride and axis, in place on the residuals
template <int ND>
static void interp_inverse_passes(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out) {
    interp_anchors<ND>(st, g, q, q);
    for (uint32_t s = 4; s >= 1; s >>= 1)
        for (int a = ND - 1; a >= 0; a--) {
            // at most N / s points per pass
            hipLaunchKernelGGL(k_interp_level<ND>, dim3(grid_for(g.N / s + 1)), dim3(256), 0, st, g, q, s, a);
        }
    hipLaunchKernelGGL(k_interp_store<ND>, dim3(grid_for(g.N)), dim3(256), 0, st, g, q, e2, out);
}

template <uint32_t S>
static void launch_tile3(hipStream_t st, const Geom& g, const int32_t* R, int32_t* V, double e2, float* out, int vec,
                         uint32_t max_grid) {
    const uint32_t span = 8 * S;
    const uint32_t ntx = (g.n[0] + span - 1) / span, nty = (g.n[1] + span - 1) / span,
                   ntz = (g.n[2] + span - 1) / span;
    const uint32_t ntiles = ntx * nty * ntz;
    const uint32_t grid = ntiles < max_grid ? ntiles : max_grid;
    hipLaunchKernelGGL(k_interp_tile3<S>, dim3(grid), dim3(256), 0, st, g, R, V, e2, out, ntx, nty, ntiles, vec);
}

void launch_interp_inverse(hipStream_t st, const Geom& g, int32_t* q, int32_t* v, double e2, float* out, int vec,
                           uint32_t max_grid) {
    if (g.ndim == 3) {
        // anchors into V, then the levels of stride 4, 2 (into V) and 1
        // (into the output)
        interp_anchors<3>(st, g, q, v);
        launch_tile3<4>(st, g, q, v, e2, out, vec, max_grid);
        launch_tile3<2>(st, g, q, v, e2, out, vec, max_grid);
        launch_tile3<1>(st, g, q, v, e2, out, vec, max_grid);
    } else if (g.ndim == 2) {
        interp_inverse_passes<2>(st, g, q, e2, out);
    } else {
        interp_inverse_passes<1>(st, g, q, e2, out);
    }
}

}  // namespace fz
