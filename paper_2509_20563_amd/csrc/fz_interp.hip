// Decoding of the interpolation predictor (FZMod-Quality pipeline, Sec. 3.3:
// the G-Interp interpolator in place of Lorenzo).  The Huffman decoders
// leave the residuals of every value in the block-major residual field;
// these kernels turn them into grid values in place, in the order the
// prediction needs (fz_common.h, interp_predict):
//   k_interp_anchor - prefix sums along one axis of the anchor grid (every
//                     coordinate a multiple of 8), one thread per line
//   k_interp_level  - the points of one stride and axis: grid value =
//                     residual + prediction from points rebuilt before, one
//                     thread per point
//   k_interp_store  - dequantisation, block-major grid values to the
//                     row-major field
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// Position of (x, y, z) in the block-major residual field.
template <int ND>
__device__ __forceinline__ uint64_t bm_index(const Geom& g, uint32_t x, uint32_t y, uint32_t z) {
    if (ND == 3) {
        const uint32_t b = (x >> 3) + g.nb[0] * ((y >> 3) + g.nb[1] * (z >> 3));
        return (uint64_t)b * kBlockElems + ((x & 7u) + 8u * ((y & 7u) + 8u * (z & 7u)));
    }
    if (ND == 2) {
        const uint32_t b = (x >> 5) + g.nb[0] * (y >> 4);
        return (uint64_t)b * kBlockElems + ((x & 31u) + 32u * (y & 15u));
    }
    return (uint64_t)(x >> 9) * kBlockElems + (x & 511u);
}

// Number of coordinates c < n with c = first + step k.
__device__ __forceinline__ uint32_t n_coords(uint32_t n, uint32_t first, uint32_t step) {
    return n > first ? (n - first + step - 1) / step : 0u;
}

template <int ND>
__global__ __launch_bounds__(256) void k_interp_anchor(Geom g, int32_t* __restrict__ q, int axis) {
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
            const uint64_t i = bm_index<ND>(g, c[0], c[1], c[2]);
            acc = (int32_t)((uint32_t)acc + (uint32_t)q[i]);
            q[i] = acc;
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
    auto q_at = [&](uint32_t x, uint32_t y, uint32_t z) -> int32_t { return q[bm_index<ND>(g, x, y, z)]; };
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += stride) {
        const uint32_t c[3] = {first[0] + step[0] * (uint32_t)(p % cnt[0]),
                               first[1] + step[1] * (uint32_t)((p / cnt[0]) % cnt[1]),
                               first[2] + step[2] * (uint32_t)(p / ((uint64_t)cnt[0] * cnt[1]))};
        const int32_t pred = interp_predict(c, n3, ND, q_at);
        const uint64_t i = bm_index<ND>(g, c[0], c[1], c[2]);
        q[i] = (int32_t)((uint32_t)q[i] + (uint32_t)pred);
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_interp_store(Geom g, const int32_t* __restrict__ q, double e2,
                                                      float* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        const uint32_t x = (uint32_t)(i % g.n[0]);
        const uint64_t r = i / g.n[0];
        const uint32_t y = (uint32_t)(r % g.n[1]), z = (uint32_t)(r / g.n[1]);
        out[i] = (float)((double)q[bm_index<ND>(g, x, y, z)] * e2);
    }
}

static uint32_t grid_for(uint64_t n) {
    uint64_t gr = (n + 255) / 256;
    if (gr < 1) gr = 1;
    if (gr > 8192) gr = 8192;
    return (uint32_t)gr;
}

template <int ND>
static void interp_inverse(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out) {
    uint32_t acnt[3] = {1, 1, 1};
    for (int a = 0; a < ND; a++) acnt[a] = (g.n[a] + 7) / 8;
    for (int a = 0; a < ND; a++) {
        uint64_t lines = (uint64_t)acnt[0] * acnt[1] * acnt[2] / acnt[a];
        hipLaunchKernelGGL(k_interp_anchor<ND>, dim3(grid_for(lines)), dim3(256), 0, st, g, q, a);
    }
    for (uint32_t s = 4; s >= 1; s >>= 1)
        for (int a = ND - 1; a >= 0; a--) {
            // at most N / s points per pass
            hipLaunchKernelGGL(k_interp_level<ND>, dim3(grid_for(g.N / s + 1)), dim3(256), 0, st, g, q, s, a);
        }
    hipLaunchKernelGGL(k_interp_store<ND>, dim3(grid_for(g.N)), dim3(256), 0, st, g, q, e2, out);
}

void launch_interp_inverse(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out) {
    if (g.ndim == 3) interp_inverse<3>(st, g, q, e2, out);
    else if (g.ndim == 2) interp_inverse<2>(st, g, q, e2, out);
    else interp_inverse<1>(st, g, q, e2, out);
}

}  // namespace fz
