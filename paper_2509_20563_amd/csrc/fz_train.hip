// Training of the block-feature selector network on the device: targets,
// feature standardisation, forward pass, backpropagation and Adam (Kingma
// and Ba).  Not part of compression or decompression; the network it
// produces is used by the selector mode of the compressor.  fp32
// throughout; sums over a minibatch run in a fixed order, so a run is
// repeatable on one device, but training is not meant to be bit-exact
// across machines (a given parameter set is).
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

namespace {
constexpr int kW1 = 2 * kNFeat, kB1 = kW1 + kNHid * kNFeat, kW2 = kB1 + kNHid, kB2 = kW2 + kNHid * kNHid,
              kW3 = kB2 + kNHid, kB3 = kW3 + kNOut * kNHid;
static_assert(kB3 + kNOut == kSelectorParams, "selector layout");
}  // namespace

// t = log2(1 + bits) per sample and predictor
__global__ void k_targets(const uint32_t* __restrict__ costs, uint64_t n, float* __restrict__ t) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += (uint64_t)gridDim.x * blockDim.x)
        t[i] = log2f(1.0f + (float)costs[i]);
}

// mean and standard deviation of each feature over the samples (one
// workgroup per feature, fixed-order tree reduction in double); writes
// mu and rs = 1 / std (1 where the feature is constant)
__global__ __launch_bounds__(256) void k_feature_stats(const float* __restrict__ feat, uint64_t n,
                                                       float* __restrict__ w) {
    __shared__ double s1[256], s2[256];
    const uint32_t f = blockIdx.x, t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (uint64_t i = t; i < n; i += 256) {
        const double v = feat[i * kNFeat + f];
        a += v;
        b += v * v;
    }
    s1[t] = a;
    s2[t] = b;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s1[t] += s1[t + h];
            s2[t] += s2[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double m = s1[0] / (double)n;
        double var = s2[0] / (double)n - m * m;
        if (var < 0.0) var = 0.0;
        const double sd = sqrt(var);
        w[f] = (float)m;
        w[kNFeat + f] = sd > 1e-12 ? (float)(1.0 / sd) : 1.0f;
    }
}

// Forward pass, one thread per sample of the batch: keeps z, h1, h2 and
// dL/dy = 2 (y - t) / (3 B), and the sample's squared error.
__global__ __launch_bounds__(256) void k_fwd(const float* __restrict__ w, const float* __restrict__ feat,
                                             const float* __restrict__ tgt, const uint32_t* __restrict__ idx,
                                             uint32_t B, float* __restrict__ Z, float* __restrict__ H1,
                                             float* __restrict__ H2, float* __restrict__ DY, float* __restrict__ SE) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const uint64_t k = idx ? idx[s] : s;
    float z[kNFeat], h1[kNHid];
    for (int i = 0; i < kNFeat; i++) {
        z[i] = (feat[k * kNFeat + i] - w[i]) * w[kNFeat + i];
        Z[(uint64_t)s * kNFeat + i] = z[i];
    }
    for (int j = 0; j < kNHid; j++) {
        float acc = w[kB1 + j];
        for (int i = 0; i < kNFeat; i++) acc += w[kW1 + j * kNFeat + i] * z[i];
        h1[j] = acc > 0.0f ? acc : 0.0f;
        H1[(uint64_t)s * kNHid + j] = h1[j];
    }
    float y[kNOut] = {w[kB3], w[kB3 + 1], w[kB3 + 2]};
    for (int j = 0; j < kNHid; j++) {
        float acc = w[kB2 + j];
        for (int i = 0; i < kNHid; i++) acc += w[kW2 + j * kNHid + i] * h1[i];
        const float h = acc > 0.0f ? acc : 0.0f;
        H2[(uint64_t)s * kNHid + j] = h;
        for (int o = 0; o < kNOut; o++) y[o] += w[kW3 + o * kNHid + j] * h;
    }
    float se = 0.0f;
    for (int o = 0; o < kNOut; o++) {
        const float e = y[o] - tgt[k * kNOut + o];
        se += e * e;
        DY[(uint64_t)s * kNOut + o] = 2.0f * e / (3.0f * (float)B);
    }
    SE[s] = se;
}

// Backpropagation through the hidden layers, one thread per sample:
// dh2 = (dy W3) where h2 > 0, dh1 = (dh2 W2) where h1 > 0.
__global__ __launch_bounds__(256) void k_bwd(const float* __restrict__ w, uint32_t B, const float* __restrict__ H1,
                                             const float* __restrict__ H2, const float* __restrict__ DY,
                                             float* __restrict__ DH1, float* __restrict__ DH2) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float d2[kNHid];
    for (int i = 0; i < kNHid; i++) {
        float acc = 0.0f;
        for (int o = 0; o < kNOut; o++) acc += DY[(uint64_t)s * kNOut + o] * w[kW3 + o * kNHid + i];
        d2[i] = H2[(uint64_t)s * kNHid + i] > 0.0f ? acc : 0.0f;
        DH2[(uint64_t)s * kNHid + i] = d2[i];
    }
    for (int i = 0; i < kNHid; i++) {
        float acc = 0.0f;
        for (int j = 0; j < kNHid; j++) acc += d2[j] * w[kW2 + j * kNHid + i];
        DH1[(uint64_t)s * kNHid + i] = H1[(uint64_t)s * kNHid + i] > 0.0f ? acc : 0.0f;
    }
}

// Weight gradients, one thread per learned parameter, summed over the
// batch in sample order: dW = delta^T * activations, db = sum delta.
__global__ __launch_bounds__(256) void k_wgrad(uint32_t B, const float* __restrict__ Z, const float* __restrict__ H1,
                                               const float* __restrict__ H2, const float* __restrict__ DY,
                                               const float* __restrict__ DH1, const float* __restrict__ DH2,
                                               float* __restrict__ grad) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint32_t)kSelectorParams) return;
    // which tensor: delta array D (width dw, column dc) times activation
    // array X (width xw, column xc); X = null for a bias
    const float *D = nullptr, *X = nullptr;
    uint32_t dw = 0, dc = 0, xw = 0, xc = 0;
    if (p < (uint32_t)kW1) {
        grad[p] = 0.0f;  // mu, rs: set from the data, not learned
        return;
    } else if (p < (uint32_t)kB1) {
        D = DH1; dw = kNHid; dc = (p - kW1) / kNFeat; X = Z; xw = kNFeat; xc = (p - kW1) % kNFeat;
    } else if (p < (uint32_t)kW2) {
        D = DH1; dw = kNHid; dc = p - kB1;
    } else if (p < (uint32_t)kB2) {
        D = DH2; dw = kNHid; dc = (p - kW2) / kNHid; X = H1; xw = kNHid; xc = (p - kW2) % kNHid;
    } else if (p < (uint32_t)kW3) {
        D = DH2; dw = kNHid; dc = p - kB2;
    } else if (p < (uint32_t)kB3) {
        D = DY; dw = kNOut; dc = (p - kW3) / kNHid; X = H2; xw = kNHid; xc = (p - kW3) % kNHid;
    } else {
        D = DY; dw = kNOut; dc = p - kB3;
    }
    float acc = 0.0f;
    if (X) {
        for (uint32_t s = 0; s < B; s++) acc += D[(uint64_t)s * dw + dc] * X[(uint64_t)s * xw + xc];
    } else {
        for (uint32_t s = 0; s < B; s++) acc += D[(uint64_t)s * dw + dc];
    }
    grad[p] = acc;
}

// Sum of the batch's squared errors / (3 B), one workgroup, fixed order.
__global__ __launch_bounds__(256) void k_batch_loss(const float* __restrict__ SE, uint32_t B, float* __restrict__ out) {
    __shared__ float r[256];
    const uint32_t t = threadIdx.x;
    float a = 0.0f;
    for (uint32_t i = t; i < B; i += 256) a += SE[i];
    r[t] = a;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (t < h) r[t] += r[t + h];
        __syncthreads();
    }
    if (t == 0) *out = r[0] / (3.0f * (float)B);
}

// Adam on the learned parameters; step number t >= 1.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < (uint32_t)kW1 || p >= (uint32_t)kSelectorParams) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

void launch_targets(hipStream_t st, const uint32_t* costs, uint64_t n, float* t) {
    uint64_t grid = (3 * n + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (grid) hipLaunchKernelGGL(k_targets, dim3((uint32_t)grid), dim3(256), 0, st, costs, n, t);
}

void launch_feature_stats(hipStream_t st, const float* feat, uint64_t n, float* w) {
    hipLaunchKernelGGL(k_feature_stats, dim3(kNFeat), dim3(256), 0, st, feat, n, w);
}

void launch_train_batch(hipStream_t st, const float* w, const float* feat, const float* tgt, const uint32_t* idx,
                        uint32_t B, TrainScratch& s, float* loss_out) {
    const uint32_t gb = (B + 255) / 256;
    hipLaunchKernelGGL(k_fwd, dim3(gb), dim3(256), 0, st, w, feat, tgt, idx, B, s.Z, s.H1, s.H2, s.DY, s.SE);
    hipLaunchKernelGGL(k_bwd, dim3(gb), dim3(256), 0, st, w, B, s.H1, s.H2, s.DY, s.DH1, s.DH2);
    hipLaunchKernelGGL(k_wgrad, dim3((kSelectorParams + 255) / 256), dim3(256), 0, st, B, s.Z, s.H1, s.H2, s.DY,
                       s.DH1, s.DH2, s.grad);
    if (loss_out) hipLaunchKernelGGL(k_batch_loss, dim3(1), dim3(256), 0, st, s.SE, B, loss_out);
}

void launch_adam(hipStream_t st, float* w, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
                 float eps) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((kSelectorParams + 255) / 256), dim3(256), 0, st, w, m, v, g, lr, b1, b2, eps,
                       c1, c2);
}

}  // namespace fz
