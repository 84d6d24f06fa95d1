// Learned level-of-detail network: inference over feature batches and one
// training step (forward, backward, Adam) with hand-written kernels.
//
// Network 8 -> 32 -> 32 -> 1 (ReLU, logit of P(refine)), BF16 weights used
// in every forward pass, FP32 master weights updated by Adam, FP32
// accumulation throughout.  Loss: mean binary cross-entropy with logits.
// Gradient sums run in a fixed order (per-sample terms, then per-chunk
// partial sums, then the chunks in index order), so a training run is
// bitwise reproducible.
#include "device_util.h"
#include "internal.h"
#include "lod_mlp.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
// per-sample record of the training pass, stored feature-major [k][n]:
// x[8], h1[32], h2[32], d1[32] (dL/da1), d2[32] (dL/da2), dz
constexpr int kOffX = 0, kOffH1 = 8, kOffH2 = 40, kOffD1 = 72, kOffD2 = 104, kOffDz = 136, kActRows = 137;

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7fffu + ((b >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(b >> 16);
}

struct MlpNorm {
    float mean[kMlpIn];
    float inv_std[kMlpIn];
};

__global__ __launch_bounds__(kNT) void k_mlp_forward(const float* __restrict__ feats, uint32_t n, MlpNorm nm,
                                                     const uint16_t* __restrict__ w, float* __restrict__ logits) {
    for (uint32_t s = blockIdx.x * kNT + threadIdx.x; s < n; s += gridDim.x * kNT) {
        float x[kMlpIn];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) x[i] = (feats[(size_t)s * kMlpIn + i] - nm.mean[i]) * nm.inv_std[i];
        logits[s] = lod_mlp_logit(w, x);
    }
}

// Forward and backward of one sample per thread; loss partial per block.
__global__ __launch_bounds__(kNT) void k_mlp_fwd_bwd(const float* __restrict__ feats, const float* __restrict__ labels,
                                                     uint32_t n, MlpNorm nm, const uint16_t* __restrict__ w,
                                                     float* __restrict__ act, float* __restrict__ loss_part) {
    __shared__ float s_w[kMlpParams];
    __shared__ float s_red[kNT];
    for (int i = threadIdx.x; i < kMlpParams; i += kNT) s_w[i] = bf16_to_f32(w[i]);
    __syncthreads();
    const uint32_t s = blockIdx.x * kNT + threadIdx.x;
    float lossv = 0.f;
    if (s < n) {
        float x[kMlpIn], a1[kMlpH], h1[kMlpH], a2[kMlpH], h2[kMlpH];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) x[i] = (feats[(size_t)s * kMlpIn + i] - nm.mean[i]) * nm.inv_std[i];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) {
            float acc = s_w[kOffB1 + j];
#pragma unroll
            for (int i = 0; i < kMlpIn; ++i) acc = fmaf(s_w[kOffW1 + j * kMlpIn + i], x[i], acc);
            a1[j] = acc;
            h1[j] = acc > 0.f ? acc : 0.f;
        }
        float z = s_w[kOffB3];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) {
            float acc = s_w[kOffB2 + j];
#pragma unroll
            for (int i = 0; i < kMlpH; ++i) acc = fmaf(s_w[kOffW2 + j * kMlpH + i], h1[i], acc);
            a2[j] = acc;
            h2[j] = acc > 0.f ? acc : 0.f;
            z = fmaf(s_w[kOffW3 + j], h2[j], z);
        }
        const float y = labels[s];
        lossv = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - y * z;
        const float p = 1.f / (1.f + expf(-z));
        const float dz = (p - y) / (float)n;
        float d2[kMlpH];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) d2[j] = a2[j] > 0.f ? dz * s_w[kOffW3 + j] : 0.f;
        float d1[kMlpH];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < kMlpH; ++j) acc = fmaf(s_w[kOffW2 + j * kMlpH + i], d2[j], acc);
            d1[i] = a1[i] > 0.f ? acc : 0.f;
        }
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) act[(size_t)(kOffX + i) * n + s] = x[i];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) {
            act[(size_t)(kOffH1 + j) * n + s] = h1[j];
            act[(size_t)(kOffH2 + j) * n + s] = h2[j];
            act[(size_t)(kOffD1 + j) * n + s] = d1[j];
            act[(size_t)(kOffD2 + j) * n + s] = d2[j];
        }
        act[(size_t)kOffDz * n + s] = dz;
    }
    // fixed-order tree reduction of the block's losses
    s_red[threadIdx.x] = lossv;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s_red[threadIdx.x] += s_red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s_red[0];
}

// Partial gradient of parameter p over the samples of chunk blockIdx.y.
__global__ __launch_bounds__(kNT) void k_mlp_grad_partial(const float* __restrict__ act, uint32_t n, uint32_t chunk,
                                                          float* __restrict__ partial) {
    const int p = blockIdx.x * kNT + threadIdx.x;
    if (p >= kMlpParams) return;
    const uint32_t lo = blockIdx.y * chunk, hi = min(n, lo + chunk);
    int ra, rb = -1;   // act rows: gradient = sum_s act[ra][s] * act[rb][s] (rb < 0: just act[ra])
    if (p < kOffB1) { ra = kOffD1 + (p - kOffW1) / kMlpIn; rb = kOffX + (p - kOffW1) % kMlpIn; }
    else if (p < kOffW2) { ra = kOffD1 + (p - kOffB1); }
    else if (p < kOffB2) { ra = kOffD2 + (p - kOffW2) / kMlpH; rb = kOffH1 + (p - kOffW2) % kMlpH; }
    else if (p < kOffW3) { ra = kOffD2 + (p - kOffB2); }
    else if (p < kOffB3) { ra = kOffDz; rb = kOffH2 + (p - kOffW3); }
    else { ra = kOffDz; }
    const float* A = act + (size_t)ra * n;
    float acc = 0.f;
    if (rb >= 0) {
        const float* B = act + (size_t)rb * n;
        for (uint32_t s = lo; s < hi; ++s) acc = fmaf(A[s], B[s], acc);
    } else {
        for (uint32_t s = lo; s < hi; ++s) acc += A[s];
    }
    partial[(size_t)blockIdx.y * kMlpParams + p] = acc;
}

struct AdamArgs {
    float* master;
    uint16_t* w;
    float* m;
    float* v;
    float lr, beta1, beta2, eps;
    int step;
    float* grad_out;
    float* loss_out;
    const float* loss_part;
    uint32_t n_loss_part;
    uint32_t n;
};

__global__ __launch_bounds__(kNT) void k_mlp_reduce_adam(const float* __restrict__ partial, uint32_t chunks, AdamArgs a) {
    const int p = blockIdx.x * kNT + threadIdx.x;
    if (p == 0 && a.loss_out) {
        float t = 0.f;
        for (uint32_t i = 0; i < a.n_loss_part; ++i) t += a.loss_part[i];
        *a.loss_out = t / (float)a.n;
    }
    if (p >= kMlpParams) return;
    float g = 0.f;
    for (uint32_t c = 0; c < chunks; ++c) g += partial[(size_t)c * kMlpParams + p];
    if (a.grad_out) a.grad_out[p] = g;
    if (a.lr > 0.f) {
        const float m = a.beta1 * a.m[p] + (1.f - a.beta1) * g;
        const float v = a.beta2 * a.v[p] + (1.f - a.beta2) * g * g;
        a.m[p] = m;
        a.v[p] = v;
        const float mh = m / (1.f - powf(a.beta1, (float)a.step));
        const float vh = v / (1.f - powf(a.beta2, (float)a.step));
        const float w = a.master[p] - a.lr * mh / (sqrtf(vh) + a.eps);
        a.master[p] = w;
        a.w[p] = f32_to_bf16(w);
    }
}

__global__ void k_bf16_from_master(const float* master, uint16_t* w) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) w[p] = f32_to_bf16(master[p]);
}

// Mean and standard deviation of each of the 8 feature columns, FP64 sums
// in a fixed order (one block).
__global__ __launch_bounds__(kNT) void k_feat_stats(const float* __restrict__ f, uint32_t n, float* __restrict__ out) {
    __shared__ double s1[kNT], s2[kNT];
    for (int k = 0; k < kMlpIn; ++k) {
        double a = 0.0, b = 0.0;
        for (uint32_t s = threadIdx.x; s < n; s += kNT) {
            const double x = f[(size_t)s * kMlpIn + k];
            a += x;
            b += x * x;
        }
        s1[threadIdx.x] = a;
        s2[threadIdx.x] = b;
        __syncthreads();
        for (int o = kNT / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                s1[threadIdx.x] += s1[threadIdx.x + o];
                s2[threadIdx.x] += s2[threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double mean = n ? s1[0] / n : 0.0;
            const double var = n ? fmax(s2[0] / n - mean * mean, 0.0) : 0.0;
            out[k] = (float)mean;
            out[kMlpIn + k] = (float)fmax(sqrt(var), 1e-6);
        }
        __syncthreads();
    }
}

}  // namespace

void launch_mlp_forward(const float* feats, uint32_t n, const float* mean, const float* stdv, const uint16_t* w,
                        float* logits, hipStream_t s) {
    MlpNorm nm;
    for (int i = 0; i < kMlpIn; ++i) {
        nm.mean[i] = mean[i];
        nm.inv_std[i] = 1.f / stdv[i];
    }
    const uint32_t grid = n ? min(4096u, ceil_div(n, (uint32_t)kNT)) : 1u;
    k_mlp_forward<<<grid, kNT, 0, s>>>(feats, n, nm, w, logits);
}

size_t mlp_train_scratch_floats(uint32_t n) {
    const uint32_t chunks = min(64u, max(1u, ceil_div(n, 512u)));
    return (size_t)kActRows * n + (size_t)chunks * kMlpParams + ceil_div(n, (uint32_t)kNT) + 16;
}

void launch_mlp_train_step(const float* feats, const float* labels, uint32_t n, const float* mean, const float* stdv,
                           float* master, uint16_t* w, float* m, float* v, int step, float lr, float* grad_out,
                           float* loss_out, float* scratch, hipStream_t s) {
    MlpNorm nm;
    for (int i = 0; i < kMlpIn; ++i) {
        nm.mean[i] = mean[i];
        nm.inv_std[i] = 1.f / stdv[i];
    }
    const uint32_t chunks = min(64u, max(1u, ceil_div(n, 512u)));
    const uint32_t chunk = ceil_div(n, chunks);
    const uint32_t nblk = ceil_div(n, (uint32_t)kNT);
    float* act = scratch;
    float* partial = act + (size_t)kActRows * n;
    float* loss_part = partial + (size_t)chunks * kMlpParams;
    k_mlp_fwd_bwd<<<nblk, kNT, 0, s>>>(feats, labels, n, nm, w, act, loss_part);
    dim3 g((kMlpParams + kNT - 1) / kNT, chunks);
    k_mlp_grad_partial<<<g, kNT, 0, s>>>(act, n, chunk, partial);
    AdamArgs a;
    a.master = master;
    a.w = w;
    a.m = m;
    a.v = v;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.step = step;
    a.grad_out = grad_out;
    a.loss_out = loss_out;
    a.loss_part = loss_part;
    a.n_loss_part = nblk;
    a.n = n;
    k_mlp_reduce_adam<<<(kMlpParams + kNT - 1) / kNT, kNT, 0, s>>>(partial, chunks, a);
}

void launch_mlp_adam(const float* grad, float* master, uint16_t* w, float* m, float* v, int step, float lr,
                     hipStream_t s) {
    AdamArgs a;
    a.master = master;
    a.w = w;
    a.m = m;
    a.v = v;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.step = step;
    a.grad_out = nullptr;
    a.loss_out = nullptr;
    a.loss_part = nullptr;
    a.n_loss_part = 0;
    a.n = 1;
    // one "chunk": the gradient itself, summed as g = 0 + grad, exactly grad
    k_mlp_reduce_adam<<<(kMlpParams + kNT - 1) / kNT, kNT, 0, s>>>(grad, 1, a);
}

void launch_bf16_from_master(const float* master, uint16_t* w, hipStream_t s) {
    k_bf16_from_master<<<(kMlpParams + 255) / 256, 256, 0, s>>>(master, w);
}

void launch_feat_stats(const float* f, uint32_t n, float* out, hipStream_t s) {
    k_feat_stats<<<1, kNT, 0, s>>>(f, n, out);
}

}  // namespace hgs
