// Image helpers for learned-LOD labels and PSNR: 2x2 box downsampling of a
// planar RGB image, and mean squared error of many image windows against
// crops of reference images.  FP64 sums in a fixed order.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

// Streaming copy (the bandwidth probe): each workgroup copies contiguous
// chunks of 4 KiB per step -- four 16-byte nontemporal loads per thread in
// flight, then four nontemporal stores -- and the grid strides over the
// chunks.  (Measured on MI355X: 5.9 TB/s read + write; a grid-stride loop
// over single 16-byte words reached 4.2-4.8, a D2D hipMemcpy 5.1.)
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const v4u* __restrict__ src, v4u* __restrict__ dst, size_t n16) {
    constexpr size_t kPer = 256 * 4;
    for (size_t base = blockIdx.x * kPer; base < n16; base += (size_t)gridDim.x * kPer) {
        v4u v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t i = base + u * 256 + threadIdx.x;
            if (i < n16) v[u] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t i = base + u * 256 + threadIdx.x;
            if (i < n16) __builtin_nontemporal_store(v[u], &dst[i]);
        }
    }
}

__global__ void k_downsample2x(const float* __restrict__ src, int W, int H, float* __restrict__ dst) {
    const size_t plane = (size_t)W * H, splane = 4 * plane;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 3 * plane; i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / plane, r = i % plane;
        const int y = (int)(r / W), x = (int)(r % W);
        const float* s = src + c * splane + (size_t)(2 * y) * (2 * W) + 2 * x;
        dst[i] = 0.25f * ((s[0] + s[1]) + (s[2 * W] + s[2 * W + 1]));
    }
}

// Mean squared error over the 3 channels of region r (block of 256 threads,
// FP64 sums in a fixed order), rounded to FP32; every thread returns it.
__device__ float region_mse_block(const RegionDev& r, double* sh) {
    const size_t np = (size_t)r.w * r.h;
    const size_t rplane = (size_t)r.ref_w * r.ref_h;
    double acc = 0.0;
    for (size_t i = threadIdx.x; i < 3 * np; i += 256) {
        const size_t c = i / np, k = i % np;
        const int y = (int)(k / r.w), x = (int)(k % r.w);
        const float a = r.img[i];
        const float b = r.ref[c * rplane + (size_t)(r.y0 + y) * r.ref_w + (r.x0 + x)];
        const double d = (double)a - (double)b;
        acc += d * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const float mse = np ? (float)(sh[0] / (3.0 * np)) : 0.f;
    __syncthreads();
    return mse;
}

// Expand-vs-keep label of candidate i: regions 2i (window with the node
// refined, the threshold cut) and 2i + 1 (the node's subtree collapsed to
// it) against the same reference crop; the window's PSNR drop from keeping
// the node, 10 log10(MSE_kept / MSE_refined) with both MSEs floored at
// 1e-10, labels "refine" when it exceeds label_db.
__global__ __launch_bounds__(256) void k_lod_labels(const RegionDev* __restrict__ reg, double label_db,
                                                    float* __restrict__ labels, float* __restrict__ drop_db) {
    __shared__ double sh[256];
    const float refined = region_mse_block(reg[2 * blockIdx.x], sh);
    const float kept = region_mse_block(reg[2 * blockIdx.x + 1], sh);
    if (threadIdx.x == 0) {
        const double a = fmax((double)refined, 1e-10), b = fmax((double)kept, 1e-10);
        const double drop = 10.0 * log10(b / a);
        if (drop_db) drop_db[blockIdx.x] = (float)drop;
        labels[blockIdx.x] = drop > label_db ? 1.f : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_region_mse(const RegionDev* __restrict__ reg, float* __restrict__ out) {
    __shared__ double sh[256];
    const RegionDev r = reg[blockIdx.x];
    const size_t np = (size_t)r.w * r.h;
    const size_t rplane = (size_t)r.ref_w * r.ref_h;
    double acc = 0.0;
    for (size_t i = threadIdx.x; i < 3 * np; i += 256) {
        const size_t c = i / np, k = i % np;
        const int y = (int)(k / r.w), x = (int)(k % r.w);
        const float a = r.img[i];
        const float b = r.ref[c * rplane + (size_t)(r.y0 + y) * r.ref_w + (r.x0 + x)];
        const double d = (double)a - (double)b;
        acc += d * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = np ? (float)(sh[0] / (3.0 * np)) : 0.f;
}

}  // namespace

void launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    k_stream_copy<<<256 * 32, 256, 0, s>>>(static_cast<const v4u*>(src), static_cast<v4u*>(dst), bytes / 16);
}

void launch_lod_labels(const RegionDev* reg, int n, double label_db, float* labels, float* drop_db, hipStream_t s) {
    if (n > 0) k_lod_labels<<<n, 256, 0, s>>>(reg, label_db, labels, drop_db);
}

void launch_downsample2x(const float* src, int W, int H, float* dst, hipStream_t s) {
    const size_t n = 3 * (size_t)W * H;
    const int grid = (int)std::min<size_t>(4096, (n + 255) / 256);
    k_downsample2x<<<grid > 0 ? grid : 1, 256, 0, s>>>(src, W, H, dst);
}

void launch_region_mse(const RegionDev* reg, int n, float* out, hipStream_t s) {
    if (n > 0) k_region_mse<<<n, 256, 0, s>>>(reg, out);
}

}  // namespace hgs
