// Front-to-back alpha compositing per 16x16 tile.
//
// One 256-thread workgroup (four wave64s) per tile, one pixel per thread.
// The tile's depth-sorted list is walked in batches: each batch is staged in
// LDS as tile-relative single-precision records (the FP64 2D mean is made
// tile-relative before rounding, so pixel offsets keep full precision), then
// every thread walks the batch for its pixel.  Per entry:
//   q = (p dx + r dy)^2 + (s dy)^2; skip unless q <= 9 (3-sigma support);
//   alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255;
//   T' = T (1 - alpha); stop before adding if T' < 1e-4;
//   C += c alpha T, D += z alpha T, T = T'.
// A workgroup leaves its list as soon as a barrier count shows every pixel
// has stopped.  This is plain FP32 vector arithmetic, no matrix cores: the
// work is a per-pixel recurrence, not a dense contraction.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = kTilePx;     // 256 threads, one per pixel
// exp(-q/2) = 2^(q * kNegHalfLog2e)
constexpr float kNegHalfLog2e = -0.72134752044448170f;

__global__ void k_ranges_zero(uint2* ranges, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ranges[i] = make_uint2(0, 0);
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, const Counters* ctr, uint32_t cap, uint2* ranges,
                         uint32_t n_tiles) {
    const uint32_t P = min(ctr->pairs, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const uint32_t k = keys[i];
        if (k >= n_tiles) continue;
        if (i == 0 || keys[i - 1] != k) ranges[k].x = i;
        if (i + 1 == P || keys[i + 1] != k) ranges[k].y = i + 1;
    }
}

template <int BATCH, bool COUNT>
__device__ __forceinline__ void composite_tile(const CompositeArgs& a, uint32_t tile, float4* s_a, float4* s_b,
                                               float2* s_c, uint32_t* s_m, uint32_t* s_red) {
    const uint32_t view = a.tile_view[tile];
    const ViewDev& V = a.views[view];
    const uint32_t local = tile - V.tile_base;
    const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < V.width && py < V.height;
    const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
    const double dx0 = (double)x0, dy0 = (double)y0;
    const uint2 rg = a.ranges[tile];
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    bool done = !inside;
    uint32_t nalg = 0;
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
        const uint32_t cnt = min((uint32_t)BATCH, rg.y - base);
        for (uint32_t j = threadIdx.x; j < cnt; j += kNT) {
            const uint32_t val = a.vals[base + j];
            const uint32_t e = val & kEntryMask;
            const Proj p = a.proj[e < a.cut_cap ? e : 0u];
            s_a[j] = make_float4((float)(p.u - dx0), (float)(p.v - dy0), p.p, p.r);
            s_b[j] = make_float4(p.s, p.opacity, p.z, p.c0);
            s_c[j] = make_float2(p.c1, p.c2);
            s_m[j] = val >> kStripShift;
        }
        __syncthreads();
        if (!done) {
            const uint32_t wbit = 1u << (threadIdx.x / kWave);
            for (uint32_t j = 0; j < cnt; ++j) {
                // entries that reach no pixel centre of this wave's strip
                if (!(__builtin_amdgcn_readfirstlane(s_m[j]) & wbit)) continue;
                const float4 A = s_a[j];
                const float ddx = fx - A.x, ddy = fy - A.y;
                const float4 B = s_b[j];
                const float t1 = fmaf(A.w, ddy, A.z * ddx);
                const float t2 = B.x * ddy;
                const float q = fmaf(t1, t1, t2 * t2);
                if (q <= 9.f) {
                    if (COUNT) ++nalg;
                    const float al = fminf(0.99f, B.y * __builtin_amdgcn_exp2f(q * kNegHalfLog2e));
                    if (al >= 1.f / 255.f) {
                        const float Tn = T * (1.f - al);
                        if (Tn < 1e-4f) {
                            done = true;
                            break;
                        }
                        const float w = al * T;
                        const float2 Cc = s_c[j];
                        C0 = fmaf(w, B.w, C0);
                        C1 = fmaf(w, Cc.x, C1);
                        C2 = fmaf(w, Cc.y, C2);
                        D = fmaf(w, B.z, D);
                        T = Tn;
                    }
                }
            }
        }
        if (__syncthreads_count(done ? 0 : 1) == 0) break;
    }
    if (inside) {
        const size_t plane = (size_t)V.width * V.height;
        const size_t o = (size_t)py * V.width + px;
        V.rgb[o] = C0 + T * V.bg[0];
        V.rgb[plane + o] = C1 + T * V.bg[1];
        V.rgb[2 * plane + o] = C2 + T * V.bg[2];
        if (V.depth) V.depth[o] = D;
        if (V.alpha) V.alpha[o] = 1.f - T;
    }
    if (COUNT) {
        uint32_t s = wave_sum(nalg);
        if (lane_id() == 0) s_red[threadIdx.x / kWave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int i = 0; i < kNT / kWave; ++i) t += s_red[i];
            if (t) atomicAdd(&a.ctr->nalg, t);
        }
        __syncthreads();
    }
}

template <int BATCH, bool COUNT>
__global__ __launch_bounds__(kNT) void k_composite(CompositeArgs a) {
    __shared__ float4 s_a[BATCH];
    __shared__ float4 s_b[BATCH];
    __shared__ float2 s_c[BATCH];
    __shared__ uint32_t s_m[BATCH];
    __shared__ uint32_t s_red[kNT / kWave];
    composite_tile<BATCH, COUNT>(a, blockIdx.x, s_a, s_b, s_c, s_m, s_red);
}

// Persistent variant: a fixed grid takes tiles from a global counter until
// the counter passes the last tile (every workgroup reaches that exit).
template <int BATCH, bool COUNT>
__global__ __launch_bounds__(kNT) void k_composite_persistent(CompositeArgs a) {
    __shared__ float4 s_a[BATCH];
    __shared__ float4 s_b[BATCH];
    __shared__ float2 s_c[BATCH];
    __shared__ uint32_t s_m[BATCH];
    __shared__ uint32_t s_red[kNT / kWave];
    __shared__ uint32_t s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&a.ctr->tile_queue, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        __syncthreads();
        if (tile >= a.total_tiles) break;
        composite_tile<BATCH, COUNT>(a, tile, s_a, s_b, s_c, s_m, s_red);
    }
}

template <int BATCH>
void launch_b(const CompositeArgs& a, hipStream_t s) {
    if (a.opts.persistent) {
        const uint32_t grid = min(a.total_tiles, 256u * 8u);
        if (a.opts.count_nalg) k_composite_persistent<BATCH, true><<<grid, kNT, 0, s>>>(a);
        else k_composite_persistent<BATCH, false><<<grid, kNT, 0, s>>>(a);
    } else {
        if (a.opts.count_nalg) k_composite<BATCH, true><<<a.total_tiles, kNT, 0, s>>>(a);
        else k_composite<BATCH, false><<<a.total_tiles, kNT, 0, s>>>(a);
    }
}

}  // namespace

void launch_ranges(const CompositeArgs& a, hipStream_t s) {
    k_ranges_zero<<<1024, 256, 0, s>>>(a.ranges, a.total_tiles);
    k_ranges<<<4096, 256, 0, s>>>(a.keys, a.ctr, a.pair_cap, a.ranges, a.total_tiles);
}

void launch_composite(const CompositeArgs& a, hipStream_t s) {
    if (a.total_tiles == 0) return;
    switch (a.opts.batch) {
        case 64: launch_b<64>(a, s); break;
        case 128: launch_b<128>(a, s); break;
        case 512: launch_b<512>(a, s); break;
        default: launch_b<256>(a, s); break;
    }
}

}  // namespace hgs
