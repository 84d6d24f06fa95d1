// Front-to-back alpha compositing per 16x16 tile.
//
// One 256-thread workgroup (four wave64s) per tile, one pixel per thread;
// each 16-lane quarter of a wave owns one 4x4 block of the tile.  The tile's
// depth-sorted list is walked in batches of BATCH entries:
//  1. staging: thread j turns entry j into a tile-relative FP32 record (the
//     FP64 2D mean is made tile-relative before rounding) and marks the 4x4
//     blocks holding a pixel centre that its 3-sigma ellipse may reach
//     (closed-form extent per band of four rows, with a relative slack of
//     1e-3 on the bound 9);
//  2. compaction: for every block, the indices of its marked entries in
//     depth order (ballots and prefix counts);
//  3. compositing: the 16 lanes of a block walk that block's list; a wave
//     runs to the longest of its four lists and shorter lists are padded
//     with a record that contributes nothing.  The body has no branches:
//       q = t1^2 + t2^2 with t1 = p dx + r dy = p x + r y + c1 and
//           t2 = s dy = s y + c2 around the tile origin;
//       x = log2(o) - q log2(e)/2, alpha = min(0.99, 2^x) = min(0.99, o e^(-q/2));
//       the entry adds only to a live pixel with q <= 9 and x >= log2(1/255)
//       (alpha >= 1/255, the cap 0.99 lying above it);
//       T' = T - alpha T; if T' < 1e-4 the pixel stops without adding,
//       else C += c alpha T, D += z alpha T, T = T'.
// A wave leaves its lists once a ballot shows all its pixels stopped, the
// workgroup once a barrier count does.  This is plain FP32 vector arithmetic,
// no matrix cores: the work is a per-pixel recurrence, not a dense
// contraction.
#include "blocks.h"
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

// [first, last + 1) of every tile's run in the tile-sorted keys, four keys
// per thread and step (16-byte loads; key arrays start 256-byte aligned).
__global__ void k_ranges(const uint32_t* __restrict__ keys, const Counters* ctr, uint32_t cap, uint2* ranges,
                         uint32_t n_tiles) {
    const uint32_t P = min(ctr->pairs, cap);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; 4ull * q < P; q += gridDim.x * blockDim.x) {
        const uint32_t i0 = 4 * q;
        uint32_t k[6];
        k[0] = i0 > 0 ? keys[i0 - 1] : 0xffffffffu;     // tile ids are below 2^31
        if (i0 + 4 <= P) {
            const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
            k[1] = v.x; k[2] = v.y; k[3] = v.z; k[4] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < P ? keys[i0 + j] : 0xffffffffu;
        }
        k[5] = i0 + 4 < P ? keys[i0 + 4] : 0xffffffffu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t kk = k[1 + j];
            if (kk >= n_tiles) continue;
            if (k[j] != kk) ranges[kk].x = i0 + j;
            if (k[j + 2] != kk) ranges[kk].y = i0 + j + 1;
        }
    }
}

template <int BATCH, bool COUNT, bool KEEP>
__device__ __forceinline__ void composite_tile(const CompositeArgs& a, uint32_t tile, StageA* s_a, StageB* s_b,
                                               StageC* s_c, uint16_t* s_idx, uint32_t* s_wc, uint32_t* s_n,
                                               uint32_t* s_red) {
    static_assert(BATCH <= kNT, "one entry per staging thread");
    const uint32_t view = a.tile_view[tile];
    const ViewDev& V = a.views[view];
    const uint32_t local = tile - V.tile_base;
    const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int g = lane >> 4, k = lane & 15;
    const int gid = w * 4 + g;                          // this lane's 4x4 block
    const int lx = g * 4 + (k & 3), ly = w * 4 + (k >> 2);
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < V.width && py < V.height;
    const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
    const double dx0 = (double)x0, dy0 = (double)y0;
    const uint2 rg = a.ranges[tile];
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    bool live = inside;
    uint32_t nalg = 0, neval = 0;
    uint32_t stop_at = 0xffffffffu;                     // list position where the pixel stopped
    if (threadIdx.x == 0) {                             // record that adds nothing
        s_a[BATCH] = StageA{0.f, 0.f, 0.f, 0.f};
        s_b[BATCH] = StageB{0.f, -__builtin_inff(), 0.f, 0.f};
        s_c[BATCH] = StageC{0.f, 0.f};
    }
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
        const uint32_t cnt = min((uint32_t)BATCH, rg.y - base);
        // 1. staging
        uint32_t m = 0;
        const int j = threadIdx.x;
        if (j < (int)cnt) {
            const uint32_t val = a.vals[base + j];
            const uint32_t e = val;
            const Proj P = a.proj[e < a.cut_cap ? e : 0u];
            const float u = (float)(P.u - dx0), v = (float)(P.v - dy0);
            s_a[j] = StageA{P.p, P.r, -fmaf(P.p, u, P.r * v), P.s};
            s_b[j] = StageB{-P.s * v, __log2f(P.opacity), P.z, P.c0};
            s_c[j] = StageC{P.c1, P.c2};
            m = block_mask(u, v, P.p, P.r, P.s);
        }
        // 2. per-block lists in depth order: each entry's rank among its
        // wave's entries marking block b, then each wave's start per block
        uint32_t pre[kBlocks];
#pragma unroll
        for (int b = 0; b < kBlocks; ++b) {
            const uint64_t bal = __ballot((m >> b) & 1u);
            pre[b] = (uint32_t)__popcll(bal & lanemask_lt());
            if (lane == 0) s_wc[w * kBlocks + b] = (uint32_t)__popcll(bal);
        }
        __syncthreads();
        if (threadIdx.x < kBlocks) {
            uint32_t t = 0;
#pragma unroll
            for (int ww = 0; ww < kNT / kWave; ++ww) {
                const uint32_t c = s_wc[ww * kBlocks + threadIdx.x];
                s_wc[ww * kBlocks + threadIdx.x] = t;
                t += c;
            }
            s_n[threadIdx.x] = t;
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kBlocks; ++b)
            if ((m >> b) & 1u) s_idx[b * BATCH + s_wc[w * kBlocks + b] + pre[b]] = (uint16_t)(j * 16);
        // 3. compositing: pad this block's list with the empty record up to
        // the wave's step count, so every step reads four offsets as they are
        const uint32_t n_mine = s_n[gid];
        const uint32_t n_wave = __builtin_amdgcn_readfirstlane(
            max(max(s_n[w * 4], s_n[w * 4 + 1]), max(s_n[w * 4 + 2], s_n[w * 4 + 3])));
        const uint32_t n_step = (n_wave + 3u) & ~3u;
        uint16_t* list = s_idx + gid * BATCH;
        for (uint32_t p = n_mine + (uint32_t)k; p < n_step; p += 16) list[p] = (uint16_t)(BATCH * 16);
        __syncthreads();
        const uint2* list4 = reinterpret_cast<const uint2*>(list);
        for (uint32_t i = 0; i < n_step; i += 4) {
            const uint2 q4 = list4[i >> 2];
            const uint32_t id4[4] = {q4.x & 0xffffu, q4.x >> 16, q4.y & 0xffffu, q4.y >> 16};
            if (COUNT) neval += 4;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t off = id4[u];
                const StageA A = *reinterpret_cast<const StageA*>(reinterpret_cast<const char*>(s_a) + off);
                const StageB B = *reinterpret_cast<const StageB*>(reinterpret_cast<const char*>(s_b) + off);
                const StageC Cc = *reinterpret_cast<const StageC*>(reinterpret_cast<const char*>(s_c) + off);
                const float t1 = fmaf(A.p, fx, fmaf(A.r, fy, A.c1));
                const float t2 = fmaf(A.s, fy, B.c2);
                const float q = fmaf(t1, t1, t2 * t2);
                const float x = fmaf(q, kNegHalfLog2e, B.lo);
                const float al = fminf(0.99f, __builtin_amdgcn_exp2f(x));
                if (COUNT) nalg += (live && q <= kQMax && i + u < n_mine) ? 1u : 0u;
                const float w0 = al * T;
                const float Tn = T - w0;
                const bool add = live && q <= kQMax && x >= kLog2AlphaMin;
                const bool keep = Tn >= 1e-4f;
                const bool take = add && keep;
                const float wgt = take ? w0 : 0.f;
                C0 = fmaf(wgt, B.col0, C0);
                C1 = fmaf(wgt, Cc.col1, C1);
                C2 = fmaf(wgt, Cc.col2, C2);
                D = fmaf(wgt, B.z, D);
                T = take ? Tn : T;
                if (KEEP) stop_at = (add && !keep) ? (base - rg.x) + (id4[u] >> 4) : stop_at;
                live = live && (keep || !add);
            }
            if (__ballot(live) == 0) break;
        }
        if (__syncthreads_count(live ? 1 : 0) == 0) break;
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
    if (KEEP) {
        const uint32_t L = !inside ? 0u : (stop_at != 0xffffffffu ? stop_at : rg.y - rg.x);
        a.state[(size_t)tile * kNT + threadIdx.x] = make_uint2(L, __float_as_uint(T));
    }
    if (COUNT) {
        const uint32_t sum = wave_sum(nalg);
        if (lane == 0) {
            s_red[2 * w] = sum;
            s_red[2 * w + 1] = neval * kWave;          // uniform per wave
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0, ev = 0;
            for (int i = 0; i < kNT / kWave; ++i) {
                t += s_red[2 * i];
                ev += s_red[2 * i + 1];
            }
            if (t) atomicAdd(&a.ctr->nalg, t);
            if (ev) atomicAdd(&a.ctr->neval, ev);
        }
        __syncthreads();
    }
}

// LDS of one workgroup.
template <int BATCH>
struct Shared {
    StageA a[BATCH + 1];
    StageB b[BATCH + 1];
    StageC c[BATCH + 1];
    alignas(16) uint16_t idx[kBlocks * BATCH];
    uint32_t wc[(kNT / kWave) * kBlocks];
    uint32_t n[kBlocks];
    uint32_t red[2 * (kNT / kWave)];
    uint32_t tile;
};

// Register budget for as many waves per SIMD as the LDS allows (seven
// 256-entry workgroups or eight smaller ones per CU): the staging gathers
// need that many to hide.
template <int BATCH, bool COUNT, bool KEEP>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(BATCH > 128 ? 7 : 8))) void k_composite(CompositeArgs a) {
    __shared__ Shared<BATCH> sh;
    composite_tile<BATCH, COUNT, KEEP>(a, blockIdx.x, sh.a, sh.b, sh.c, sh.idx, sh.wc, sh.n, sh.red);
}

// Persistent variant: a fixed grid takes tiles from a global counter until
// the counter passes the last tile (every workgroup reaches that exit).
template <int BATCH, bool COUNT, bool KEEP>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(BATCH > 128 ? 7 : 8))) void k_composite_persistent(CompositeArgs a) {
    __shared__ Shared<BATCH> sh;
    for (;;) {
        if (threadIdx.x == 0) sh.tile = atomicAdd(&a.ctr->tile_queue, 1u);
        __syncthreads();
        const uint32_t tile = sh.tile;
        __syncthreads();
        if (tile >= a.total_tiles) break;
        composite_tile<BATCH, COUNT, KEEP>(a, tile, sh.a, sh.b, sh.c, sh.idx, sh.wc, sh.n, sh.red);
        __syncthreads();
    }
}

// Counting and keeping pixel states are not combined (the counters are a
// profiling aid): a kept state takes precedence.
template <int BATCH>
void launch_b(const CompositeArgs& a, hipStream_t s) {
    const bool keep = a.state != nullptr;
    if (a.opts.persistent) {
        const uint32_t grid = min(a.total_tiles, 256u * 8u);
        if (keep) k_composite_persistent<BATCH, false, true><<<grid, kNT, 0, s>>>(a);
        else if (a.opts.count_nalg) k_composite_persistent<BATCH, true, false><<<grid, kNT, 0, s>>>(a);
        else k_composite_persistent<BATCH, false, false><<<grid, kNT, 0, s>>>(a);
    } else {
        if (keep) k_composite<BATCH, false, true><<<a.total_tiles, kNT, 0, s>>>(a);
        else if (a.opts.count_nalg) k_composite<BATCH, true, false><<<a.total_tiles, kNT, 0, s>>>(a);
        else k_composite<BATCH, false, false><<<a.total_tiles, kNT, 0, s>>>(a);
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
        default: launch_b<256>(a, s); break;
    }
}

}  // namespace hgs
