// Front-to-back alpha compositing per tile.
//
// One workgroup per TW x TH tile (8x8, 16x8, 16x16, 32x8 or 32x16 pixels),
// TW * TH / PX threads; each thread evaluates PX horizontally adjacent pixels
// of one 4x4 pixel block, the 16 / PX threads of a block sharing the block's
// entries.  The tile's depth-sorted list is walked in batches of BATCH
// entries:
//  1. staging: thread j turns entry j into FP32 records and marks the 4x4
//     blocks holding a pixel centre that its 3-sigma ellipse may reach
//     (closed-form extent per band of four rows, with a relative slack of
//     1e-3 on the bound 9);
//  2. compaction: for every block, the indices of its marked entries in
//     depth order (ballots and prefix counts);
//  3. compositing: the threads of a block walk that block's list; a wave
//     runs to the longest of its blocks' lists and shorter lists are padded
//     with a record that contributes nothing.  The body has no branches:
//       q = t1^2 + t2^2 with t1 = p dx + r dy = p x + (r y + c1) and
//           t2 = s dy = s y + c2 (the bracket and t2 are shared by the
//           pixels of a thread, which lie on one row);
//       Q = q log2(e)/2 - log2(o), alpha = min(0.99, 2^-Q) = min(0.99,
//       o e^(-q/2)), the factors scaled by sqrt(log2(e)/2) when staged and
//       -log2(o) folded into the shared row term (two FMAs per pixel);
//       the entry adds only to a live pixel with Q <= Qmax (q <= 9 and
//       alpha >= 1/255, the cap 0.99 lying above 1/255);
//       T' = T - alpha T; if T' < 1e-4 the pixel stops without adding,
//       else C += c alpha T, D += z alpha T, T = T'.
// A wave leaves its lists once a ballot shows all its pixels stopped, the
// workgroup once a barrier count does.  This is plain FP32 vector arithmetic,
// no matrix cores: the work is a per-pixel recurrence, not a dense
// contraction.
//
// Every pixel's arithmetic is the same for every tile shape, thread count and
// batch depth: its coordinates are taken relative to the corner of the
// 16 x 16 pixel square of the image grid that holds it (a tile 32 pixels wide
// stages its entries for both of its squares), its entries are visited in
// list order, and an entry left out of a block's list cannot reach the
// block's pixels.  Images are therefore bitwise independent of the launch
// shape.
#include "blocks.h"
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

// Launch shape: tile TW x TH pixels, PX pixels per thread.  A "cell" is the
// tile's part inside one 16-pixel-wide column of the image grid: the unit of
// the records' coordinate origin.  Each wave's blocks lie inside one cell.
template <int TW, int TH, int PX>
struct Shape {
    static constexpr int NT = TW * TH / PX;         // threads
    static constexpr int NW = NT / kWave;           // waves
    static constexpr int CW = TW < 16 ? TW : 16;    // cell width
    static constexpr int NC = TW / CW;              // cells
    static constexpr int CBX = CW / 4;              // block columns per cell
    static constexpr int BPC = CBX * (TH / 4);      // blocks per cell
    static constexpr int NB = NC * BPC;             // blocks
    static constexpr int LPB = 16 / PX;             // threads per block
    static constexpr int CPR = 4 / PX;              // threads per block row
    static constexpr int BPW = kWave / LPB;         // blocks per wave
    static_assert(NT % kWave == 0, "whole waves");
    static_assert(BPC % BPW == 0, "a wave's blocks lie in one cell");
    static_assert(NB <= 32, "block masks are 32 bits");
};

// Staged entry, per cell: t1 = p x + r y + c1, t2 = s y + c2 over pixel
// centres relative to the cell's grid corner, all five factors scaled by kS;
// nlo = -log2(opacity); qmax = entry_qmax(nlo).  Shared: the colour.
struct alignas(16) RecA { float p, r, c1, s; };
struct alignas(16) RecB { float c2, nlo, qmax, z; };
struct alignas(16) RecC { float col0, col1, col2; };

template <int TW, int TH, int PX, int BATCH>
struct Shared {
    using S = Shape<TW, TH, PX>;
    RecA a[S::NC][BATCH + 1];
    RecB b[S::NC][BATCH + 1];
    RecC c[BATCH + 1];
    alignas(16) uint16_t idx[S::NB * BATCH];
    uint32_t wc[S::NW * S::NB];
    uint32_t n[S::NB];
    uint32_t red[2 * S::NW];
    uint32_t tile;
};

// Waves per SIMD the kernel is compiled for (its register budget): as many
// as the LDS of one workgroup allows, at most what the shape's registers
// allow without spilling -- per-block list counts (one register per block
// during compaction) and PX pixels of accumulators.
template <int TW, int TH, int PX, int BATCH>
constexpr int waves_per_simd() {
    using S = Shape<TW, TH, PX>;
    constexpr int lds = (int)sizeof(Shared<TW, TH, PX, BATCH>);
    constexpr int wg = (160 * 1024) / lds;
    constexpr int w = wg * S::NW / 4;
    constexpr int regs = S::NB > 16 ? (PX == 4 ? 5 : (PX == 2 ? 6 : 7)) : 8;
    constexpr int c = w < regs ? w : regs;
    return c < 1 ? 1 : c;
}

__global__ void k_ranges_zero(uint2* ranges, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ranges[i] = make_uint2(0, 0);
}

// [first, last + 1) of every tile's run in the grouped pair keys, four keys
// per thread and step (16-byte loads; key arrays start 256-byte aligned).
// A key view << shift | local names the tile tile_base(view) + local of the
// pass; equal keys form one run.
__global__ void k_ranges(const uint32_t* __restrict__ keys, const Counters* ctr, uint32_t cap, uint2* ranges,
                         uint32_t n_tiles, const ViewDev* views, int n_views, int shift) {
    __shared__ uint32_t s_base[kMaxViews];
    for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_base[v] = views[v].tile_base;
    __syncthreads();
    const uint32_t P = min(ctr->pairs, cap);
    const uint32_t lmask = (1u << shift) - 1u;
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
            const bool first = k[j] != kk, last = k[j + 2] != kk;
            if (!first && !last) continue;
            const uint32_t v = kk >> shift;
            if (v >= (uint32_t)n_views) continue;
            const uint32_t t = s_base[v] + (kk & lmask);
            if (t >= n_tiles) continue;
            if (first) ranges[t].x = i0 + j;
            if (last) ranges[t].y = i0 + j + 1;
        }
    }
}

// The compositing walk of one wave over its blocks' lists (cell CELL of the
// records): n_step entries (a multiple of four), `list` this thread's block
// list.  Returns normally when the lists end or every pixel of the wave
// stopped.
template <int TW, int TH, int PX, int BATCH, bool COUNT, bool KEEP, int CELL>
__device__ __forceinline__ void walk(Shared<TW, TH, PX, BATCH>& sh, const uint16_t* list, uint32_t n_step,
                                     uint32_t n_mine, uint32_t pos0, const float (&fx)[PX], float fy, float (&T)[PX],
                                     float (&C0)[PX], float (&C1)[PX], float (&C2)[PX], float (&D)[PX],
                                     bool (&live)[PX], uint32_t& nalg, uint32_t& neval, uint32_t& stop_at) {
    const char* ra = reinterpret_cast<const char*>(sh.a[CELL]);
    const char* rb = reinterpret_cast<const char*>(sh.b[CELL]);
    const char* rc = reinterpret_cast<const char*>(sh.c);
    const uint2* list4 = reinterpret_cast<const uint2*>(list);
    for (uint32_t i = 0; i < n_step; i += 4) {
        const uint2 q4 = list4[i >> 2];
        const uint32_t id4[4] = {q4.x & 0xffffu, q4.x >> 16, q4.y & 0xffffu, q4.y >> 16};
        if (COUNT) neval += 4 * PX;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t off = id4[u];
            const RecA A = *reinterpret_cast<const RecA*>(ra + off);
            const RecB B = *reinterpret_cast<const RecB*>(rb + off);
            const RecC Cc = *reinterpret_cast<const RecC*>(rc + off);
            // shared by the thread's pixels (one row)
            const float ry = fmaf(A.r, fy, A.c1);
            const float t2 = fmaf(A.s, fy, B.c2);
            const float t22 = fmaf(t2, t2, B.nlo);
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                const float t1 = fmaf(A.p, fx[j], ry);
                const float Q = fmaf(t1, t1, t22);
                const float al = fminf(0.99f, __builtin_amdgcn_exp2f(-Q));
                if (COUNT) nalg += (live[j] && Q <= fmaf(kQMax, kS2, B.nlo) && i + u < n_mine) ? 1u : 0u;
                const float w0 = al * T[j];
                const float Tn = T[j] - w0;
                const bool add = live[j] && Q <= B.qmax;
                const bool keep = Tn >= 1e-4f;
                const bool take = add && keep;
                const float wgt = take ? w0 : 0.f;
                C0[j] = fmaf(wgt, Cc.col0, C0[j]);
                C1[j] = fmaf(wgt, Cc.col1, C1[j]);
                C2[j] = fmaf(wgt, Cc.col2, C2[j]);
                D[j] = fmaf(wgt, B.z, D[j]);
                T[j] = take ? Tn : T[j];
                if (KEEP) stop_at = (add && !keep) ? pos0 + (off >> 4) : stop_at;
                live[j] = live[j] && (keep || !add);
            }
        }
        bool any = false;
#pragma unroll
        for (int j = 0; j < PX; ++j) any = any || live[j];
        if (__ballot(any) == 0) break;
    }
}

template <int TW, int TH, int PX, int BATCH, bool COUNT, bool KEEP>
__device__ __forceinline__ void composite_tile(const CompositeArgs& a, uint32_t tile,
                                               Shared<TW, TH, PX, BATCH>& sh) {
    using S = Shape<TW, TH, PX>;
    static_assert(BATCH <= S::NT, "one entry per staging thread");
    static_assert(!KEEP || (TW == kTile && TH == kTile && PX == 1), "kept states use the default launch shape");
    const uint32_t view = a.tile_view[tile];
    const ViewDev& V = a.views[view];
    const uint32_t local = tile - V.tile_base;
    const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
    const int x0 = tx * TW, y0 = ty * TH;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int g = lane / S::LPB, k = lane % S::LPB;
    const int blk = w * S::BPW + g;                     // this thread's block (cell-major)
    const int cell = blk / S::BPC, lb = blk % S::BPC;
    const int wcell = (w * S::BPW) / S::BPC;            // the wave's cell (uniform)
    const int lx0 = cell * S::CW + (lb % S::CBX) * 4 + (k % S::CPR) * PX;
    const int ly = (lb / S::CBX) * 4 + k / S::CPR;
    // grid corner of each cell: x0 rounded down to 16 (plus 16 per cell), y0 likewise
    const int gx0 = x0 & ~15, gy0 = y0 & ~15;
    float fx[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) fx[j] = (float)(x0 + lx0 + j - (gx0 + 16 * cell)) + 0.5f;
    const float fy = (float)(y0 + ly - gy0) + 0.5f;
    const int py = y0 + ly;
    bool inside[PX];
    bool live[PX];
    float T[PX], C0[PX], C1[PX], C2[PX], D[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        inside[j] = x0 + lx0 + j < V.width && py < V.height;
        live[j] = inside[j];
        T[j] = 1.f;
        C0[j] = C1[j] = C2[j] = D[j] = 0.f;
    }
    const uint2 rg = a.ranges[tile];
    uint32_t nalg = 0, neval = 0;
    uint32_t stop_at = 0xffffffffu;                     // list position where the pixel stopped
    if (threadIdx.x == 0) {                             // record that adds nothing
#pragma unroll
        for (int c = 0; c < S::NC; ++c) {
            sh.a[c][BATCH] = RecA{0.f, 0.f, 0.f, 0.f};
            sh.b[c][BATCH] = RecB{0.f, __builtin_inff(), -__builtin_inff(), 0.f};
        }
        sh.c[BATCH] = RecC{0.f, 0.f, 0.f};
    }
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
        const uint32_t cnt = min((uint32_t)BATCH, rg.y - base);
        // 1. staging
        uint32_t m = 0;
        const int j = threadIdx.x;
        if (j < (int)cnt) {
            const uint32_t e = a.vals[base + j];
            const Proj P = a.proj[e < a.cut_cap ? e : 0u];
            const float nlo = -__log2f(P.opacity);
            const float qmax = entry_qmax(nlo);
#pragma unroll
            for (int c = 0; c < S::NC; ++c) {
                const float u = (float)(P.u - (double)(gx0 + 16 * c)), v = (float)(P.v - (double)gy0);
                const float c1 = -fmaf(P.p, u, P.r * v), c2 = -P.s * v;
                sh.a[c][j] = RecA{kS * P.p, kS * P.r, kS * c1, kS * P.s};
                sh.b[c][j] = RecB{kS * c2, nlo, qmax, P.z};
            }
            sh.c[j] = RecC{P.c0, P.c1, P.c2};
            m = block_mask_tile<TW, TH>((float)(P.u - (double)x0), (float)(P.v - (double)y0), P.p, P.r, P.s);
        }
        // 2. per-block lists in depth order: each entry's rank among its
        // wave's entries marking block b, then each wave's start per block
        uint32_t pre[S::NB];
#pragma unroll
        for (int b = 0; b < S::NB; ++b) {
            const uint64_t bal = __ballot((m >> b) & 1u);
            pre[b] = (uint32_t)__popcll(bal & lanemask_lt());
            if (lane == 0) sh.wc[w * S::NB + b] = (uint32_t)__popcll(bal);
        }
        __syncthreads();
        if (threadIdx.x < S::NB) {
            uint32_t t = 0;
#pragma unroll
            for (int ww = 0; ww < S::NW; ++ww) {
                const uint32_t c = sh.wc[ww * S::NB + threadIdx.x];
                sh.wc[ww * S::NB + threadIdx.x] = t;
                t += c;
            }
            sh.n[threadIdx.x] = t;
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < S::NB; ++b)
            if ((m >> b) & 1u) sh.idx[b * BATCH + sh.wc[w * S::NB + b] + pre[b]] = (uint16_t)(j * 16);
        // 3. compositing: pad this block's list with the empty record up to
        // the wave's step count, so every step reads four offsets as they are
        const uint32_t n_mine = sh.n[blk];
        uint32_t n_wave = 0;
#pragma unroll
        for (int b = 0; b < S::BPW; ++b) n_wave = max(n_wave, sh.n[w * S::BPW + b]);
        n_wave = __builtin_amdgcn_readfirstlane(n_wave);
        const uint32_t n_step = (n_wave + 3u) & ~3u;
        uint16_t* list = sh.idx + blk * BATCH;
        for (uint32_t p = n_mine + (uint32_t)k; p < n_step; p += S::LPB) list[p] = (uint16_t)(BATCH * 16);
        __syncthreads();
        if constexpr (S::NC == 1) {
            walk<TW, TH, PX, BATCH, COUNT, KEEP, 0>(sh, list, n_step, n_mine, base - rg.x, fx, fy, T, C0, C1, C2, D,
                                                     live, nalg, neval, stop_at);
        } else if (wcell == 0) {
            walk<TW, TH, PX, BATCH, COUNT, KEEP, 0>(sh, list, n_step, n_mine, base - rg.x, fx, fy, T, C0, C1, C2, D,
                                                     live, nalg, neval, stop_at);
        } else {
            walk<TW, TH, PX, BATCH, COUNT, KEEP, 1>(sh, list, n_step, n_mine, base - rg.x, fx, fy, T, C0, C1, C2, D,
                                                     live, nalg, neval, stop_at);
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < PX; ++q) any = any || live[q];
        if (__syncthreads_count(any ? 1 : 0) == 0) break;
    }
    const size_t plane = (size_t)V.width * V.height;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        if (inside[q]) {
            const size_t o = (size_t)py * V.width + (x0 + lx0 + q);
            V.rgb[o] = C0[q] + T[q] * V.bg[0];
            V.rgb[plane + o] = C1[q] + T[q] * V.bg[1];
            V.rgb[2 * plane + o] = C2[q] + T[q] * V.bg[2];
            if (V.depth) V.depth[o] = D[q];
            if (V.alpha) V.alpha[o] = 1.f - T[q];
        }
    }
    if (KEEP) {
        const uint32_t L = !inside[0] ? 0u : (stop_at != 0xffffffffu ? stop_at : rg.y - rg.x);
        a.state[(size_t)tile * kTilePx + threadIdx.x] = make_uint2(L, __float_as_uint(T[0]));
    }
    if (COUNT) {
        const uint32_t sum = wave_sum(nalg);
        if (lane == 0) {
            sh.red[2 * w] = sum;
            sh.red[2 * w + 1] = neval * kWave;         // uniform per wave
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0, ev = 0;
            for (int i = 0; i < S::NW; ++i) {
                t += sh.red[2 * i];
                ev += sh.red[2 * i + 1];
            }
            if (t) atomicAdd(&a.ctr->nalg, t);
            if (ev) atomicAdd(&a.ctr->neval, ev);
        }
        __syncthreads();
    }
}

// Workgroups go to the eight XCDs in turn, each XCD with its own L2, while
// neighbouring tiles of a view stage many of the same records.  Within each
// full window of kXcdWindow consecutive workgroups, XCD x takes a contiguous
// eighth of the window's tiles; a partial last window keeps the identity.
// A bijection on [0, n).
constexpr uint32_t kXcdWindow = 2048;
static_assert(kXcdWindow % 8 == 0, "eight equal shares per window");
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t r = b % kXcdWindow, w0 = b - r;
    if (n - w0 < kXcdWindow) return b;
    return w0 + (r % 8) * (kXcdWindow / 8) + r / 8;
}

// Register budget for as many waves per SIMD as the LDS allows: the staging
// gathers need that many to hide.
template <int TW, int TH, int PX, int BATCH, bool COUNT, bool KEEP>
__global__ __launch_bounds__(TW * TH / PX) __attribute__((
    amdgpu_waves_per_eu(waves_per_simd<TW, TH, PX, BATCH>()))) void k_composite(CompositeArgs a) {
    __shared__ Shared<TW, TH, PX, BATCH> sh;
    composite_tile<TW, TH, PX, BATCH, COUNT, KEEP>(a, xcd_tile(blockIdx.x, gridDim.x), sh);
}

// Persistent variant (default shape): a fixed grid takes tiles from a global
// counter until the counter passes the last tile (every workgroup reaches
// that exit).
template <int BATCH, bool COUNT, bool KEEP>
__global__ __launch_bounds__(kTilePx) __attribute__((amdgpu_waves_per_eu(BATCH > 128 ? 7 : 8))) void
k_composite_persistent(CompositeArgs a) {
    __shared__ Shared<kTile, kTile, 1, BATCH> sh;
    for (;;) {
        if (threadIdx.x == 0) sh.tile = atomicAdd(&a.ctr->tile_queue, 1u);
        __syncthreads();
        const uint32_t tile = sh.tile;
        __syncthreads();
        if (tile >= a.total_tiles) break;
        composite_tile<kTile, kTile, 1, BATCH, COUNT, KEEP>(a, tile, sh);
        __syncthreads();
    }
}

// One launch shape: the batch depth is capped at the workgroup's thread
// count (one entry per staging thread).
template <int TW, int TH, int PX>
void launch_shape(const CompositeArgs& a, hipStream_t s) {
    constexpr int NT = Shape<TW, TH, PX>::NT;
    const int batch = a.opts.batch < NT ? a.opts.batch : NT;
    const bool count = a.opts.count_nalg;
    const uint32_t grid = a.total_tiles;
#define HGS_COMPOSITE(B)                                                                        \
    do {                                                                                        \
        if constexpr ((B) <= NT) {                                                              \
            if (count) k_composite<TW, TH, PX, (B), true, false><<<grid, NT, 0, s>>>(a);        \
            else k_composite<TW, TH, PX, (B), false, false><<<grid, NT, 0, s>>>(a);             \
        }                                                                                       \
    } while (0)
    if (batch <= 64) HGS_COMPOSITE(64);
    else if (batch <= 128) HGS_COMPOSITE(128);
    else HGS_COMPOSITE(256);
#undef HGS_COMPOSITE
}

// The default shape, also persistent and with kept pixel states.  Counting
// and keeping pixel states are not combined (the counters are a profiling
// aid): a kept state takes precedence.
template <int BATCH>
void launch_default(const CompositeArgs& a, hipStream_t s) {
    const bool keep = a.state != nullptr;
    if (a.opts.persistent) {
        const uint32_t grid = min(a.total_tiles, 256u * 8u);
        if (keep) k_composite_persistent<BATCH, false, true><<<grid, kTilePx, 0, s>>>(a);
        else if (a.opts.count_nalg) k_composite_persistent<BATCH, true, false><<<grid, kTilePx, 0, s>>>(a);
        else k_composite_persistent<BATCH, false, false><<<grid, kTilePx, 0, s>>>(a);
    } else {
        if (keep) k_composite<kTile, kTile, 1, BATCH, false, true><<<a.total_tiles, kTilePx, 0, s>>>(a);
        else if (a.opts.count_nalg) k_composite<kTile, kTile, 1, BATCH, true, false><<<a.total_tiles, kTilePx, 0, s>>>(a);
        else k_composite<kTile, kTile, 1, BATCH, false, false><<<a.total_tiles, kTilePx, 0, s>>>(a);
    }
}

}  // namespace

bool tile_shape_ok(int tw, int th, int px) {
    const bool shape = (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) ||
                       (tw == 32 && th == 8) || (tw == 32 && th == 16);
    // a wave's blocks must lie in one 16-pixel column of the tile: 32x8
    // tiles hold only 8 blocks per column, a 4-pixel thread's wave 16
    return shape && (px == 1 || px == 2 || px == 4) && (tw * th) / px >= 64 && !(tw == 32 && th == 8 && px == 4);
}

void launch_ranges(const CompositeArgs& a, hipStream_t s) {
    k_ranges_zero<<<1024, 256, 0, s>>>(a.ranges, a.total_tiles);
    k_ranges<<<4096, 256, 0, s>>>(a.keys, a.ctr, a.pair_cap, a.ranges, a.total_tiles, a.views, a.n_views,
                                  a.key_shift);
}

void launch_composite(const CompositeArgs& a, hipStream_t s) {
    if (a.total_tiles == 0) return;
    const int tw = a.opts.tile_w, th = a.opts.tile_h, px = a.opts.px;
    // kept pixel states and the persistent queue use the default shape
    // (tiles of kTile x kTile, as binned; one pixel per thread)
    if (tw == kTile && th == kTile && (px == 1 || a.state != nullptr || a.opts.persistent)) {
        switch (a.opts.batch) {
            case 64: launch_default<64>(a, s); break;
            case 128: launch_default<128>(a, s); break;
            default: launch_default<256>(a, s); break;
        }
        return;
    }
    if (tw == 8 && th == 8) launch_shape<8, 8, 1>(a, s);
    else if (tw == 16 && th == 8) {
        if (px == 2) launch_shape<16, 8, 2>(a, s);
        else launch_shape<16, 8, 1>(a, s);
    } else if (tw == 16 && th == 16) {
        if (px == 4) launch_shape<16, 16, 4>(a, s);
        else launch_shape<16, 16, 2>(a, s);
    } else if (tw == 32 && th == 8) {
        if (px == 2) launch_shape<32, 8, 2>(a, s);
        else launch_shape<32, 8, 1>(a, s);
    } else {
        if (px == 4) launch_shape<32, 16, 4>(a, s);
        else if (px == 2) launch_shape<32, 16, 2>(a, s);
        else launch_shape<32, 16, 1>(a, s);
    }
}

}  // namespace hgs
