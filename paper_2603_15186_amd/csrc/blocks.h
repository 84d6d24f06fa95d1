// Shared by the compositor and its backward pass: the staged per-entry
// record and the 4x4 pixel blocks of a 16x16 tile an entry's 3-sigma
// ellipse may reach.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace hgs {

constexpr int kBlocks = 16;                 // 4x4-pixel blocks per tile
constexpr float kQMax = 9.f;
constexpr float kQMask = 9.f * 1.001f;      // bound used to mark blocks

// alpha = min(0.99, o e^(-q/2)) = min(0.99, 2^-Q) with
// Q = (kS t1)^2 + (kS t2)^2 - log2(o), kS = sqrt(log2(e) / 2): the conic
// factors are scaled by kS when an entry is staged and -log2(o) is folded
// into a thread's row term, so a pixel needs two FMAs for Q.  An entry adds
// to a pixel only where Q <= entry_qmax: q <= 9 and alpha >= 1/255.
constexpr float kS = 0.84932180028801904f;              // sqrt(log2(e) / 2)
constexpr float kS2 = kS * kS;
constexpr float kQCap = 7.99435343685885793f;           // -log2(1/255)

// The bound on Q of an entry with nlo = -log2(opacity).
__device__ __forceinline__ float entry_qmax(float nlo) { return fminf(kQCap, fmaf(kQMax, kS2, nlo)); }

// One staged Gaussian: t1 = p x + r y + c1, t2 = s y + c2 over tile-relative
// pixel centres (x, y); lo = log2(opacity).
struct alignas(16) StageA { float p, r, c1, s; };
struct alignas(16) StageB { float c2, lo, z, col0; };
struct alignas(16) StageC { float col1, col2; };

// Blocks of a TW x TH tile (TW, TH in {8, 16, 32} x {8, 16}) that may hold
// a pixel centre with q <= kQMask, numbered cell-major: a cell is the tile's
// part within one 16-pixel column of the pixel grid (min(TW, 16) wide),
// blocks row-major inside it.  u, v: the mean relative to the tile origin.
// Per band of four pixel rows, the ellipse's x-extent over the band's
// continuous range of centre heights is found in closed form: for a height
// dy the ellipse spans x = u + (-r dy +- sqrt(Q - (s dy)^2)) / p, and the
// extreme ends over the band sit at its heights nearest to dy* = -/+ r
// sqrt(Q) / (s sqrt(r^2 + s^2)) (the rightmost and leftmost points).  The
// extent covers every row's span, so no block is missed.  A mask only has to
// be a superset of the blocks an entry reaches (an entry listed for a block
// it cannot reach adds nothing there), so the reciprocals and square roots
// are the hardware approximations (a few ulp): the bound's 1e-3 relative
// enlargement and the 1e-3 px edge slack lie far above their error.
template <int TW, int TH>
__device__ __forceinline__ uint32_t block_mask_tile(float u, float v, float p, float r, float s) {
    constexpr int CW = TW < 16 ? TW : 16;           // cell width
    constexpr int CBX = CW / 4;                     // block columns per cell
    constexpr int BPC = CBX * (TH / 4);             // blocks per cell
    constexpr float kSqrtQ = 3.0015f;               // sqrt(kQMask), rounded up
    const float R = kSqrtQ * __builtin_amdgcn_rcpf(s);
    const float ystar = -r * kSqrtQ * __builtin_amdgcn_rcpf(s * __builtin_amdgcn_sqrtf(fmaf(r, r, s * s)));
    const float ip = __builtin_amdgcn_rcpf(p);
    uint32_t m = 0;
#pragma unroll
    for (int band = 0; band < TH / 4; ++band) {
        const float y0 = fmaxf((float)(4 * band) + 0.5f - v, -R);
        const float y1 = fminf((float)(4 * band) + 3.5f - v, R);
        const float yr = fminf(fmaxf(ystar, y0), y1), yl = fminf(fmaxf(-ystar, y0), y1);
        const float sr = s * yr, sl = s * yl;
        const float xr = u + (__builtin_amdgcn_sqrtf(fmaxf(fmaf(-sr, sr, kQMask), 0.f)) - r * yr) * ip;
        const float xl = u - (__builtin_amdgcn_sqrtf(fmaxf(fmaf(-sl, sl, kQMask), 0.f)) + r * yl) * ip;
        const int c0 = max(0, (int)ceilf(xl - 0.501f)), c1 = min(TW - 1, (int)floorf(xr - 0.499f));
        if (y0 <= y1 && c0 <= c1) {
            // block columns c0/4 .. c1/4 of the tile, then split by cell
            const uint32_t cols = (2u << ((uint32_t)c1 >> 2)) - (1u << ((uint32_t)c0 >> 2));
#pragma unroll
            for (int cell = 0; cell < TW / CW; ++cell)
                m |= ((cols >> (cell * CBX)) & ((1u << CBX) - 1u)) << (cell * BPC + band * CBX);
        }
    }
    return m;
}

// The 4x4 blocks of a kTile x kTile tile (bit 4 * band + column group).
__device__ __forceinline__ uint32_t block_mask(float u, float v, float p, float r, float s) {
    return block_mask_tile<kTile, kTile>(u, v, p, r, s);
}

}  // namespace hgs
