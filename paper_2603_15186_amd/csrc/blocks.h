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

constexpr float kLog2AlphaMin = -7.99435343685885793f;   // log2(1/255)

// One staged Gaussian: t1 = p x + r y + c1, t2 = s y + c2 over tile-relative
// pixel centres (x, y); lo = log2(opacity).
struct alignas(16) StageA { float p, r, c1, s; };
struct alignas(16) StageB { float c2, lo, z, col0; };
struct alignas(16) StageC { float col1, col2; };

// Blocks (bit 4 * band + column group) that may hold a pixel centre with
// q <= kQMask.  Per band of four pixel rows, the ellipse's x-extent over the
// band's continuous range of centre heights is found in closed form: for a
// height dy the ellipse spans x = u + (-r dy +- sqrt(Q - (s dy)^2)) / p, and
// the extreme ends over the band sit at its heights nearest to
// dy* = -/+ r sqrt(Q) / (s sqrt(r^2 + s^2)) (the rightmost and leftmost
// points).  The extent covers every row's span, so no block is missed.
__device__ __forceinline__ uint32_t block_mask(float u, float v, float p, float r, float s) {
    const float R = sqrtf(kQMask) / s;
    const float ystar = -r * sqrtf(kQMask) / (s * sqrtf(fmaf(r, r, s * s)));
    const float ip = 1.f / p;
    uint32_t m = 0;
#pragma unroll
    for (int band = 0; band < kTile / 4; ++band) {
        const float y0 = fmaxf((float)(4 * band) + 0.5f - v, -R);
        const float y1 = fminf((float)(4 * band) + 3.5f - v, R);
        const float yr = fminf(fmaxf(ystar, y0), y1), yl = fminf(fmaxf(-ystar, y0), y1);
        const float sr = s * yr, sl = s * yl;
        const float xr = u + (sqrtf(fmaxf(fmaf(-sr, sr, kQMask), 0.f)) - r * yr) * ip;
        const float xl = u - (sqrtf(fmaxf(fmaf(-sl, sl, kQMask), 0.f)) + r * yl) * ip;
        // 1e-3 px absorbs the rounding of this single-precision evaluation
        const int c0 = max(0, (int)ceilf(xl - 0.501f)), c1 = min(kTile - 1, (int)floorf(xr - 0.499f));
        if (y0 <= y1 && c0 <= c1)
            m |= ((2u << ((uint32_t)c1 >> 2)) - (1u << ((uint32_t)c0 >> 2))) << (4 * band);
    }
    return m;
}

}  // namespace hgs
