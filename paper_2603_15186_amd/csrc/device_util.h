// Wave64 and workgroup primitives for gfx950: prefix sums over wavefronts
// and blocks, digit matching by ballots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hgs {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint2 wave_incl_scan2(uint2 x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t a = __shfl_up(x.x, d, kWave);
        uint32_t b = __shfl_up(x.y, d, kWave);
        if (l >= d) { x.x += a; x.y += b; }
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Exclusive scan over a block of NT threads; returns the thread's exclusive
// prefix and writes the block total to *total.  `sh` holds NT/64 + 1 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* sh, uint32_t* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave, l = lane_id();
    uint32_t inc = wave_incl_scan(x);
    if (l == kWave - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; ++i) { uint32_t t = sh[i]; sh[i] = run; run += t; }
        sh[NW] = run;
    }
    __syncthreads();
    uint32_t r = sh[w] + inc - x;
    *total = sh[NW];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ uint2 block_excl_scan2(uint2 x, uint2* sh, uint2* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave, l = lane_id();
    uint2 inc = wave_incl_scan2(x);
    if (l == kWave - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint2 run = make_uint2(0, 0);
        for (int i = 0; i < NW; ++i) {
            uint2 t = sh[i];
            sh[i] = run;
            run.x += t.x; run.y += t.y;
        }
        sh[NW] = run;
    }
    __syncthreads();
    uint2 r = make_uint2(sh[w].x + inc.x - x.x, sh[w].y + inc.y - x.y);
    *total = sh[NW];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ uint4 block_excl_scan4(uint4 x, uint4* sh, uint4* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave, l = lane_id();
    uint4 inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t a = __shfl_up(inc.x, d, kWave), b = __shfl_up(inc.y, d, kWave);
        const uint32_t c = __shfl_up(inc.z, d, kWave), e = __shfl_up(inc.w, d, kWave);
        if (l >= d) { inc.x += a; inc.y += b; inc.z += c; inc.w += e; }
    }
    if (l == kWave - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 run = make_uint4(0, 0, 0, 0);
        for (int i = 0; i < NW; ++i) {
            const uint4 t = sh[i];
            sh[i] = run;
            run.x += t.x; run.y += t.y; run.z += t.z; run.w += t.w;
        }
        sh[NW] = run;
    }
    __syncthreads();
    const uint4 r = make_uint4(sh[w].x + inc.x - x.x, sh[w].y + inc.y - x.y, sh[w].z + inc.z - x.z,
                               sh[w].w + inc.w - x.w);
    *total = sh[NW];
    __syncthreads();
    return r;
}

// Lanes of the wave (among `active`) whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

__host__ __device__ __forceinline__ uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

}  // namespace hgs
