// Stable LSD radix sort of 32-bit (key, value) pairs with 8-bit digits, for
// wave64.  Each pass is three launches with no inter-workgroup waiting:
//   upsweep   : each block histograms the digits of its contiguous chunk;
//   row scan  : one block per digit scans that digit's per-block counts;
//   downsweep : each block ranks its chunk stably (ballot digit matching per
//               wave, per-wave counters in LDS) and scatters.
// Element counts live in device memory so the launches can be captured in a
// graph; a block whose chunk is empty exits after writing zeros.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
constexpr int kItems = 8;
constexpr int kSub = kNT * kItems;        // elements per sub-tile
constexpr int kMinChunk = 4096;

__device__ __forceinline__ void chunk_of(uint32_t n, uint32_t cap, int G, int b, uint32_t* lo, uint32_t* hi) {
    n = n < cap ? n : cap;
    uint32_t chunk = ceil_div(n, (uint32_t)G);
    if (chunk < (uint32_t)kMinChunk) chunk = kMinChunk;
    chunk = ceil_div(chunk, (uint32_t)kSub) * kSub;
    uint64_t s = (uint64_t)b * chunk, e = s + chunk;
    if (s > n) s = n;
    if (e > n) e = n;
    *lo = (uint32_t)s;
    *hi = (uint32_t)e;
}

__global__ __launch_bounds__(kNT) void k_upsweep(const uint32_t* __restrict__ keys, const uint32_t* count,
                                                 uint32_t cap, int shift, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    uint32_t lo, hi;
    chunk_of(*count, cap, G, b, &lo, &hi);
    for (uint32_t base = lo; base < hi; base += kNT) {
        const uint32_t i = base + t;
        const bool valid = i < hi;
        const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_digit8(d, act);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[t * G + b] = h[t];   // digit-major
}

// One block per digit: exclusive scan of hist[d][0..G) in place; the digit
// total goes to totals[d].
__global__ __launch_bounds__(1024) void k_rowscan(uint32_t* __restrict__ hist, int G, uint32_t* __restrict__ totals) {
    __shared__ uint32_t sh[1024 / kWave + 1];
    const int d = blockIdx.x, t = threadIdx.x;
    uint32_t* row = hist + (size_t)d * G;
    uint32_t run = 0;
    for (int base = 0; base < G; base += 1024) {
        const int i = base + t;
        const uint32_t x = i < G ? row[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(x, sh, &tot);
        if (i < G) row[i] = run + ex;
        run += tot;
    }
    if (t == 0) totals[d] = run;
}

__global__ __launch_bounds__(kNT) void k_downsweep(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                   const uint32_t* count, uint32_t cap, int shift,
                                                   const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_cnt[kNT / kWave][256];
    __shared__ uint32_t s_scan[kNT / kWave + 1];
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    const int w = t / kWave, l = lane_id();
    uint32_t lo, hi;
    chunk_of(*count, cap, G, b, &lo, &hi);
    if (lo >= hi) return;
    // digit base = exclusive scan of the digit totals, plus this block's
    // exclusive offset within the digit's row
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kNT>(totals[t], s_scan, &tot);
        s_off[t] = ex + hist[t * G + b];
    }
    for (uint32_t base = lo; base < hi; base += kSub) {
#pragma unroll
        for (int k = 0; k < kNT / kWave; ++k) s_cnt[k][t] = 0;
        __syncthreads();
        uint32_t key[kItems], val[kItems], rank[kItems];
        const uint32_t seg = base + (uint32_t)w * (kWave * kItems);
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const uint32_t i = seg + r * kWave + l;
            const bool valid = i < hi;
            key[r] = valid ? kin[i] : 0u;
            val[r] = valid ? vin[i] : 0u;
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint64_t act = __ballot(valid);
            const uint64_t peers = match_digit8(d, act);
            const uint64_t below = peers & lanemask_lt();
            uint32_t before = 0;
            if (valid) before = s_cnt[w][d];
            rank[r] = before + (uint32_t)__popcll(below);
            if (valid && below == 0) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        {
            // per digit t: bases of each wave's run, then advance the digit
            uint32_t run = s_off[t];
#pragma unroll
            for (int k = 0; k < kNT / kWave; ++k) {
                const uint32_t c = s_cnt[k][t];
                s_cnt[k][t] = run;
                run += c;
            }
            s_off[t] = run;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const uint32_t i = seg + r * kWave + l;
            if (i < hi) {
                const uint32_t d = (key[r] >> shift) & 255u;
                const uint32_t pos = s_cnt[w][d] + rank[r];
                kout[pos] = key[r];
                vout[pos] = val[r];
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_sort(const SortArgs& a, hipStream_t s) {
    const int passes = (a.key_bits + 7) / 8;
    const int G = kSortBlocks;
    uint32_t* hist = a.hist;
    uint32_t* totals = a.hist + 256 * G;
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_upsweep<<<G, kNT, 0, s>>>(a.keys[cur], a.count, a.cap, shift, hist);
        k_rowscan<<<256, 1024, 0, s>>>(hist, G, totals);
        k_downsweep<<<G, kNT, 0, s>>>(a.keys[cur], a.vals[cur], a.keys[cur ^ 1], a.vals[cur ^ 1], a.count, a.cap,
                                      shift, hist, totals);
        cur ^= 1;
    }
    return cur;
}

}  // namespace hgs
