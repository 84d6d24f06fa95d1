// Stable LSD radix sort of 32-bit (key, value) pairs for wave64.
//
// A sort over `bits` key bits runs ceil(bits / D) passes with digits of
// ceil(bits / passes) bits, D the widest digit allowed (6..11: up to 2048
// buckets), so a 17-bit tile key takes two or three passes and a 32-bit depth
// key three to six.  The input is cut into at most kSortMaxGroups groups, each
// the smallest multiple of kSortGroup elements that keeps their number in that
// bound; a workgroup takes groups b, b + G, b + 2G, ... so that the groups in flight
// at any moment form one contiguous window of the input and each digit's
// output advances as one front (writes of neighbouring groups land next to
// each other and fill whole cache lines).  Each pass is three launches with
// no inter-workgroup waiting:
//   upsweep   : the digit histogram of every group (LDS atomics into
//               per-wave histograms), digit-major;
//   row scan  : one block per digit scans that digit's per-group counts;
//   downsweep : each group is ranked stably sub-tile by sub-tile -- lanes
//               with equal digits are found by ballots over the digit bits,
//               per-wave counters live in LDS -- and its keys and values are
//               scattered.
// Element counts live in device memory so the launches can be captured in a
// graph.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
constexpr int kNW = kNT / kWave;
static_assert(kSortGroup % (kNT * 16) == 0, "a group holds whole sub-tiles of every width");

__device__ __forceinline__ uint32_t n_of(const uint32_t* count, uint32_t cap) {
    const uint32_t n = *count;
    return n < cap ? n : cap;
}

// Elements per histogram group of an n-element sort (a multiple of
// kSortGroup; at most kSortMaxGroups groups).
__device__ __forceinline__ uint32_t group_size(uint32_t n) {
    const uint32_t per = ceil_div(n, (uint32_t)kSortGroup * (uint32_t)kSortMaxGroups);
    return (per > 1u ? per : 1u) * (uint32_t)kSortGroup;
}

// Lanes of the wave (among `active`) whose DB-bit digit equals this lane's.
template <int DB>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < DB; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

// Digit histogram of every group the block owns: per-wave LDS histograms
// take one atomic add per key (counts do not depend on order), four keys per
// thread and step with 16-byte loads (groups start at multiples of
// kSortGroup).
template <int DB>
__global__ __launch_bounds__(kNT) void k_upsweep(const uint32_t* __restrict__ keys, const uint32_t* count,
                                                 uint32_t cap, int shift, uint32_t MASK, uint32_t* __restrict__ hist,
                                                 uint32_t stride) {
    constexpr int NB = 1 << DB;
    __shared__ uint32_t h[kNW][NB];
    const int t = threadIdx.x;
    uint32_t* hw = h[t / kWave];
    const uint32_t n = n_of(count, cap);
    const uint32_t gs = group_size(n), ng = ceil_div(n, gs);
    for (uint32_t g = blockIdx.x; g < ng; g += gridDim.x) {
        for (int i = t; i < NB; i += kNT) {
#pragma unroll
            for (int w = 0; w < kNW; ++w) h[w][i] = 0;
        }
        __syncthreads();
        const uint32_t lo = g * gs;
        const uint32_t hi = min(lo + gs, n);
        uint32_t base = lo;
        for (; base + 4 * kNT <= hi; base += 4 * kNT) {
            const uint4 k4 = *reinterpret_cast<const uint4*>(keys + base + 4 * t);
            atomicAdd(&hw[(k4.x >> shift) & MASK], 1u);
            atomicAdd(&hw[(k4.y >> shift) & MASK], 1u);
            atomicAdd(&hw[(k4.z >> shift) & MASK], 1u);
            atomicAdd(&hw[(k4.w >> shift) & MASK], 1u);
        }
        for (uint32_t i = base + t; i < hi; i += kNT) atomicAdd(&hw[(keys[i] >> shift) & MASK], 1u);
        __syncthreads();
        for (int i = t; i < NB; i += kNT) {
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < kNW; ++w) c += h[w][i];
            hist[(size_t)i * stride + g] = c;   // digit-major
        }
        __syncthreads();
    }
}

// One block per digit: exclusive scan of the digit's per-group counts
// hist[d][0..groups) in place; the digit total goes to totals[d].
__global__ __launch_bounds__(1024) void k_rowscan(uint32_t* __restrict__ hist, const uint32_t* count, uint32_t cap,
                                                  uint32_t stride, uint32_t* __restrict__ totals) {
    __shared__ uint32_t sh[1024 / kWave + 1];
    const int d = blockIdx.x, t = threadIdx.x;
    const uint32_t n = n_of(count, cap);
    const uint32_t ng = ceil_div(n, group_size(n));
    uint32_t* row = hist + (size_t)d * stride;
    uint32_t run = 0;
    for (uint32_t base = 0; base < ng; base += 1024) {
        const uint32_t i = base + (uint32_t)t;
        const uint32_t x = i < ng ? row[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(x, sh, &tot);
        if (i < ng) row[i] = run + ex;
        run += tot;
    }
    if (t == 0) totals[d] = run;
}

// Downsweep with a local reorder: each sub-tile of kItems * kNT elements is
// ranked (stable within the sub-tile), placed in LDS in digit order, then
// written out in that order so that consecutive lanes store consecutive
// addresses of one digit's run.
template <int DB, int ITEMS>
__global__ __launch_bounds__(kNT) void k_downsweep(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                   const uint32_t* count, uint32_t cap, int shift, uint32_t MASK,
                                                   const uint32_t* __restrict__ hist, uint32_t stride,
                                                   const uint32_t* __restrict__ totals) {
    constexpr int NB = 1 << DB;
    constexpr int PER = NB / kNT > 0 ? NB / kNT : 1;      // digits per thread
    constexpr int SUB = kNT * ITEMS;
    static_assert(kSortGroup % SUB == 0, "whole sub-tiles per group");
    __shared__ uint32_t s_start[NB];                     // first output position of digit d
    __shared__ uint32_t s_off[NB];                       // global position of the next element of digit d
    __shared__ uint32_t s_loc[NB];                       // start of digit d inside the staged sub-tile
    __shared__ uint32_t s_cnt[kNW][NB];
    __shared__ uint32_t s_scan[kNW + 1];
    __shared__ uint32_t s_key[SUB];
    __shared__ uint32_t s_val[SUB];
    const int t = threadIdx.x;
    const int w = t / kWave, l = lane_id();
    const uint32_t n = n_of(count, cap);
    const uint32_t gs = group_size(n), ng = ceil_div(n, gs);
    if (blockIdx.x >= ng) return;
    {
        uint32_t mine[PER];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int d = t * PER + k;
            mine[k] = d < NB ? totals[d] : 0u;
            sum += mine[k];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan<kNT>(sum, s_scan, &tot);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int d = t * PER + k;
            if (d < NB) s_start[d] = ex;
            ex += mine[k];
        }
    }
    for (uint32_t g = blockIdx.x; g < ng; g += gridDim.x) {
        __syncthreads();
        for (int d = t; d < NB; d += kNT) s_off[d] = s_start[d] + hist[(size_t)d * stride + g];
        const uint32_t lo = g * gs;
        const uint32_t hi = min(lo + gs, n);
        for (uint32_t base = lo; base < hi; base += SUB) {
            for (int i = t; i < NB; i += kNT) {
#pragma unroll
                for (int k = 0; k < kNW; ++k) s_cnt[k][i] = 0;
            }
            __syncthreads();
            uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
            const uint32_t seg = base + (uint32_t)w * (kWave * ITEMS);
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t i = seg + r * kWave + l;
                const bool valid = i < hi;
                key[r] = valid ? kin[i] : 0u;
                val[r] = valid ? vin[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t i = seg + r * kWave + l;
                const bool valid = i < hi;
                const uint32_t d = (key[r] >> shift) & MASK;
                const uint64_t act = __ballot(valid);
                const uint64_t peers = match_digit<DB>(d, act);
                const uint64_t below = peers & lanemask_lt();
                uint32_t before = 0;
                if (valid) before = s_cnt[w][d];
                rank[r] = before + (uint32_t)__popcll(below);
                if (valid && below == 0) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
            }
            __syncthreads();
            // per digit: local start of each wave's run inside the sub-tile
            {
                uint32_t mine[PER];
                uint32_t sum = 0;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int d = t * PER + k;
                    uint32_t c = 0;
                    if (d < NB) {
#pragma unroll
                        for (int q = 0; q < kNW; ++q) c += s_cnt[q][d];
                    }
                    mine[k] = c;
                    sum += c;
                }
                uint32_t tot;
                uint32_t ex = block_excl_scan<kNT>(sum, s_scan, &tot);
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int d = t * PER + k;
                    if (d < NB) {
                        s_loc[d] = ex;
                        uint32_t run = ex;
#pragma unroll
                        for (int q = 0; q < kNW; ++q) {
                            const uint32_t c = s_cnt[q][d];
                            s_cnt[q][d] = run;
                            run += c;
                        }
                    }
                    ex += mine[k];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t i = seg + r * kWave + l;
                if (i < hi) {
                    const uint32_t d = (key[r] >> shift) & MASK;
                    const uint32_t p = s_cnt[w][d] + rank[r];
                    s_key[p] = key[r];
                    s_val[p] = val[r];
                }
            }
            __syncthreads();
            const uint32_t n_sub = (hi - base) < (uint32_t)SUB ? (hi - base) : (uint32_t)SUB;
            for (uint32_t p = t; p < n_sub; p += kNT) {
                const uint32_t k = s_key[p];
                const uint32_t d = (k >> shift) & MASK;
                const uint32_t pos = s_off[d] + (p - s_loc[d]);
                kout[pos] = k;
                vout[pos] = s_val[p];
            }
            __syncthreads();
            // advance each digit's global position by its count in this sub-tile
            for (int d = t; d < NB; d += kNT) {
                const uint32_t next = (d + 1 < NB) ? s_loc[d + 1] : n_sub;
                s_off[d] += next - s_loc[d];
            }
            __syncthreads();
        }
    }
}

// One pass over digit bits [shift, shift + nbits) (nbits <= DB).
template <int DB>
void pass(const SortArgs& a, int cur, int shift, int nbits, hipStream_t s) {
    const int G = kSortBlocks;
    const uint32_t stride = a.hist_stride;
    uint32_t* hist = a.hist;
    uint32_t* totals = a.hist + (size_t)kSortBins * stride;
    const uint32_t mask = nbits >= 32 ? 0xffffffffu : ((1u << nbits) - 1u);
    k_upsweep<DB><<<G, kNT, 0, s>>>(a.keys[cur], a.count, a.cap, shift, mask, hist, stride);
    k_rowscan<<<1 << DB, 1024, 0, s>>>(hist, a.count, a.cap, stride, totals);
    constexpr int ITEMS = DB <= 8 ? 16 : 8;
    k_downsweep<DB, ITEMS><<<G, kNT, 0, s>>>(a.keys[cur], a.vals[cur], a.keys[cur ^ 1], a.vals[cur ^ 1], a.count,
                                             a.cap, shift, mask, hist, stride, totals);
}

}  // namespace

int launch_sort(const SortArgs& a, hipStream_t s) {
    const int maxdb = a.max_digit_bits < 6 ? 6 : (a.max_digit_bits > 11 ? 11 : a.max_digit_bits);
    const int passes = (a.key_bits + maxdb - 1) / maxdb;
    const int db = (a.key_bits + passes - 1) / passes;
    int cur = 0, shift = 0;
    for (int p = 0; p < passes; ++p) {
        // the last pass may cover fewer bits: its mask drops key bits above key_bits
        const int nbits = a.key_bits - shift < db ? a.key_bits - shift : db;
        switch (db) {
            case 1: case 2: case 3: case 4: case 5: case 6: pass<6>(a, cur, shift, nbits, s); break;
            case 7: pass<7>(a, cur, shift, nbits, s); break;
            case 8: pass<8>(a, cur, shift, nbits, s); break;
            case 9: pass<9>(a, cur, shift, nbits, s); break;
            case 10: pass<10>(a, cur, shift, nbits, s); break;
            default: pass<11>(a, cur, shift, nbits, s); break;
        }
        shift += db;
        cur ^= 1;
    }
    return cur;
}

}  // namespace hgs
