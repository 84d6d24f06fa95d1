// Shortest-path planning on the collision map (the navigable areas of Sec.
// III-C serve collision checks and path planning; expert trajectories come
// from a shortest-path planner, Sec. IV):
//
//   * navigable map: a cell is navigable when a disc robot centred on it
//     meets no occupied cell;
//   * distance fields: per goal cell, the least cost of an 8-connected path
//     (orthogonal move 1, diagonal move sqrt 2, a diagonal move only between
//     two navigable side cells) from every cell, kept as the pair (a, b) of
//     orthogonal and diagonal moves of such a path, which is unique since
//     sqrt 2 is irrational.  Pairs are ordered by their FP64 costs, which
//     is exact for grids of up to 2^24 cells (see pair_cost);
//   * trajectories: from a start cell, repeatedly the first neighbour in the
//     order E, W, S, N, SE, SW, NE, NW whose pair plus the move's unit equals
//     the current pair, until the goal.  That neighbour is found once per
//     cell and field (a byte per cell), so a trajectory is a chain of byte
//     loads.
//
// The distance field is computed by tiled relaxation: the grid is split
// into 32 x 32 tiles; in each round every tile whose 3 x 3 neighbourhood
// changed in the previous round loads itself and a one-cell halo into LDS
// and relaxes its cells to a local fixed point by directional sweeps (see
// k_dist_round), then writes back what improved.  Relaxation only lowers pairs toward the
// exact distances, so the result does not depend on the order of rounds,
// tiles or threads; the host repeats rounds until one changes nothing.
#include "device_util.h"
#include "grid.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
constexpr int kT = 32;                     // tile edge (cells)
constexpr int kH = kT + 2;                 // tile with its halo
constexpr uint64_t kUnreached = ~0ull;
constexpr uint64_t kOrth = 1ull;           // (a, b) packed a | b << 32
constexpr uint64_t kDiag = 1ull << 32;
constexpr double kSqrt2 = 1.4142135623730951;

// Offsets of move m in the order E, W, S, N, SE, SW, NE, NW (x to the
// right, y down the rows), from 2-bit fields of an immediate offset by one:
// a per-lane move index then costs no memory access.
__device__ __forceinline__ int step_dx(uint32_t m) { return (int)((0x2252u >> (2 * m)) & 3u) - 1; }
__device__ __forceinline__ int step_dy(uint32_t m) { return (int)((0x0A25u >> (2 * m)) & 3u) - 1; }

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kNT) void k_navigable(NavArgs a) {
    const int64_t N = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)kNT + threadIdx.x; c < N; c += (int64_t)gridDim.x * kNT) {
        const int i = (int)(c % a.nx), j = (int)(c / a.nx);
        double x, y;
        {
#pragma clang fp contract(off)
            x = a.x0 + ((double)i + 0.5) * a.cell;
            y = a.y0 + ((double)j + 0.5) * a.cell;
        }
        a.nav[c] = disc_hits(a.map, a.x0, a.y0, a.cell, a.nx, a.ny, x, y, a.radius) ? 0 : 1;
    }
}

// Fields start unreached except valid goals (navigable cells in the grid),
// whose tiles are the active set of round 0.
__global__ __launch_bounds__(kNT) void k_dist_init(DistArgs d) {
    const int64_t N = (int64_t)d.nx * d.ny;
    const int64_t tiles = (int64_t)d.tiles_x * d.tiles_y;
    const int64_t total = N * d.n_goals;
    for (int64_t k = blockIdx.x * (int64_t)kNT + threadIdx.x; k < total; k += (int64_t)gridDim.x * kNT) {
        const int64_t g = k / N, c = k % N;
        const int32_t goal = d.goals[g];
        const bool ok = goal >= 0 && goal < N && d.nav[goal] != 0;
        d.dist[k] = (ok && c == goal) ? 0ull : kUnreached;
    }
    for (int64_t k = blockIdx.x * (int64_t)kNT + threadIdx.x; k < tiles * d.n_goals; k += (int64_t)gridDim.x * kNT) {
        const int64_t g = k / tiles, t = k % tiles;
        const int32_t goal = d.goals[g];
        const bool ok = goal >= 0 && goal < N && d.nav[goal] != 0;
        const int64_t gt = ok ? (int64_t)((goal / d.nx) / kT) * d.tiles_x + (goal % d.nx) / kT : -1;
        d.flags[0][k] = t == gt ? 1 : 0;
        d.flags[1][k] = 0;
    }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0;
}

// Cost a + b sqrt 2 of a reached pair, rounded once (within 2^-28 of the
// exact value for a + b < 2^24).  For grids of at most 2^24 cells two
// different pairs differ in cost by at least 1 / (2 sqrt 2 |db| + 1) > 2e-8
// (|da^2 - 2 db^2| >= 1), so comparing these costs orders pairs exactly and
// equal pairs have equal costs.
__device__ __forceinline__ double pair_cost(uint64_t p) {
    return fma((double)(uint32_t)(p >> 32), kSqrt2, (double)(uint32_t)p);
}

// One round: block (tile, group of kGW goals), one wave per goal.  The
// tile's navigability and each interior cell's legal moves are shared by
// the goals; each wave loads its goal's tile and halo into LDS and relaxes
// it to a local fixed point by directional sweeps: in the x phase lanes
// 0-31 sweep the 32 rows eastward and lanes 32-63 westward, each step
// relaxing a column's cells from the column behind (orthogonal and both
// diagonals), so a value crosses the tile in one sweep; the y phase does
// the same for the columns southward and northward.  Lanes of one wave run
// in step, so a cell is written by at most one lane per step and every
// write is a minimum over values read at that step: relaxation stays
// monotone.  The wave stops after two phases in a row that change nothing.
constexpr int kGW = kNT / kWave;           // goals per workgroup

struct DistShared {
    uint64_t d[kGW][kH * kH];              // pairs, one 64-bit LDS access each
    uint8_t nav[kH * kH];
    uint8_t mv[kH * kH];                   // legal moves of interior cells
};

// Best of a cell's pair cur and the candidates from the three cells behind
// it (pairs v0 orthogonal, v1 and v2 diagonal, legal when move bits b0..b2
// of its mask m are set and the cell is reached).  An illegal candidate
// costs infinity, so its pair (which may have wrapped) is never chosen.
// The cheaper of (cur, c0) and of (c1, c2) are found side by side, then the
// cheaper of the two: equal costs mean equal pairs, so the grouping of the
// tests does not change the pair returned.
__device__ __forceinline__ uint64_t relax_pair(uint64_t cur, uint32_t m, uint64_t v0, int b0, uint64_t v1, int b1,
                                               uint64_t v2, int b2) {
    const double inf = __builtin_huge_val();
    const uint64_t c0 = v0 + kOrth, c1 = v1 + kDiag, c2 = v2 + kDiag;
    const double kc = cur == kUnreached ? inf : pair_cost(cur);
    const double k0 = ((m >> b0) & 1u) && v0 != kUnreached ? pair_cost(c0) : inf;
    const double k1 = ((m >> b1) & 1u) && v1 != kUnreached ? pair_cost(c1) : inf;
    const double k2 = ((m >> b2) & 1u) && v2 != kUnreached ? pair_cost(c2) : inf;
    const bool t0 = k0 < kc, t1 = k2 < k1;
    const uint64_t p01 = t0 ? c0 : cur, p12 = t1 ? c2 : c1;
    const double q01 = t0 ? k0 : kc, q12 = t1 ? k2 : k1;
    return q12 < q01 ? p12 : p01;
}

// The value of lane l - 1 (from_below) or l + 1 (from_above) in the wave;
// lanes 0 and 63 receive zero.
__device__ __forceinline__ uint64_t from_below(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x138, 0xf, 0xf, false);   // wave_shr:1
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x138, 0xf, 0xf, false);
    return (uint64_t)hi << 32 | lo;
}
__device__ __forceinline__ uint64_t from_above(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x130, 0xf, 0xf, false);   // wave_shl:1
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x130, 0xf, 0xf, false);
    return (uint64_t)hi << 32 | lo;
}

// One phase of a wave's sweeps over its tile: lane li (1..kT) walks line li
// (cells li*A + x*L, x = 1..kT), lanes 0-31 forward and 32-63 backward, and
// relaxes each cell from the three cells one step behind (o0 on its line,
// o1 and o2 on lines li - 1 and li + 1).  This lane and its neighbours in
// the wave wrote those three at the step before, so their pairs come from
// registers (lane shifts) rather than from LDS; lines 1 and kT take their
// outer one from the halo, as does every lane at the first step.  A cell's
// own pair is read ahead of its step: the lanes sweeping the other way
// reach the cells of a lane's first half only after it has passed them
// (from their step kT/2 on) and write those of its second half only before
// it gets there (in their first kT/2 steps), so once the second half's
// reads follow the first half's writes, every pair used equals what a read
// at the step itself would return, and storing a cell's pair unchanged
// overwrites nothing newer.  Returns whether the lane changed a cell.
template <int L, int A>
__device__ __forceinline__ bool sweep(uint64_t* sd, const uint8_t* mv, int li, int fwd, int x0, int b0, int b1,
                                      int b2) {
    constexpr int kHalf = kT / 2, kChunk = 4, kChunks = kHalf / kChunk;
    int q0 = li * A + x0 * L, dq = fwd * L;
    // formed anew at every call: nothing derived from them is hoisted out
    // of the caller's loop over phases to stay live in registers
    __asm__ volatile("" : "+v"(q0), "+v"(dq));
    const int o0 = -dq, o1 = -A - dq, o2 = A - dq;
    const int ob = li == 1 ? o1 : o2;
    // The reads of a half go out one chunk of steps ahead of their use; the
    // (compiler-only) fences keep later chunks from being hoisted into the
    // registers, and the second half's reads after the first half's writes.
    __asm__ volatile("" ::: "memory");
    uint64_t best = sd[q0 + o0];
    const uint64_t up0 = sd[q0 + o1], dn0 = sd[q0 + o2];
    bool ch = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint64_t cur[2][kChunk], hal[2][kChunk];
        uint32_t m[2][kChunk];
        int qb[2];
        auto load = [&](int c) {
            // the chunk's first cell, opaque to the compiler so that it
            // forms the chunk's addresses then instead of keeping every
            // step's address in a register from the start
            qb[c & 1] = q0 + dq * (h * kHalf + c * kChunk);
            __asm__ volatile("" : "+v"(qb[c & 1]));
#pragma unroll
            for (int s = 0; s < kChunk; ++s) {
                const int q = qb[c & 1] + dq * s;
                cur[c & 1][s] = sd[q];
                hal[c & 1][s] = sd[q + ob];
                m[c & 1][s] = mv[q];
            }
        };
        __asm__ volatile("" ::: "memory");
        load(0);
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            __asm__ volatile("" ::: "memory");
            if (c + 1 < kChunks) load(c + 1);
#pragma unroll
            for (int s = 0; s < kChunk; ++s) {
                const int st = h * kHalf + c * kChunk + s;
                uint64_t v1 = up0, v2 = dn0;
                if (st > 0) {
                    const uint64_t lb = from_below(best), la = from_above(best);
                    v1 = li == 1 ? hal[c & 1][s] : lb;
                    v2 = li == kT ? hal[c & 1][s] : la;
                }
                const uint64_t nb = relax_pair(cur[c & 1][s], m[c & 1][s], best, b0, v1, b1, v2, b2);
                sd[qb[c & 1] + dq * s] = nb;
                ch |= nb != cur[c & 1][s];
                best = nb;
            }
        }
        __asm__ volatile("" ::: "memory");
    }
    return ch;
}

__global__ __launch_bounds__(kNT) void k_dist_round(DistArgs d, int round, int slot) {
    // After a round of the batch that changed no tile the fields are
    // settled: the rest of the batch returns at once (its counts stay zero,
    // and the host stops at the first zero count, so the tile flags these
    // rounds leave as they were are never read).
    if (slot > 0 && d.active[slot - 1] == 0) return;
    __shared__ DistShared S;
    const int t = blockIdx.x;
    const int tx = t % d.tiles_x, ty = t / d.tiles_x;
    const int64_t tiles = (int64_t)d.tiles_x * d.tiles_y;
    const int gx0 = tx * kT - 1, gy0 = ty * kT - 1;
    for (int k = threadIdx.x; k < kH * kH; k += kNT) {
        const int gx = gx0 + k % kH, gy = gy0 + k / kH;
        const bool in = gx >= 0 && gy >= 0 && gx < d.nx && gy < d.ny;
        S.nav[k] = (in && d.nav[(size_t)gy * d.nx + gx] != 0) ? 1 : 0;
    }
    __syncthreads();
    // bit m: move m of E, W, S, N, SE, SW, NE, NW leads to a navigable
    // cell (diagonals between navigable side cells)
    for (int k = threadIdx.x; k < kH * kH; k += kNT) {
        const int lx = k % kH, ly = k / kH;
        uint32_t m = 0;
        if (lx >= 1 && lx <= kT && ly >= 1 && ly <= kT && S.nav[k]) {
            const bool e = S.nav[k + 1], w = S.nav[k - 1], so = S.nav[k + kH], no = S.nav[k - kH];
            m = (e ? 1u : 0u) | (w ? 2u : 0u) | (so ? 4u : 0u) | (no ? 8u : 0u);
            if (e && so && S.nav[k + kH + 1]) m |= 16u;
            if (w && so && S.nav[k + kH - 1]) m |= 32u;
            if (e && no && S.nav[k - kH + 1]) m |= 64u;
            if (w && no && S.nav[k - kH - 1]) m |= 128u;
        }
        S.mv[k] = (uint8_t)m;
    }
    __syncthreads();
    // from here each wave works alone on its goal
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int g = blockIdx.y * kGW + w;
    if (g >= d.n_goals) return;
    const uint8_t* prev = d.flags[round & 1] + g * tiles;
    uint8_t* next = d.flags[(round + 1) & 1] + g * tiles;
    int act = 0;
    for (int v = max(ty - 1, 0); v <= min(ty + 1, d.tiles_y - 1); ++v)
        for (int u = max(tx - 1, 0); u <= min(tx + 1, d.tiles_x - 1); ++u) act |= prev[v * d.tiles_x + u];
    if (!act) {
        if (lane == 0) next[t] = 0;
        return;
    }
    uint64_t* D = d.dist + (size_t)g * d.nx * d.ny;
    uint64_t* sd = S.d[w];
    // all of a lane's loads in flight together, then the LDS stores
    constexpr int kLoads = (kH * kH + kWave - 1) / kWave;
    uint64_t ld[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
        const int k = lane + j * kWave;
        const int gx = gx0 + k % kH, gy = gy0 + k / kH;
        const bool in = k < kH * kH && gx >= 0 && gy >= 0 && gx < d.nx && gy < d.ny;
        ld[j] = in ? load_relaxed(D + (size_t)gy * d.nx + gx) : kUnreached;
    }
#pragma unroll
    for (int j = 0; j < kLoads; ++j)
        if (lane + j * kWave < kH * kH) sd[lane + j * kWave] = ld[j];
    // lanes 0-31 sweep east / south, lanes 32-63 west / north; li is the
    // lane's row (x phase) or column (y phase), 1..32
    const int fwd = lane < 32 ? 1 : -1, li = (lane & 31) + 1;
    const int x0 = fwd > 0 ? 1 : kT;
    // move bits of the cells behind: W, NW, SW (east) or E, NE, SE (west);
    // N, NW, NE (south) or S, SW, SE (north)
    const int xb0 = fwd > 0 ? 1 : 0, xb1 = fwd > 0 ? 7 : 6, xb2 = fwd > 0 ? 5 : 4;
    const int yb0 = fwd > 0 ? 3 : 2, yb1 = fwd > 0 ? 7 : 5, yb2 = fwd > 0 ? 6 : 4;
    // An x phase that changes nothing leaves every cell relaxed over E, W
    // and the four diagonals, a y phase over N, S and the diagonals: two
    // phases in a row that change nothing, in either order, mark a fixed
    // point over all eight moves.
    bool any = false;
    for (int quiet = 0, ph = 0; quiet < 2; ph ^= 1) {
        const bool ch = ph == 0 ? sweep<1, kH>(sd, S.mv, li, fwd, x0, xb0, xb1, xb2)
                                : sweep<kH, 1>(sd, S.mv, li, fwd, x0, yb0, yb1, yb2);
        any |= ch;
        quiet = __ballot(ch) ? 0 : quiet + 1;
    }
    bool wrote = false;
    if (__ballot(any)) {
        constexpr int kCells = kT * kT / kWave;
        uint64_t old[kCells];
#pragma unroll
        for (int j = 0; j < kCells; ++j) {
            const int k = lane + j * kWave;
            const int gx = gx0 + k % kT + 1, gy = gy0 + k / kT + 1;
            old[j] = gx < d.nx && gy < d.ny ? load_relaxed(D + (size_t)gy * d.nx + gx) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kCells; ++j) {
            const int k = lane + j * kWave;
            const int q = (k / kT + 1) * kH + k % kT + 1;
            const int gx = gx0 + k % kT + 1, gy = gy0 + k / kT + 1;
            const uint64_t v = sd[q];
            if (gx < d.nx && gy < d.ny && v != old[j]) {
                store_relaxed(D + (size_t)gy * d.nx + gx, v);
                wrote = true;
            }
        }
    }
    const bool blk = __ballot(wrote) != 0;
    if (lane == 0) {
        next[t] = blk ? 1 : 0;
        if (blk) atomicAdd(d.active + slot, 1u);
    }
}

// Step of every cell of every field: the first move (0..7 in the order E,
// W, S, N, SE, SW, NE, NW) to a neighbour whose pair plus the move's unit is
// the cell's pair; kGoal at a goal, kNone when unreached or when no move
// fits (dist is then no distance field).
constexpr uint8_t kGoal = 0xfe, kNone = 0xff;

__global__ __launch_bounds__(kNT) void k_steps(TraceArgs a) {
    const int64_t N = (int64_t)a.nx * a.ny;
    const int64_t total = N * a.n_goals;
    for (int64_t k = blockIdx.x * (int64_t)kNT + threadIdx.x; k < total; k += (int64_t)gridDim.x * kNT) {
        const int64_t c = k % N;
        const uint64_t* D = a.dist + (k - c);
        const uint64_t v = D[c];
        uint8_t step = kNone;
        if (v == 0) {
            step = kGoal;
        } else if (v != kUnreached && a.nav[c]) {
            const int i = (int)(c % a.nx), j = (int)(c / a.nx);
            for (int m = 0; m < 8; ++m) {
                const int u = i + step_dx(m), w = j + step_dy(m);
                if (u < 0 || w < 0 || u >= a.nx || w >= a.ny) continue;
                const int64_t n = (int64_t)w * a.nx + u;
                if (!a.nav[n]) continue;
                if (m >= 4 && !(a.nav[(int64_t)j * a.nx + u] && a.nav[(int64_t)w * a.nx + i])) continue;
                const uint64_t dv = D[n];
                if (dv != kUnreached && dv + (m < 4 ? kOrth : kDiag) == v) {
                    step = (uint8_t)m;
                    break;
                }
            }
        }
        a.steps[(k / N) * a.stride + c] = step;
    }
}

// Walk of query q from cell s down its field's moves (rd(c): the move of
// cell c), storing up to cap cells; returns the path's cell count, or -1
// when a cell has no move (dist is then no distance field).  When rows of
// paths are 16-byte aligned the cells go out four at a time (the last four
// kept in registers), a quarter of the scattered stores.
template <class Rd>
__device__ __forceinline__ int32_t walk(const TraceArgs& a, int64_t q, int32_t s, Rd rd) {
    const int64_t N = (int64_t)a.nx * a.ny;
    int32_t* out = a.paths + q * a.cap;
    const bool vec = (a.cap & 3) == 0 && (reinterpret_cast<uintptr_t>(a.paths) & 15) == 0;
    int64_t c = s, m = 0;
    int32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;   // the last four cells, c3 the latest
    uint32_t st;
    for (;;) {
        c0 = c1;
        c1 = c2;
        c2 = c3;
        c3 = (int32_t)c;
        if (!vec) {
            if (m < a.cap) out[m] = c3;
        } else if ((m & 3) == 3 && m < a.cap) {
            *reinterpret_cast<int4*>(out + m - 3) = make_int4(c0, c1, c2, c3);
        }
        ++m;
        st = rd(c);
        if (st >= kGoal || m > N) break;      // kGoal and kNone are the codes above the moves
        c += (int64_t)step_dy(st) * a.nx + step_dx(st);
    }
    if (vec) {                             // the cells after the last full four
        const int r = (int)(m & 3);
        if (r >= 3 && m - 3 < a.cap) out[m - 3] = c1;
        if (r >= 2 && m - 2 < a.cap) out[m - 2] = c2;
        if (r >= 1 && m - 1 < a.cap) out[m - 1] = c3;
    }
    return st == kGoal ? (int32_t)m : -1;
}

__device__ __forceinline__ bool query_ok(const TraceArgs& a, int32_t s, int32_t slot) {
    const int64_t N = (int64_t)a.nx * a.ny;
    return slot >= 0 && slot < a.n_goals && s >= 0 && s < N && a.dist[(size_t)slot * N + s] != kUnreached;
}

// One query per thread, the moves read from global memory (L2).
__global__ __launch_bounds__(kNT) void k_trace(TraceArgs a) {
    for (int64_t q = blockIdx.x * (int64_t)kNT + threadIdx.x; q < a.n; q += (int64_t)gridDim.x * kNT) {
        const int32_t s = a.starts[q], slot = a.slots[q];
        int32_t len = 0;
        if (query_ok(a, s, slot)) {
            const uint8_t* S = a.steps + (size_t)slot * a.stride;
            len = walk(a, q, s, [&](int64_t c) { return S[c]; });
        }
        a.lengths[q] = len;
    }
}

// kTraceSplit workgroups per goal, each with the goal's moves staged in LDS
// (a walk step then waits for an LDS read rather than an L2 round trip).
// Workgroup part gathers the goal's queries q with q % kTraceSplit == part,
// in passes of kTraceList queries, and walks them one per thread, so a
// goal's walks spread over kTraceSplit compute units; the workgroups of
// goal 0 also end the queries of no goal.
constexpr int kTraceTable = 128 * 1024;    // bytes: the grids whose moves fit
constexpr int kTraceList = 4096;
constexpr int kTraceSplit = 8;

__global__ __launch_bounds__(kNT) void k_trace_lds(TraceArgs a) {
    __shared__ __align__(16) uint8_t L[kTraceTable];
    __shared__ int32_t list[kTraceList];
    __shared__ uint32_t cnt;
    const int g = blockIdx.x / kTraceSplit, part = blockIdx.x % kTraceSplit;
    const uint4* src = reinterpret_cast<const uint4*>(a.steps + (size_t)g * a.stride);
    for (int k = threadIdx.x; k < (int)(a.stride / 16); k += kNT) reinterpret_cast<uint4*>(L)[k] = src[k];
    for (int64_t base = 0; base < a.n; base += kTraceList) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();                   // (first pass: also the staged moves)
        const int64_t end = min(a.n, base + (int64_t)kTraceList);
        for (int64_t q = base + part + (int64_t)threadIdx.x * kTraceSplit; q < end; q += kNT * kTraceSplit) {
            const int32_t slot = a.slots[q];
            if (slot == g || (g == 0 && (slot < 0 || slot >= a.n_goals)))
                list[atomicAdd(&cnt, 1u)] = (int32_t)(q - base);
        }
        __syncthreads();
        const uint32_t k = cnt;
        for (uint32_t i = threadIdx.x; i < k; i += kNT) {
            const int64_t q = base + list[i];
            const int32_t s = a.starts[q], slot = a.slots[q];
            a.lengths[q] = query_ok(a, s, slot) ? walk(a, q, s, [&](int64_t c) { return L[c]; }) : 0;
        }
        __syncthreads();                   // list and count are reused
    }
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + kNT - 1) / kNT;
    return (unsigned)(b < 1 ? 1 : (b < 4096 ? b : 4096));
}

}  // namespace

int dist_tile() { return kT; }

void launch_navigable(const NavArgs& a, hipStream_t s) {
    k_navigable<<<grid_for((int64_t)a.nx * a.ny), kNT, 0, s>>>(a);
}

void launch_dist_init(const DistArgs& d, hipStream_t s) {
    k_dist_init<<<grid_for((int64_t)d.nx * d.ny * d.n_goals), kNT, 0, s>>>(d);
}

void launch_dist_rounds(const DistArgs& d, int round0, int n_rounds, hipStream_t s) {
    k_zero_u32<<<1, 64, 0, s>>>(d.active, n_rounds);
    const dim3 grid((unsigned)(d.tiles_x * d.tiles_y), (unsigned)((d.n_goals + kGW - 1) / kGW));
    for (int r = 0; r < n_rounds; ++r) k_dist_round<<<grid, kNT, 0, s>>>(d, round0 + r, r);
}

void launch_trace(const TraceArgs& a, hipStream_t s) {
    if (a.n == 0) return;
    k_steps<<<grid_for((int64_t)a.nx * a.ny * a.n_goals), kNT, 0, s>>>(a);
    // moves in LDS when a goal's fit and every workgroup's scan of the
    // queries stays small
    if (a.stride <= kTraceTable && (int64_t)a.n_goals * kTraceSplit * a.n <= ((int64_t)1 << 26))
        k_trace_lds<<<a.n_goals * kTraceSplit, kNT, 0, s>>>(a);
    else
        k_trace<<<grid_for(a.n), kNT, 0, s>>>(a);
}

}  // namespace hgs
