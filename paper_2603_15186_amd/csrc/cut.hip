// Level-of-detail cut on the GPU.
//
// Top-down, level-synchronous traversal of the hierarchy for all views at
// once (NavGSim Sec. III-B: LOD rendering selects Gaussians from different
// levels of the tree).  The frontier holds (node, view) entries of one level,
// a node's views mostly next to each other (see k_level_emit).  Per level:
//   count : each block decides its contiguous chunk (in the learned cut the
//           network settles the candidates right there), stores the
//           decisions and reduces (emitted, children) counts;
//   scan  : one block scans the per-block counts, advances the cut size and
//           sets the next frontier size (capacity checks here);
//   emit  : each block reads its chunk's decisions back, scans within the
//           block and writes emitted ids and child ids in order.
// A level's grid is sized to its frontier's bound (nodes of the level times
// views), at most kCutBlocks workgroups.
// Ids come out ascending per view because ids are level-major, children
// of a node are contiguous and ordered like their parents, and each view's
// entries keep their order through the emission.
//
// The node test is exact: FP64 with +, -, * only, in a fixed order, with FMA
// contraction disabled, so every IEEE FP64 implementation selects the same
// node set.
#include "device_util.h"
#include "internal.h"
#include "lod_mlp.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
constexpr int kNW = kNT / kWave;

enum : uint32_t { kDrop = 0, kEmit = 1, kExpand = 2, kCandidate = 4 };

// Decide a node for a view: dropped (sphere outside the frustum), emitted,
// or expanded into its children.  kCandidate is or-ed into kExpand when the
// threshold rule refines the node and its projected size is at most s_hi
// pixels: the band in which the learned rule may keep the node instead (the
// count pass lets the network make that choice).
__device__ __forceinline__ uint32_t node_decision(const ViewDev& V, int k, float4 b, int nchild, double s_hi) {
#pragma clang fp contract(off)
    NodeGeom g;
    node_geometry(V, b, &g);
    if (g.pz + g.r < V.znear) return kDrop;
    const double rr = g.r * g.r;
    const double eL = V.fx * g.px + V.cx * g.pz;
    if (eL < 0.0 && eL * eL > rr * V.nl) return kDrop;
    const double eR = V.fx * g.px + (V.cx - V.W) * g.pz;
    if (eR > 0.0 && eR * eR > rr * V.nr) return kDrop;
    const double eT = V.fy * g.py + V.cy * g.pz;
    if (eT < 0.0 && eT * eT > rr * V.nt) return kDrop;
    const double eB = V.fy * g.py + (V.cy - V.H) * g.pz;
    if (eB > 0.0 && eB * eB > rr * V.nb) return kDrop;
    if (nchild == 0) return kEmit;
    const double a = V.f2 * g.r;
    const double lhs = a * a;
    const double rhs = V.tau2 * g.d2;
    if (!(lhs > rhs)) return kEmit;
    if (k == V.keep_node) return kEmit;
    const bool cand = lhs <= (s_hi * s_hi) * g.d2;
    return kExpand | (cand ? kCandidate : 0u);
}

struct LevelCtx {
    const float4* bound;
    const int2* child;
    const ViewDev* views;
    int n_views;
    const uint2* in;
    uint32_t* in_count;
    uint2* out;
    uint32_t out_cap;
    uint2* cut;
    uint32_t cut_cap;
    uint4* tmp;               // [G] block counts, then offsets; [G] = level bases
    uint8_t* dec;             // per frontier entry: decision of the count pass
    bool defer;               // learned cut: the count pass lets the network settle candidates
    const float* w32;         // learned cut: FP32 weights (uniform: read through the scalar cache)
    Counters* ctr;
    int mode;
    const void* mlp;
    double s_hi;
    uint2* cand;
    uint32_t cand_cap;
    int level;
    bool leaves;              // the last level: every node is a leaf (no child ranges to read)
    bool group;               // children laid out child-major per group of a node's views
    int out_slot;             // index of the next frontier's counter
};

__device__ __forceinline__ void chunk_of(uint32_t n, int G, int b, uint32_t* lo, uint32_t* hi) {
    uint32_t chunk = ceil_div(n, (uint32_t)G);
    if (chunk < (uint32_t)kNT) chunk = kNT;
    chunk = ceil_div(chunk, (uint32_t)kNT) * kNT;
    uint64_t s = (uint64_t)b * chunk, e = s + chunk;
    *lo = (uint32_t)(s < n ? s : n);
    *hi = (uint32_t)(e < n ? e : n);
}

// (emitted, children, candidate) counts of a decision
__device__ __forceinline__ uint4 counts_of(const LevelCtx& c, uint32_t d, int nchild) {
    const uint32_t kind = d & 3u;
    return make_uint4(kind == kEmit ? 1u : 0u, kind == kExpand ? (uint32_t)nchild : 0u,
                      (c.cand != nullptr && (d & kCandidate)) ? 1u : 0u, 0u);
}

// Count pass: decide every entry of the block's chunk once, remember the
// decision for the emit pass, reduce the counts.  In the learned cut
// (DEFER) the candidates of each 256 entries are settled right here: their
// features are computed one lane per candidate and the matrix cores
// evaluate the network over the group (64 entries per wave; the network's
// work is negligible, so the group is not compacted).  The network keeps a
// candidate (emits it) unless its probability reaches p*.
//
// With node-grouped frontiers, the pass's views are staged in LDS when
// there are at most kLdsViews: a wave's entries span several views (a
// node's views are next to each other), and LDS serves a lane's own view
// without a gather.  Staged are the leading words through the side-plane
// normals and keep_node, all that the node test and the features read.
constexpr int kLdsViews = 64;
constexpr int kCutViewWords = (int)((offsetof(ViewDev, nb) + sizeof(double)) / 8);
static_assert(offsetof(ViewDev, o) == 0 && offsetof(ViewDev, nb) % 8 == 0, "views start with their FP64 words");

template <bool DEFER>
__global__ __launch_bounds__(kNT) void k_level_count(LevelCtx c, uint32_t in_cap) {
    __shared__ uint4 sh[kNT / kWave + 1];
    __shared__ float s_x[DEFER ? kNT * kMlpXStride : 1];
    __shared__ float s_w[DEFER ? kMlpParams : 1];  // the network's FP32 weights
    __shared__ uint64_t s_view[kLdsViews * kCutViewWords];
    __shared__ int32_t s_keep[kLdsViews];
    uint32_t n = *c.in_count;
    n = n < in_cap ? n : in_cap;
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, &lo, &hi);
    if (lo >= hi) {
        if (threadIdx.x == 0) c.tmp[blockIdx.x] = make_uint4(0, 0, 0, 0);
        return;
    }
    if (DEFER)
        for (int k = threadIdx.x; k < kMlpParams; k += kNT) s_w[k] = c.w32[k];
    // (view-major frontiers keep a wave on one view: scalar loads serve it)
    const bool lds_views = c.group && c.n_views <= kLdsViews;
    if (lds_views) {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(c.views);
        for (int k = threadIdx.x; k < c.n_views * kCutViewWords; k += kNT) {
            const int v = k / kCutViewWords, q = k - v * kCutViewWords;
            s_view[k] = src[(size_t)v * (sizeof(ViewDev) / 8) + q];
        }
        for (int v = threadIdx.x; v < c.n_views; v += kNT) s_keep[v] = c.views[v].keep_node;
        __syncthreads();
    }
    // f applied to view v (the staged words; the others, which neither the
    // node test nor the features read, stay zero)
    auto with_view = [&](uint32_t v, auto&& f) {
        if (lds_views) {
            uint64_t wd[sizeof(ViewDev) / 8];
#pragma unroll
            for (int q = 0; q < (int)(sizeof(ViewDev) / 8); ++q)
                wd[q] = q < kCutViewWords ? s_view[v * kCutViewWords + q] : 0ull;
            ViewDev V;
            __builtin_memcpy(&V, wd, sizeof V);
            V.keep_node = s_keep[v];
            return f(V);
        }
        return on_view(c.views, v, f);
    };
    const int w = threadIdx.x / kWave;
    uint4 acc = make_uint4(0, 0, 0, 0);
    auto decide = [&](bool valid, uint2 e, float4 b, int2 ch) -> uint32_t {
        if (!valid) return kDrop;
        return with_view(e.y, [&](const ViewDev& V) { return node_decision(V, (int)e.x, b, ch.y, c.s_hi); });
    };
    // the network's say on the group's candidates (every thread takes part)
    auto settle = [&](uint32_t d, uint2 e, float4 b) -> uint32_t {
        const bool cand = (d & kCandidate) != 0;
        if (!__syncthreads_or(cand)) return d;     // also orders s_x's reuse and publishes s_w
        const LodMlpDev& m = *(const LodMlpDev*)c.mlp;
        float f[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) f[k] = 0.f;
        if (cand) {
            with_view(e.y, [&](const ViewDev& V) {
                NodeGeom g;
                node_geometry(V, b, &g);
                lod_features(m, V, (int)e.x, b, g, c.level, f);
            });
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) f[k] = (f[k] - m.mean[k]) * m.inv_std[k];
        }
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) s_x[threadIdx.x * kMlpXStride + k] = f[k];
        __syncthreads();
        const float z = lod_mlp_logit_mfma(s_w, s_x + w * kWave * kMlpXStride);
        return (cand && !(1.f / (1.f + __expf(-z)) >= m.p_star)) ? (uint32_t)kEmit : d;
    };
    auto count = [&](uint32_t i, bool valid, uint32_t d, int2 ch) {
        if (!valid) return;
        c.dec[i] = (uint8_t)d;
        const uint4 r = counts_of(c, d, ch.y);
        acc.x += r.x;
        acc.y += r.y;
        acc.z += r.z;
    };
    // two entries per lane and step: their gathers are in flight together
    for (uint32_t s = lo; s < hi; s += 2 * kNT) {
        const uint32_t i0 = s + threadIdx.x, i1 = i0 + kNT;
        const bool v0 = i0 < hi, v1 = i1 < hi;
        const uint2 e0 = v0 ? c.in[i0] : make_uint2(0, 0);
        const uint2 e1 = v1 ? c.in[i1] : make_uint2(0, 0);
        const float4 b0 = c.bound[e0.x], b1 = c.bound[e1.x];
        const int2 ch0 = c.leaves ? make_int2(0, 0) : c.child[e0.x];
        const int2 ch1 = c.leaves ? make_int2(0, 0) : c.child[e1.x];
        uint32_t d0 = decide(v0, e0, b0, ch0);
        uint32_t d1 = decide(v1, e1, b1, ch1);
        if (DEFER) {
            d0 = settle(d0, e0, b0);
            d1 = settle(d1, e1, b1);
        }
        count(i0, v0, d0, ch0);
        count(i1, v1, d1, ch1);
    }
    uint4 tot;
    block_excl_scan4<kNT>(acc, sh, &tot);
    if (threadIdx.x == 0) c.tmp[blockIdx.x] = tot;
}

// Exclusive scan of the G <= 4 * 1024 block counts (four consecutive ones
// per thread).
__global__ __launch_bounds__(1024) void k_level_scan(LevelCtx c, int G, uint32_t in_cap) {
    __shared__ uint4 sh[1024 / kWave + 1];
    const int t = threadIdx.x;
    uint4 x[4];
    uint4 sum = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        x[j] = b < G ? c.tmp[b] : make_uint4(0, 0, 0, 0);
        sum.x += x[j].x;
        sum.y += x[j].y;
        sum.z += x[j].z;
    }
    uint4 tot;
    uint4 ex = block_excl_scan4<1024>(sum, sh, &tot);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        if (b < G) c.tmp[b] = ex;
        ex.x += x[j].x;
        ex.y += x[j].y;
        ex.z += x[j].z;
    }
    if (t == 0) {
        Counters* k = c.ctr;
        const uint32_t n_in = *c.in_count;
        k->visited += n_in < in_cap ? n_in : in_cap;
        const uint32_t base = k->cut;
        const uint32_t cbase = k->cand;
        c.tmp[G] = make_uint4(base, 0, cbase, 0);
        if (c.cand != nullptr) {
            const uint64_t want = (uint64_t)cbase + tot.z;
            if (want > c.cand_cap) {
                k->overflow |= kOvCand;
                if (want > k->need_cand) k->need_cand = (uint32_t)(want < 0xffffffffull ? want : 0xffffffffull);
            }
            k->cand = (uint32_t)(want < c.cand_cap ? want : c.cand_cap);
        }
        const uint64_t want_cut = (uint64_t)base + tot.x;
        if (want_cut > c.cut_cap) {
            k->overflow |= kOvCut;
            if (want_cut > k->need_cut) k->need_cut = (uint32_t)(want_cut < 0xffffffffull ? want_cut : 0xffffffffull);
        }
        k->cut = (uint32_t)(want_cut < c.cut_cap ? want_cut : c.cut_cap);
        if (tot.y > c.out_cap) {
            k->overflow |= kOvFrontier;
            if (tot.y > k->need_frontier) k->need_frontier = tot.y;
        }
        k->frontier[c.out_slot] = tot.y < c.out_cap ? tot.y : c.out_cap;
    }
}

// Each thread takes kEmitPer consecutive entries of the chunk, so that one
// workgroup scan places 1,024 entries.  The children an iteration appends
// to the next frontier form one run; it is assembled in LDS (up to
// kEmitStage entries, the rest stored directly) and written out coalesced.
// Within the run, the children of one group (consecutive entries of the
// same node, one per view) are laid out child-major: (c0, v1), (c0, v2),
// ..., (c1, v1), ...  A node's views thus stay next to each other at every
// level, so that the passes reading a node's data per entry (this cut's
// node tests, the projection's Gaussian and SH reads) find it in cache for
// the second and later views.  Each view's entries keep their order.
constexpr int kEmitPer = 4;
constexpr uint32_t kEmitStage = 4096;
// Views are grouped kCutViewGroup at a time; within a group the frontier
// is node-major (a node's views next to each other).  Larger groups share
// more of a node's reads between views; smaller ones keep fewer views in a
// wave (32 measured best on 50-view batches, between 16 and 64).
constexpr uint32_t kCutViewGroup = 32;

__global__ __launch_bounds__(kNT) void k_level_emit(LevelCtx c, uint32_t in_cap) {
    __shared__ uint4 sh[kNT / kWave + 1];
    __shared__ uint2 s_out[kEmitStage];
    __shared__ uint2 s_last[kNT];                       // (node, view group) of each thread's last entry
    __shared__ uint32_t s_gbase[kEmitPer * kNT + 1];    // children before each group, then the total
    uint32_t n = *c.in_count;
    n = n < in_cap ? n : in_cap;
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, &lo, &hi);
    if (lo >= hi) return;
    uint4 off = c.tmp[blockIdx.x];
    const uint32_t base = c.tmp[gridDim.x].x;
    const uint32_t cbase = c.tmp[gridDim.x].z;
    for (uint32_t s = lo; s < hi; s += kEmitPer * kNT) {
        // chunks start at multiples of kNT, so i0 is a multiple of kEmitPer
        const uint32_t i0 = s + kEmitPer * threadIdx.x;
        uint2 e[kEmitPer];
        uint32_t d[kEmitPer];
        if (i0 + kEmitPer <= hi) {
            const uint4 q0 = *reinterpret_cast<const uint4*>(c.in + i0);
            const uint4 q1 = *reinterpret_cast<const uint4*>(c.in + i0 + 2);
            e[0] = make_uint2(q0.x, q0.y);
            e[1] = make_uint2(q0.z, q0.w);
            e[2] = make_uint2(q1.x, q1.y);
            e[3] = make_uint2(q1.z, q1.w);
            const uint32_t dd = *reinterpret_cast<const uint32_t*>(c.dec + i0);
#pragma unroll
            for (int j = 0; j < kEmitPer; ++j) d[j] = (dd >> (8 * j)) & 0xffu;
        } else {
#pragma unroll
            for (int j = 0; j < kEmitPer; ++j) {
                const bool v = i0 + j < hi;
                e[j] = v ? c.in[i0 + j] : make_uint2(0, 0);
                d[j] = v ? c.dec[i0 + j] : (uint32_t)kDrop;
            }
        }
        uint4 r[kEmitPer];
        int first[kEmitPer];
        bool head[kEmitPer];
        uint4 mine = make_uint4(0, 0, 0, 0);
        const bool grouped = c.group && !c.leaves;
        if (grouped) {
            s_last[threadIdx.x] = make_uint2(e[kEmitPer - 1].x, e[kEmitPer - 1].y / kCutViewGroup);
            __syncthreads();
        }
        uint2 prev = (grouped && threadIdx.x > 0) ? s_last[threadIdx.x - 1] : make_uint2(~0u, ~0u);
#pragma unroll
        for (int j = 0; j < kEmitPer; ++j) {
            const bool expand = (d[j] & 3u) == kExpand;
            const int2 ch = (expand && !c.leaves) ? c.child[e[j].x] : make_int2(0, 0);
            first[j] = ch.x;
            r[j] = counts_of(c, d[j], ch.y);
            // a group starts where the node or the view group changes (node
            // ids are below 2^31)
            const uint32_t vg = e[j].y / kCutViewGroup;
            head[j] = e[j].x != prev.x || vg != prev.y;
            prev = make_uint2(e[j].x, vg);
            mine.x += r[j].x;
            mine.y += r[j].y;
            mine.z += r[j].z;
            mine.w += head[j] ? 1u : 0u;
        }
        uint4 tot;
        uint4 ex = block_excl_scan4<kNT>(mine, sh, &tot);
        uint32_t grp[kEmitPer], ey[kEmitPer];
        {
            uint4 run = ex;
#pragma unroll
            for (int j = 0; j < kEmitPer; ++j) {
                run.w += head[j] ? 1u : 0u;
                grp[j] = run.w - 1u;                    // this entry's group within the iteration
                ey[j] = run.y;
                if (grouped && head[j]) s_gbase[grp[j]] = run.y;
                run.y += r[j].y;
            }
        }
        if (grouped) {
            if (threadIdx.x == 0) s_gbase[tot.w] = tot.y;
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kEmitPer; ++j) {
            if (r[j].x) {
                const uint64_t pos = (uint64_t)base + off.x + ex.x;
                if (pos < c.cut_cap) c.cut[pos] = e[j];
            }
            if (r[j].z) {
                const uint64_t pos = (uint64_t)cbase + off.z + ex.z;
                if (pos < c.cand_cap) c.cand[pos] = e[j];
            }
            const uint32_t m = r[j].y;
            if (m) {
                // every expanding entry of the group has this node's m
                // children: the group's children are m * n_exp, this entry
                // is the rank-th expanding one (ungrouped: its children in
                // order at ey)
                uint32_t gb = ey[j], n_exp = 1, rank = 0;
                if (grouped) {
                    gb = s_gbase[grp[j]];
                    n_exp = (s_gbase[grp[j] + 1] - gb) / m;
                    rank = (ey[j] - gb) / m;
                }
                for (uint32_t q = 0; q < m; ++q) {
                    const uint32_t L = gb + q * n_exp + rank;
                    const uint2 child = make_uint2((uint32_t)(first[j] + (int)q), e[j].y);
                    if (L < kEmitStage) {
                        s_out[L] = child;
                    } else {
                        const uint64_t pos = (uint64_t)off.y + L;
                        if (pos < c.out_cap) c.out[pos] = child;
                    }
                }
            }
            ex.x += r[j].x;
            ex.z += r[j].z;
        }
        if (!c.leaves) {
            __syncthreads();
            const uint32_t staged = tot.y < kEmitStage ? tot.y : kEmitStage;
            for (uint32_t q = threadIdx.x; q < staged; q += kNT) {
                const uint64_t pos = (uint64_t)off.y + q;
                if (pos < c.out_cap) c.out[pos] = s_out[q];
            }
            __syncthreads();
        }
        off.x += tot.x;
        off.y += tot.y;
        off.z += tot.z;
    }
}

// Frontier of every view's roots (nodes [0, n_roots)): grouped, view
// groups in order and node-major within a group; otherwise view-major.
__global__ void k_init_roots(uint2* out, uint32_t n_roots, uint32_t n_views, uint32_t cap, Counters* ctr, int slot,
                             bool grouped) {
    const uint32_t total = n_roots * n_views;
    const uint32_t per = n_roots * kCutViewGroup;          // entries of a full group
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t vb = i / per, loc = i - vb * per;
        const uint32_t nb = min(kCutViewGroup, n_views - vb * kCutViewGroup);
        const uint2 e = grouped ? make_uint2(loc / nb, vb * kCutViewGroup + loc % nb) : make_uint2(i % n_roots, i / n_roots);
        if (i < cap) out[i] = e;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (total > cap) {
            ctr->overflow |= kOvFrontier;
            if (total > ctr->need_frontier) ctr->need_frontier = total;
        }
        ctr->frontier[slot] = total < cap ? total : cap;
    }
}

// Every listed id (or 0..n-1 when ids is null) for every view, view-major.
__global__ void k_emit_all(uint2* cut, const int32_t* ids, uint32_t n, uint32_t n_views, uint32_t cap, Counters* ctr) {
    const uint64_t total = (uint64_t)n * n_views;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total && i < cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = (uint32_t)(i % n);
        cut[i] = make_uint2(ids ? (uint32_t)ids[k] : k, (uint32_t)(i / n));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (total > cap) {
            ctr->overflow |= kOvCut;
            ctr->need_cut = (uint32_t)(total < 0xffffffffull ? total : 0xffffffffull);
        }
        ctr->cut = (uint32_t)(total < cap ? total : cap);
    }
}

// Features and screen footprint of each collected candidate.  The level of
// a node is recovered from the geometry record (mlp_geom.level_offset).
__global__ void k_lod_features(const uint2* cand, const uint32_t* count, const ViewDev* views, LodMlpDev m,
                               float* feats, int4* rects) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint2 e = cand[i];
        const ViewDev& V = views[e.y];
        const float4 b = m.bound[e.x];
        NodeGeom g;
        node_geometry(V, b, &g);
        int level = 0;
        while (level + 1 < m.n_levels && (int64_t)e.x >= m.level_offset[level + 1]) ++level;
        float f[kMlpIn];
        lod_features(m, V, (int)e.x, b, g, level, f);
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) feats[(size_t)i * kMlpIn + k] = f[k];
        // footprint: projection of the bounding sphere (centre +- f r / z),
        // the whole image when the sphere reaches the near plane; clamped to
        // the image and never empty
        int x0 = 0, y0 = 0, x1 = (int)V.W - 1, y1 = (int)V.H - 1;
        if (g.pz - g.r > V.znear) {
            const double u = V.fx * g.px / g.pz + V.cx, v = V.fy * g.py / g.pz + V.cy;
            const double ru = V.fx * g.r / (g.pz - g.r) + 1.0, rv = V.fy * g.r / (g.pz - g.r) + 1.0;
            const double lox = fmin(fmax(floor(u - ru), 0.0), V.W - 1.0), hix = fmin(fmax(ceil(u + ru), 0.0), V.W - 1.0);
            const double loy = fmin(fmax(floor(v - rv), 0.0), V.H - 1.0), hiy = fmin(fmax(ceil(v + rv), 0.0), V.H - 1.0);
            x0 = (int)lox; x1 = (int)hix; y0 = (int)loy; y1 = (int)hiy;
        }
        rects[i] = make_int4(x0, y0, x1, y1);
    }
}

}  // namespace

void launch_lod_features(const uint2* cand, const uint32_t* count, const ViewDev* views, const void* mlp_geom,
                         float* feats, int4* rects, hipStream_t s) {
    k_lod_features<<<1024, 256, 0, s>>>(cand, count, views, *(const LodMlpDev*)mlp_geom, feats, rects);
}

void launch_cut(const CutArgs& a, hipStream_t s) {
    const int G = kCutBlocks;
    static_assert(kCutBlocks <= 4 * 1024, "the level scan takes four counts per thread");
    if (a.flat || a.mode == HGS_LOD_ALL_LEAVES) {
        const uint32_t n = a.flat ? (uint32_t)a.n_nodes : (uint32_t)a.n_leaves;
        const int32_t* ids = a.flat ? nullptr : a.leaf_ids;
        k_emit_all<<<2048, 256, 0, s>>>(a.cut, ids, n, (uint32_t)a.n_views, a.cut_cap, a.ctr);
        return;
    }
    const uint32_t n_roots = (uint32_t)a.level_offset_host[1];
    k_init_roots<<<64, 256, 0, s>>>(a.frontier[0], n_roots, (uint32_t)a.n_views, a.frontier_cap, a.ctr, 0,
                                    a.group_children);
    int cur = 0;
    for (int L = 0; L < a.n_levels; ++L) {
        LevelCtx c;
        c.bound = a.bound;
        c.child = a.child;
        c.views = a.views;
        c.n_views = a.n_views;
        c.in = a.frontier[cur];
        c.in_count = &a.ctr->frontier[cur];
        c.out = a.frontier[cur ^ 1];
        c.out_cap = a.frontier_cap;
        c.cut = a.cut;
        c.cut_cap = a.cut_cap;
        c.tmp = a.scan_tmp;
        c.dec = a.dec;
        // p* = 0 refines every candidate: nothing for the network to decide
        c.defer = a.mode == HGS_LOD_LEARNED && a.mlp != nullptr && a.p_star > 0.f;
        c.w32 = a.mlp_w32;
        c.ctr = a.ctr;
        c.mode = a.mode;
        c.mlp = a.mlp;
        c.s_hi = a.s_hi;
        c.cand = a.cand;
        c.cand_cap = a.cand_cap;
        c.level = L;
        c.leaves = L == a.n_levels - 1;
        c.group = a.group_children;
        c.out_slot = cur ^ 1;
        // the frontier holds at most (nodes of level L) x views entries;
        // small levels get a grid of that size (the chunking keeps the
        // entries' order, so the cut does not depend on the grid)
        const uint64_t bound = (uint64_t)(a.level_offset_host[L + 1] - a.level_offset_host[L]) * (uint64_t)a.n_views;
        const int GL = (int)std::min<uint64_t>((uint64_t)G, std::max<uint64_t>(1, (bound + kNT - 1) / kNT));
        // a leaf is never refined, so the last level has no candidates
        if (c.defer && !c.leaves)
            k_level_count<true><<<GL, kNT, 0, s>>>(c, a.frontier_cap);
        else
            k_level_count<false><<<GL, kNT, 0, s>>>(c, a.frontier_cap);
        k_level_scan<<<1, 1024, 0, s>>>(c, GL, a.frontier_cap);
        k_level_emit<<<GL, kNT, 0, s>>>(c, a.frontier_cap);
        cur ^= 1;
    }
}

}  // namespace hgs
