// Host side of the C ABI: context, validation, scene upload, cameras,
// capacity management and the render sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <array>
#include <vector>
#include <mutex>

#include "internal.h"
#include "lod_mlp.h"

using namespace hgs;

namespace {

struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
};

// Work buffers of one pipeline pass.  With two lanes, consecutive passes
// alternate between two sets on two streams, so one pass's compositing
// overlaps the next pass's cut, projection and binning.
struct Work {
    DevMem frontier[2], cut, proj, dkey[2], dval[2], ntiles, bins, offsets, dec;
    DevMem pkey[2], pval[2], scan_tmp, hist;
};

}  // namespace

struct hgs_ctx {
    int device = 0;
    std::string err;
    // scene
    bool loaded = false;
    bool hier = false;
    int64_t n = 0;
    int sh_degree = 0;
    int n_levels = 0;
    std::vector<int64_t> level_offset;
    int64_t n_leaves = 0;
    DevMem geo, sh, bound, child, leaf_ids, parent, nodefeat, lvl;
    // views
    std::vector<hgs_camera> cams;
    ViewDev* views_host = nullptr;    // pinned mirror
    DevMem views;
    DevMem tile_view;
    uint32_t total_tiles = 0;
    hipEvent_t views_copied = nullptr;
    bool views_dirty = true;
    // passes: a batch runs as consecutive groups of views, one pipeline pass
    // per group, when a single pass would not fit the entry index space (or
    // the caller caps the views per pass); every buffer is reused per pass
    std::vector<uint32_t> tile_abs;   // tile offset of each view in the batch
    std::vector<int> pass_v0;         // first view of each pass, then the view count
    int pass_views = 0;               // HGS_OPT_PASS_VIEWS (0: no cap)
    int want_passes = 1;
    // lod
    int lod_mode = HGS_LOD_THRESHOLD;
    float tau = 1.0f;
    bool mlp_loaded = false;
    DevMem mlp_w, mlp_w32, mlp_dev;
    LodMlpDev mlp_host{};
    double s_hi = 64.0;               // candidate band of the learned cut (pixels)
    DevMem train_scratch, region_dev, surf;
    int32_t n_surf = 0;
    // options
    bool sync_check = true, auto_regrow = true, use_graph = false;
    RenderOpts ropts;
    // work buffers
    uint32_t frontier_cap = 0, cut_cap = 0, pair_cap = 0;
    Work w[2];                        // per lane
    DevMem ranges, counters;          // shared: indexed by absolute tile / by pass
    int lanes = 1;                    // HGS_OPT_LANES
    hipStream_t lane_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    Counters* ctr_host = nullptr;     // pinned
    bool last_valid = false;
    int64_t regrows = 0;
    uint32_t forced_cap = 0;          // test hook: start from this capacity
    int sort_digit_bits = 8;          // widest radix digit
    double mean_lo[3] = {0, 0, 0}, mean_hi[3] = {0, 0, 0};   // bounding box of every node's mean
    bool depth_full = false;          // a depth fell outside its bound: sort all 32 key bits from then on
    // captured render (HGS_OPT_USE_GRAPH): recorded on cap_stream, replayed
    // on the caller's stream while nothing it depends on has changed
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    int64_t graph_launches = 0;
    // stage timing: 6 events per render (start, cut, project, binning, composite start, end)
    bool stage_timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double acc_ms[5] = {0, 0, 0, 0, 0};
    int64_t acc_n = 0;
    // sort scratch for hgs_sort_pairs
    DevMem sort_k, sort_v, sort_n, sort_hist;
    DevMem px_state;                  // per pixel of the last render: stop position, final T
    // distance-field scratch: goals, tile flags, per-round change counts
    DevMem nav_goals, nav_flags, nav_active, nav_steps;
    // backward pass: per-entry gradients and per-view image gradients; the
    // last render's final pair buffer and whether it blended levels
    DevMem egrad, dimg, brec;
    ImgGrad* dimg_host = nullptr;        // pinned, kMaxViews entries
    hipEvent_t dimg_copied = nullptr;
    // stage timing of backward passes: (start, compositing done, end)
    std::vector<std::array<hipEvent_t, 3>> bwd_ev;
    double bwd_ms[2] = {0, 0};
    int64_t bwd_n = 0;
    int last_pair_buf = 0;
    int last_lane = 0;
    bool last_blend = false;
    bool last_keep = false;           // the last render kept its pixel states (px_state)
    bool last_default_tiles = true;   // the last render binned to kTile x kTile tiles
    uint32_t* nav_active_host = nullptr;   // pinned
    void* scratch = nullptr;          // this device's static scratch area (hgs_sort_pairs_noalloc)
};

namespace {

hgs_status fail(hgs_ctx* c, hgs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(c, call)                                                                          \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail((c), HGS_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void release(DevMem& m) {
    if (m.p) (void)hipFree(m.p);
    m.p = nullptr;
    m.bytes = 0;
}

void invalidate_graph(hgs_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_valid = false;
}

hgs_status ensure(hgs_ctx* c, DevMem& m, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (m.bytes >= bytes) return HGS_OK;
    invalidate_graph(c);     // a captured render holds the old address
    release(m);
    hipError_t e = hipMalloc(&m.p, bytes);
    if (e != hipSuccess) {
        m.p = nullptr;
        (void)hipGetLastError();
        return fail(c, HGS_E_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    m.bytes = bytes;
    return HGS_OK;
}

template <typename T>
T* P(const DevMem& m) { return static_cast<T*>(m.p); }

bool finite(float x) { return std::isfinite(x); }

float bf16_to_f32_host(uint16_t h) {
    const uint32_t b = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

int bits_for(uint32_t n) {
    int b = 1;
    while (b < 32 && (1ull << b) < n) ++b;
    return b;
}

// Pair sort keys are view << bits_for(tiles of the largest view) | tile
// within the view, below 2^31.
bool pair_keys_fit(int n_views, uint64_t max_view_tiles) {
    return max_view_tiles < (1ull << 31) && bits_for((uint32_t)n_views) + bits_for((uint32_t)max_view_tiles) <= 31;
}

__global__ void k_reset(Counters* c) {
    if (threadIdx.x == 0) {
        Counters z = {};
        *c = z;
    }
}

hgs_status alloc_work(hgs_ctx* c) {
    hgs_status s;
    const size_t F = c->frontier_cap, M = c->cut_cap, Pc = c->pair_cap;
    for (int l = 0; l < c->lanes; ++l) {
        Work& w = c->w[l];
        for (int i = 0; i < 2; ++i)
            if ((s = ensure(c, w.frontier[i], F * sizeof(uint2)))) return s;
        if ((s = ensure(c, w.dec, F))) return s;
        if ((s = ensure(c, w.cut, M * sizeof(uint2)))) return s;
        if ((s = ensure(c, w.proj, M * sizeof(Proj)))) return s;
        for (int i = 0; i < 2; ++i) {
            if ((s = ensure(c, w.dkey[i], M * 4))) return s;
            if ((s = ensure(c, w.dval[i], M * 4))) return s;
            if ((s = ensure(c, w.pkey[i], Pc * 4))) return s;
            if ((s = ensure(c, w.pval[i], Pc * 4))) return s;
        }
        if ((s = ensure(c, w.ntiles, M * 4))) return s;
        if ((s = ensure(c, w.bins, M * sizeof(BinRec)))) return s;
        if ((s = ensure(c, w.offsets, M * 4))) return s;
        if ((s = ensure(c, w.scan_tmp, (std::max(kScanBlocks, kCutBlocks) + 1) * sizeof(uint4)))) return s;
        if ((s = ensure(c, w.hist, kSortHistBytes))) return s;
    }
    return HGS_OK;
}

// Lane of pass g and the work set it uses.
int lane_of(const hgs_ctx* c, int g) { return c->lanes > 1 ? g % c->lanes : 0; }

void release_work(Work& w) {
    DevMem* all[] = {&w.frontier[0], &w.frontier[1], &w.cut, &w.proj, &w.dkey[0], &w.dkey[1], &w.dval[0],
                     &w.dval[1], &w.ntiles, &w.bins, &w.offsets, &w.dec, &w.pkey[0], &w.pkey[1], &w.pval[0],
                     &w.pval[1], &w.scan_tmp, &w.hist};
    for (DevMem* m : all) release(*m);
}

// Cut entries are addressed by 28-bit indices inside pair values; pairs by
// 32-bit positions.
constexpr uint64_t kEntryLimit = (uint64_t)kEntryMask + 1;
constexpr uint64_t kPairLimit = 0xF0000000ull;

uint32_t clamp_cap(uint64_t x, uint64_t lim = kEntryLimit) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(x, 1024), lim);
}

void initial_caps(hgs_ctx* c) {
    if (c->forced_cap) {
        c->cut_cap = c->frontier_cap = c->forced_cap;
        c->pair_cap = c->forced_cap;
        return;
    }
    const uint64_t V = c->cams.size();
    const uint64_t per_view = c->hier ? (uint64_t)c->n_leaves : (uint64_t)c->n;
    const uint64_t budget = 48ull << 20;     // entries
    uint64_t m = std::min<uint64_t>(V * per_view, budget);
    if (!c->hier || c->lod_mode == HGS_LOD_ALL_LEAVES) m = std::min<uint64_t>(V * per_view, 1ull << 31);
    c->cut_cap = std::max(c->cut_cap, clamp_cap(m));
    c->frontier_cap = std::max(c->frontier_cap, clamp_cap(std::min<uint64_t>(m, budget), kPairLimit));
    c->pair_cap = std::max(c->pair_cap, clamp_cap(std::min<uint64_t>(8 * (uint64_t)c->cut_cap, 256ull << 20), kPairLimit));
}

hgs_status upload_views(hgs_ctx* c, hipStream_t s, const hgs_output* outs) {
    const int V = (int)c->cams.size();
    bool changed = c->views_dirty;
    for (int v = 0; v < V; ++v) {
        ViewDev& d = c->views_host[v];
        if (d.rgb != outs[v].rgb || d.depth != outs[v].depth || d.alpha != outs[v].alpha) changed = true;
    }
    if (!changed) return HGS_OK;
    HIP_TRY(c, hipEventSynchronize(c->views_copied));   // previous copy done with the mirror
    for (int v = 0; v < V; ++v) {
        ViewDev& d = c->views_host[v];
        d.rgb = outs[v].rgb;
        d.depth = outs[v].depth;
        d.alpha = outs[v].alpha;
    }
    HIP_TRY(c, hipMemcpyAsync(c->views.p, c->views_host, sizeof(ViewDev) * V, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipEventRecord(c->views_copied, s));
    c->views_dirty = false;
    return HGS_OK;
}

hgs_status harvest_events(hgs_ctx* c) {
    for (auto& e : c->bwd_ev) {
        HIP_TRY(c, hipEventSynchronize(e[2]));
        float a = 0.f, b = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&a, e[0], e[1]));
        HIP_TRY(c, hipEventElapsedTime(&b, e[0], e[2]));
        c->bwd_ms[0] += a;
        c->bwd_ms[1] += b;
        ++c->bwd_n;
        for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
    c->bwd_ev.clear();
    for (size_t b = 0; b + 6 <= c->ev_used; b += 6) {
        HIP_TRY(c, hipEventSynchronize(c->ev_pool[b + 5]));
        float t[5];
        HIP_TRY(c, hipEventElapsedTime(&t[0], c->ev_pool[b], c->ev_pool[b + 1]));
        HIP_TRY(c, hipEventElapsedTime(&t[1], c->ev_pool[b + 1], c->ev_pool[b + 2]));
        HIP_TRY(c, hipEventElapsedTime(&t[2], c->ev_pool[b + 2], c->ev_pool[b + 4]));
        HIP_TRY(c, hipEventElapsedTime(&t[3], c->ev_pool[b + 4], c->ev_pool[b + 5]));
        HIP_TRY(c, hipEventElapsedTime(&t[4], c->ev_pool[b], c->ev_pool[b + 5]));
        for (int i = 0; i < 5; ++i) c->acc_ms[i] += t[i];
    }
    c->ev_used = 0;
    return HGS_OK;
}

// Event slot k of the current render, creating pool entries on demand.
hipEvent_t stage_event(hgs_ctx* c, int k) {
    const size_t i = c->ev_used + k;
    while (c->ev_pool.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[i];
}

void mark(hgs_ctx* c, int k, hipStream_t s) {
    if (!c->stage_timing) return;
    hipEvent_t e = stage_event(c, k);
    if (e) (void)hipEventRecord(e, s);
}

int n_passes(const hgs_ctx* c) { return c->pass_v0.size() < 2 ? 1 : (int)c->pass_v0.size() - 1; }

uint32_t pass_tile0(const hgs_ctx* c, int g) {
    const int v = c->pass_v0[g];
    return v < (int)c->cams.size() ? c->tile_abs[v] : c->total_tiles;
}

// Group the views into about `want` consecutive passes of similar pixel
// count (at most pass_views views each) and make every view's tile base, and
// the tile -> view table, relative to its pass.  upload_table: rewrite the
// device table (the layout changed); otherwise only the host mirror moves.
hgs_status plan_passes(hgs_ctx* c, int want, bool upload_table) {
    const int V = (int)c->cams.size();
    want = std::max(c->lanes, want);
    want = std::max(1, std::min(want, V));
    uint64_t total = 0;
    for (const hgs_camera& k : c->cams) total += (uint64_t)k.width * k.height;
    std::vector<int> v0{0};
    uint64_t acc = 0;
    int in_pass = 0;
    for (int v = 0; v < V; ++v) {
        acc += (uint64_t)c->cams[v].width * c->cams[v].height;
        ++in_pass;
        const bool full = c->pass_views > 0 && in_pass >= c->pass_views;
        if (v + 1 < V && (full || acc * (uint64_t)want >= total * (uint64_t)v0.size())) {
            v0.push_back(v + 1);
            in_pass = 0;
        }
    }
    v0.push_back(V);
    if (upload_table || v0 != c->pass_v0) {
        upload_table = true;
        invalidate_graph(c);
    }
    c->pass_v0 = v0;
    c->want_passes = want;
    HIP_TRY(c, hipEventSynchronize(c->views_copied));   // the mirror may still be in flight
    std::vector<uint32_t> tv(upload_table ? c->total_tiles : 0);
    for (size_t g = 0; g + 1 < v0.size(); ++g) {
        const uint32_t t0 = c->tile_abs[v0[g]];
        for (int v = v0[g]; v < v0[g + 1]; ++v) {
            ViewDev& d = c->views_host[v];
            d.tile_base = c->tile_abs[v] - t0;
            if (!upload_table) continue;
            const uint32_t nt = (uint32_t)(d.tiles_x * d.tiles_y);
            for (uint32_t t = 0; t < nt; ++t) tv[c->tile_abs[v] + t] = (uint32_t)(v - v0[g]);
        }
    }
    if (upload_table && c->total_tiles)
        HIP_TRY(c, hipMemcpy(c->tile_view.p, tv.data(), (size_t)c->total_tiles * 4, hipMemcpyHostToDevice));
    c->views_dirty = true;
    return HGS_OK;
}

// One pipeline pass over the views of pass g (counters slot g).
void enqueue_pass(hgs_ctx* c, hipStream_t s, int g) {
    Work& W = c->w[lane_of(c, g)];
    Counters* ctr = P<Counters>(c->counters) + g;
    const int v0 = c->pass_v0[g], v1 = c->pass_v0[g + 1];
    const uint32_t t0 = pass_tile0(c, g), t1 = pass_tile0(c, g + 1);
    if (c->stage_timing && c->ev_used >= 6 * 512) (void)harvest_events(c);
    mark(c, 0, s);
    k_reset<<<1, 64, 0, s>>>(ctr);
    CutArgs ca{};
    ca.bound = P<float4>(c->bound);
    ca.child = P<int2>(c->child);
    ca.leaf_ids = P<int32_t>(c->leaf_ids);
    ca.n_leaves = c->n_leaves;
    ca.n_nodes = c->n;
    ca.level_offset_host = c->level_offset.data();
    ca.n_levels = c->n_levels;
    ca.mode = c->lod_mode;
    ca.flat = !c->hier;
    ca.views = P<ViewDev>(c->views) + v0;
    ca.n_views = v1 - v0;
    ca.frontier[0] = P<uint2>(W.frontier[0]);
    ca.frontier[1] = P<uint2>(W.frontier[1]);
    ca.frontier_cap = c->frontier_cap;
    ca.cut = P<uint2>(W.cut);
    ca.cut_cap = c->cut_cap;
    ca.scan_tmp = P<uint4>(W.scan_tmp);
    ca.dec = P<uint8_t>(W.dec);
    ca.ctr = ctr;
    ca.mlp = (c->lod_mode == HGS_LOD_LEARNED && c->mlp_loaded) ? c->mlp_dev.p : nullptr;
    ca.p_star = c->mlp_host.p_star;
    ca.mlp_w32 = c->mlp_loaded ? P<float>(c->mlp_w32) : nullptr;
    ca.s_hi = c->s_hi;
    ca.cand = nullptr;
    ca.cand_cap = 0;
    // node-grouped frontiers, except under LOD blending (its projection
    // takes a view's sibling as the cut entry before it) and for renders
    // that keep pixel states for the backward pass (whose compositing
    // gathers each tile's entry records: 8.74 ms with the plain order,
    // 8.99 ms node-grouped)
    ca.group_children = !c->ropts.lod_blend && !c->ropts.keep_state;
    launch_cut(ca, s);
    mark(c, 1, s);

    // pair keys: view << key_shift | tile within the view, so that once the
    // entries are grouped by view only the tile bits need sorting
    uint32_t max_tiles = 1;
    for (int v = v0; v < v1; ++v)
        max_tiles = std::max(max_tiles, (uint32_t)(c->views_host[v].tiles_x * c->views_host[v].tiles_y));
    const int key_shift = bits_for(max_tiles);

    ProjectArgs pa{};
    pa.cut = ca.cut;
    pa.cut_cap = c->cut_cap;
    pa.geo = P<float4>(c->geo);
    pa.sh = P<float>(c->sh);
    pa.n = c->n;
    pa.sh_degree = c->sh_degree;
    pa.views = ca.views;
    pa.n_views = ca.n_views;
    pa.lds_views = ca.group_children && ca.n_views <= kProjectLdsViews;
    pa.proj = P<Proj>(W.proj);
    pa.depth_key = P<uint32_t>(W.dkey[0]);
    // Binned depths lie in (znear, distance to the farthest corner of the
    // means' bounding box] of their view, so the sort needs only the bits
    // that span that range of FP32 bit patterns (a depth outside raises
    // kOvDepth and the batch is redone with all 32 bits).
    int depth_bits = 32;
    pa.depth_base = 0;
    pa.depth_top = 0xffffffffu;
    if (!c->depth_full) {
        float zn = 0.f;
        double dmax = 0.0;
        for (int v = v0; v < v1; ++v) {
            const ViewDev& d = c->views_host[v];
            zn = v == v0 ? (float)d.znear : std::min(zn, (float)d.znear);
            double far2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double e = std::max(std::fabs(c->mean_lo[k] - d.o[k]), std::fabs(c->mean_hi[k] - d.o[k]));
                far2 += e * e;
            }
            dmax = std::max(dmax, std::sqrt(far2));
        }
        const float top = (float)(dmax * (1.0 + 1e-6) + 1e-6);
        uint32_t bb, tb;
        std::memcpy(&bb, &zn, 4);
        std::memcpy(&tb, &top, 4);
        if (zn > 0.f && tb > bb) {
            pa.depth_base = bb;
            pa.depth_top = tb;
            depth_bits = bits_for(tb - bb + 1u);
        }
    }
    pa.depth_val = P<uint32_t>(W.dval[0]);
    pa.ntiles = P<uint32_t>(W.ntiles);
    pa.bins = P<BinRec>(W.bins);
    pa.exact_tiles = c->ropts.exact_tiles;
    pa.ctr = ctr;
    pa.blend = c->ropts.lod_blend && c->hier && c->lod_mode != HGS_LOD_ALL_LEAVES;
    pa.parent = P<int32_t>(c->parent);
    pa.bound = P<float4>(c->bound);
    pa.child = P<int2>(c->child);
    pa.tile_w = c->ropts.tile_w;
    pa.tile_h = c->ropts.tile_h;
    pa.key_shift = key_shift;
    // When the view fits above the depth bits, one sort on (view, depth)
    // gives the view-grouped depth order; otherwise a stable pass on the
    // entries' views (read from the cut) follows the depth sort.
    const int view_bits = ca.n_views > 1 ? bits_for((uint32_t)ca.n_views) : 0;
    const bool view_in_key = ca.n_views > 1 && depth_bits + view_bits <= 32;
    pa.view_shift = view_in_key ? depth_bits : 0;
    launch_project(pa, s);
    mark(c, 2, s);

    SortArgs sa{};
    sa.keys[0] = P<uint32_t>(W.dkey[0]);
    sa.keys[1] = P<uint32_t>(W.dkey[1]);
    sa.vals[0] = P<uint32_t>(W.dval[0]);
    sa.vals[1] = P<uint32_t>(W.dval[1]);
    sa.count = &ctr->cut;
    sa.cap = c->cut_cap;
    sa.key_bits = view_in_key ? depth_bits + view_bits : depth_bits;
    sa.max_digit_bits = c->sort_digit_bits;
    sa.hist = P<uint32_t>(W.hist);
    int dr = launch_sort(sa, s);
    if (ca.n_views > 1 && !view_in_key) {
        // stable pass on the entries' views: depth order within each view
        launch_view_keys(sa.vals[dr], ca.cut, &ctr->cut, c->cut_cap, sa.keys[dr], s);
        SortArgs sv = sa;
        sv.keys[0] = sa.keys[dr];
        sv.keys[1] = sa.keys[dr ^ 1];
        sv.vals[0] = sa.vals[dr];
        sv.vals[1] = sa.vals[dr ^ 1];
        sv.key_bits = bits_for((uint32_t)ca.n_views);
        dr ^= launch_sort(sv, s);
    }

    EmitArgs ea{};
    ea.order = sa.vals[dr];
    ea.ntiles = pa.ntiles;
    ea.bins = pa.bins;
    ea.proj = pa.proj;
    ea.cut_cap = c->cut_cap;
    ea.offsets = P<uint32_t>(W.offsets);
    ea.keys = P<uint32_t>(W.pkey[0]);
    ea.vals = P<uint32_t>(W.pval[0]);
    ea.pair_cap = c->pair_cap;
    ea.exact_tiles = c->ropts.exact_tiles;
    ea.scan_tmp = ca.scan_tmp;
    ea.ctr = ctr;
    ea.tile_w = c->ropts.tile_w;
    ea.tile_h = c->ropts.tile_h;
    launch_emit(ea, s);

    SortArgs pb{};
    pb.keys[0] = P<uint32_t>(W.pkey[0]);
    pb.keys[1] = P<uint32_t>(W.pkey[1]);
    pb.vals[0] = P<uint32_t>(W.pval[0]);
    pb.vals[1] = P<uint32_t>(W.pval[1]);
    pb.count = &ctr->pairs;
    pb.cap = c->pair_cap;
    pb.key_bits = key_shift;
    pb.max_digit_bits = c->sort_digit_bits;
    pb.hist = sa.hist;
    const int pr = launch_sort(pb, s);
    c->last_pair_buf = pr;
    c->last_lane = lane_of(c, g);
    c->last_blend = pa.blend;
    c->last_keep = c->ropts.keep_state;
    c->last_default_tiles = c->ropts.tile_w == kTile && c->ropts.tile_h == kTile;

    CompositeArgs xa{};
    xa.keys = pb.keys[pr];
    xa.vals = pb.vals[pr];
    xa.pair_cap = c->pair_cap;
    xa.cut_cap = c->cut_cap;
    xa.ranges = P<uint2>(c->ranges) + t0;
    xa.total_tiles = t1 - t0;
    xa.proj = pa.proj;
    xa.views = ca.views;
    xa.tile_view = P<uint32_t>(c->tile_view) + t0;
    xa.n_views = ca.n_views;
    xa.key_shift = key_shift;
    xa.opts = c->ropts;
    xa.ctr = ctr;
    xa.state = c->ropts.keep_state ? P<uint2>(c->px_state) + (size_t)t0 * kTilePx : nullptr;
    launch_ranges(xa, s);
    mark(c, 4, s);
    launch_composite(xa, s);
    mark(c, 5, s);
    if (c->stage_timing) c->ev_used += 6;
}

// Passes in order; with two lanes the odd passes run on the second stream
// (forked from and joined back into s by events), each lane in order on its
// own work set.
void enqueue_render(hgs_ctx* c, hipStream_t s) {
    const int np = n_passes(c);
    const bool two = c->lanes > 1 && np > 1 && c->lane_stream;
    if (two) {
        (void)hipEventRecord(c->fork_ev, s);
        (void)hipStreamWaitEvent(c->lane_stream, c->fork_ev, 0);
    }
    for (int g = 0; g < np; ++g) enqueue_pass(c, two && (g & 1) ? c->lane_stream : s, g);
    if (two) {
        (void)hipEventRecord(c->join_ev, c->lane_stream);
        (void)hipStreamWaitEvent(s, c->join_ev, 0);
    }
    if (c->stage_timing) ++c->acc_n;
}

// Overflow bits of all passes and the largest need of any pass.
Counters merge_passes(const hgs_ctx* c, uint64_t* need_cut_sum) {
    Counters m{};
    uint64_t sum = 0;
    for (int g = 0; g < n_passes(c); ++g) {
        const Counters& k = c->ctr_host[g];
        m.overflow |= k.overflow;
        m.need_frontier = std::max(m.need_frontier, k.need_frontier);
        m.need_cut = std::max(m.need_cut, k.need_cut);
        m.need_pairs = std::max(m.need_pairs, k.need_pairs);
        m.need_cand = std::max(m.need_cand, k.need_cand);
        sum += std::max(k.need_cut, k.cut);
    }
    if (need_cut_sum) *need_cut_sum = sum;
    return m;
}

hgs_status read_counters(hgs_ctx* c, hipStream_t s) {
    HIP_TRY(c, hipMemcpyAsync(c->ctr_host, c->counters.p, sizeof(Counters) * n_passes(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return HGS_OK;
}

// Node-geometry part of the learned-LOD record (pointers into the scene).
LodMlpDev mlp_geometry(hgs_ctx* c) {
    LodMlpDev m{};
    m.nodefeat = P<float4>(c->nodefeat);
    m.bound = P<float4>(c->bound);
    m.level_offset = P<int64_t>(c->lvl);
    m.n_levels = c->n_levels;
    return m;
}

hgs_status grow_from(hgs_ctx* c, const Counters& k) {
    auto grow = [](uint32_t cap, uint32_t need, uint64_t lim) {
        uint64_t g = std::max<uint64_t>((uint64_t)need + need / 4, 2ull * cap);
        return clamp_cap(g, lim);
    };
    if (k.overflow & kOvFrontier) c->frontier_cap = grow(c->frontier_cap, k.need_frontier, kPairLimit);
    if (k.overflow & kOvCut) c->cut_cap = grow(c->cut_cap, k.need_cut, kEntryLimit);
    if (k.overflow & kOvPairs) c->pair_cap = grow(c->pair_cap, k.need_pairs, kPairLimit);
    if (k.overflow & kOvDepth) {
        c->depth_full = true;
        invalidate_graph(c);
    }
    // a cut overflow leaves the pair count unknown; keep pairs proportional
    if (k.overflow & kOvCut)
        c->pair_cap = std::max(c->pair_cap, clamp_cap(std::min<uint64_t>(8ull * c->cut_cap, kPairLimit), kPairLimit));
    ++c->regrows;
    return alloc_work(c);
}

}  // namespace

namespace {

// Plan-cache key: scene size, view sizes and LOD (FNV-1a over the sizes).
std::string plan_key(const hgs_ctx* c) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t x) {
        for (int i = 0; i < 8; ++i) {
            h ^= (x >> (8 * i)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (const hgs_camera& k : c->cams) mix(((uint64_t)k.width << 32) | (uint32_t)k.height);
    char buf[160];
    std::snprintf(buf, sizeof buf, "n%lld_v%zu_%016llx_lod%d_tau%.6g_l%d", (long long)c->n, c->cams.size(),
                  (unsigned long long)h, c->lod_mode, (double)c->tau, c->lanes);
    return buf;
}

bool read_plan(const char* path, const std::string& key, hgs_plan* p) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        hgs_plan q{};
        q.lanes = 1;
        q.tile_w = q.tile_h = kTile;
        q.pixels_per_thread = 1;
        const int got = std::sscanf(line, "%255s %d %d %d %lf %lf %d %d %d %d", k, &q.batch_depth, &q.persistent,
                                    &q.sort_digit_bits, &q.ms, &q.ms_default, &q.lanes, &q.tile_w, &q.tile_h,
                                    &q.pixels_per_thread);
        if (got >= 6 && key == k && tile_shape_ok(q.tile_w, q.tile_h, q.pixels_per_thread)) {
            if (got == 6) q.lanes = 1;
            *p = q;          // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

// Mean render time of the current options over reps renders (after one
// checked render that settles the buffer capacities).
hgs_status time_plan(hgs_ctx* c, hipStream_t s, const hgs_output* outs, int reps, hipEvent_t e0, hipEvent_t e1,
                     double* ms) {
    hgs_status st = hgs_render(c, s, outs);
    if (st) return st;
    c->sync_check = false;
    HIP_TRY(c, hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) enqueue_render(c, s);
    HIP_TRY(c, hipEventRecord(e1, s));
    HIP_TRY(c, hipEventSynchronize(e1));
    c->sync_check = true;
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / reps;
    return HGS_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------ static scratch memory

namespace {

// hgs_sort_pairs_noalloc sorts in a fixed area that every context on a GPU
// shares: the second key and value arrays of the ping-pong, the element
// count and the digit histograms of at most kStaticSortGroups groups.
constexpr uint32_t kStaticSortMax = HGS_SORT_NOALLOC_MAX;
constexpr uint32_t kStaticSortGroups = kStaticSortMax / kSortGroup;
static_assert(kStaticSortMax % kSortGroup == 0, "whole histogram groups");
constexpr size_t kScratchPing = (size_t)kStaticSortMax * 4;
constexpr size_t kScratchHistOff = 2 * kScratchPing + 256;
constexpr size_t kScratchBytes = kScratchHistOff + (size_t)kSortBins * (kStaticSortGroups + 1) * 4;
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: each device's address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current;
// looked up once per device.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

__global__ void k_set_count(uint32_t* count, uint32_t n) {
    if (threadIdx.x == 0) *count = n;
}

__global__ void k_copy_pairs(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs, uint32_t* kd,
                             uint32_t* vd, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

}  // namespace

hgs_status hgs_create(int32_t device, hgs_ctx** out) {
    if (!out) return HGS_E_INVALID;
    *out = nullptr;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd <= 0) {
        (void)hipGetLastError();
        return HGS_E_HIP;
    }
    if (device < 0 || device >= nd || device >= kMaxDevices) return HGS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return HGS_E_HIP;
    void* scr = nullptr;
    if (scratch_address(device, &scr) != hipSuccess) {
        (void)hipGetLastError();
        return HGS_E_HIP;
    }
    hgs_ctx* c = new (std::nothrow) hgs_ctx();
    if (!c) return HGS_E_OOM;
    c->device = device;
    c->scratch = scr;
    if (ensure(c, c->counters, sizeof(Counters) * kMaxViews) != HGS_OK ||
        hipHostMalloc((void**)&c->ctr_host, sizeof(Counters) * kMaxViews, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->views_copied, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&c->dimg_host, sizeof(ImgGrad) * kMaxViews, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->dimg_copied, hipEventDisableTiming) != hipSuccess) {
        hgs_destroy(c);
        return HGS_E_HIP;
    }
    std::memset(c->ctr_host, 0, sizeof(Counters) * kMaxViews);
    *out = c;
    return HGS_OK;
}

void hgs_destroy(hgs_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    DevMem* all[] = {&c->geo, &c->sh, &c->bound, &c->child, &c->leaf_ids, &c->parent, &c->nodefeat, &c->lvl,
                     &c->train_scratch, &c->region_dev, &c->surf, &c->views,
                     &c->tile_view, &c->mlp_w, &c->mlp_w32, &c->mlp_dev, &c->ranges,
                     &c->counters, &c->sort_k, &c->sort_v, &c->sort_n, &c->sort_hist, &c->px_state, &c->nav_goals, &c->nav_flags,
                     &c->nav_active, &c->nav_steps, &c->egrad, &c->dimg, &c->brec};
    for (DevMem* m : all) release(*m);
    for (Work& w : c->w) release_work(w);
    if (c->lane_stream) (void)hipStreamDestroy(c->lane_stream);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    for (auto& e : c->bwd_ev)
        for (hipEvent_t x : e) (void)hipEventDestroy(x);
    if (c->nav_active_host) (void)hipHostFree(c->nav_active_host);
    if (c->views_host) (void)hipHostFree(c->views_host);
    if (c->ctr_host) (void)hipHostFree(c->ctr_host);
    if (c->views_copied) (void)hipEventDestroy(c->views_copied);
    if (c->dimg_copied) (void)hipEventDestroy(c->dimg_copied);
    if (c->dimg_host) (void)hipHostFree(c->dimg_host);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    invalidate_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

const char* hgs_last_error(const hgs_ctx* c) { return c ? c->err.c_str() : "no context"; }

hgs_status hgs_load_scene(hgs_ctx* c, const hgs_gaussians* g, const hgs_hierarchy* h) {
    if (!c) return HGS_E_INVALID;
    std::string why;
    hgs_status s = hgs::validate_scene(g, h, &why);
    if (s != HGS_OK) return fail(c, s, "%s", why.c_str());
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t n = g->n;
    const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
    // host-side re-layout: geo = 3 float4 per Gaussian; SH as given, the
    // 3 K coefficients of a Gaussian contiguous ([g][k][c])
    std::vector<float4> geo((size_t)n * 3);
    for (int64_t i = 0; i < n; ++i) {
        geo[3 * i] = make_float4(g->means[3 * i], g->means[3 * i + 1], g->means[3 * i + 2], g->opacity[i]);
        geo[3 * i + 1] = make_float4(g->quats[4 * i], g->quats[4 * i + 1], g->quats[4 * i + 2], g->quats[4 * i + 3]);
        geo[3 * i + 2] = make_float4(g->scales[3 * i], g->scales[3 * i + 1], g->scales[3 * i + 2], 0.f);
    }
    std::vector<float> sh(g->sh, g->sh + (size_t)n * K * 3);
    double mlo[3] = {0, 0, 0}, mhi[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            const double x = g->means[3 * i + k];
            mlo[k] = i == 0 ? x : std::min(mlo[k], x);
            mhi[k] = i == 0 ? x : std::max(mhi[k], x);
        }
    // new buffers first, so a failure leaves the old scene intact
    DevMem ngeo, nsh, nbound, nchild, nleaf, nparent, nfeat, nlvl;
    auto cleanup = [&]() {
        release(ngeo); release(nsh); release(nbound); release(nchild); release(nleaf); release(nparent); release(nfeat);
        release(nlvl);
    };
    if ((s = ensure(c, ngeo, geo.size() * sizeof(float4))) || (s = ensure(c, nsh, sh.size() * sizeof(float)))) {
        cleanup();
        return s;
    }
    hipError_t e = hipMemcpy(ngeo.p, geo.data(), geo.size() * sizeof(float4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(nsh.p, sh.data(), sh.size() * sizeof(float), hipMemcpyHostToDevice);
    std::vector<int64_t> lo;
    int64_t n_leaves = n;
    if (e == hipSuccess && h) {
        std::vector<float4> bound((size_t)n);
        std::vector<int2> child((size_t)n);
        std::vector<int32_t> leaves;
        std::vector<float4> feat((size_t)n * 3);
        for (int64_t i = 0; i < n; ++i) {
            bound[i] = make_float4(h->bound[4 * i], h->bound[4 * i + 1], h->bound[4 * i + 2], h->bound[4 * i + 3]);
            child[i] = make_int2(h->child_count[i] > 0 ? h->first_child[i] : 0, h->child_count[i]);
            if (h->child_count[i] == 0) leaves.push_back((int32_t)i);
        }
        // learned-LOD node record (three float4): thinnest axis and children's
        // colour variance; the parent's bounding sphere (radius -1: a root);
        // opacity and child count
        for (int64_t i = 0; i < n; ++i) {
            const float* q = g->quats + 4 * i;
            const double qn = std::sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
            const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
            const float* sc = g->scales + 3 * i;
            const int a = (sc[0] <= sc[1] && sc[0] <= sc[2]) ? 0 : (sc[1] <= sc[2] ? 1 : 2);
            double col[3];
            if (a == 0) { col[0] = 1 - 2 * (y * y + z * z); col[1] = 2 * (x * y + w * z); col[2] = 2 * (x * z - w * y); }
            else if (a == 1) { col[0] = 2 * (x * y - w * z); col[1] = 1 - 2 * (x * x + z * z); col[2] = 2 * (y * z + w * x); }
            else { col[0] = 2 * (x * z + w * y); col[1] = 2 * (y * z - w * x); col[2] = 1 - 2 * (x * x + y * y); }
            double var = 0.0;
            const int32_t cc = h->child_count[i];
            if (cc > 1) {
                double m[3] = {0, 0, 0}, m2 = 0;
                for (int32_t j = 0; j < cc; ++j) {
                    const int64_t ch = h->first_child[i] + j;
                    for (int k = 0; k < 3; ++k) {
                        const double v = g->sh[(size_t)ch * K * 3 + k];
                        m[k] += v;
                        m2 += v * v;
                    }
                }
                var = m2 / cc - (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / ((double)cc * cc);
                var *= 0.28209479177387814 * 0.28209479177387814;
            }
            feat[3 * i] = make_float4((float)col[0], (float)col[1], (float)col[2], (float)std::max(var, 0.0));
            const int32_t par = h->parent[i];
            feat[3 * i + 1] = par >= 0 ? bound[par] : make_float4(0.f, 0.f, 0.f, -1.f);
            feat[3 * i + 2] = make_float4(g->opacity[i], (float)cc, 0.f, 0.f);
        }
        if ((s = ensure(c, nbound, bound.size() * sizeof(float4))) || (s = ensure(c, nchild, child.size() * sizeof(int2))) ||
            (s = ensure(c, nleaf, leaves.size() * sizeof(int32_t))) || (s = ensure(c, nparent, (size_t)n * 4)) ||
            (s = ensure(c, nfeat, feat.size() * sizeof(float4))) ||
            (s = ensure(c, nlvl, sizeof(int64_t) * (size_t)(h->n_levels + 1)))) {
            cleanup();
            return s;
        }
        e = hipMemcpy(nbound.p, bound.data(), bound.size() * sizeof(float4), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(nchild.p, child.data(), child.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(nleaf.p, leaves.data(), leaves.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(nparent.p, h->parent, (size_t)n * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(nfeat.p, feat.data(), feat.size() * sizeof(float4), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(nlvl.p, h->level_offset, sizeof(int64_t) * (size_t)(h->n_levels + 1), hipMemcpyHostToDevice);
        lo.assign(h->level_offset, h->level_offset + h->n_levels + 1);
        n_leaves = (int64_t)leaves.size();
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(c, HGS_E_HIP, "scene upload failed: %s", hipGetErrorString(e));
    }
    release(c->geo); release(c->sh); release(c->bound); release(c->child); release(c->leaf_ids);
    release(c->parent); release(c->nodefeat); release(c->lvl);
    c->geo = ngeo; c->sh = nsh; c->bound = nbound; c->child = nchild; c->leaf_ids = nleaf;
    c->parent = nparent; c->nodefeat = nfeat; c->lvl = nlvl;
    invalidate_graph(c);
    c->hier = h != nullptr;
    c->n = n;
    c->sh_degree = g->sh_degree;
    c->level_offset = lo;
    c->n_levels = h ? h->n_levels : 0;
    c->n_leaves = n_leaves;
    for (int k = 0; k < 3; ++k) {
        c->mean_lo[k] = mlo[k];
        c->mean_hi[k] = mhi[k];
    }
    c->depth_full = false;
    c->loaded = true;
    c->mlp_loaded = false;
    c->last_valid = false;
    if (!c->cams.empty()) {
        initial_caps(c);
        if ((s = alloc_work(c))) return s;
    }
    return HGS_OK;
}

hgs_status hgs_set_cameras(hgs_ctx* c, int32_t n, const hgs_camera* cams) {
    if (!c) return HGS_E_INVALID;
    if (n < 1 || n > kMaxViews || !cams) return fail(c, HGS_E_INVALID, "need 1..%d cameras", kMaxViews);
    for (int v = 0; v < n; ++v) {
        const hgs_camera& k = cams[v];
        if (k.width < 1 || k.height < 1 || k.width > 8192 || k.height > 8192)
            return fail(c, HGS_E_INVALID, "camera %d: size must be 1..8192", v);
        if (!(k.fx > 0.f) || !(k.fy > 0.f) || !finite(k.cx) || !finite(k.cy) || !(k.znear > 0.f) || !finite(k.znear))
            return fail(c, HGS_E_INVALID, "camera %d: focal lengths and znear must be positive", v);
        for (int i = 0; i < 9; ++i)
            if (!finite(k.R[i])) return fail(c, HGS_E_INVALID, "camera %d: rotation not finite", v);
        for (int i = 0; i < 3; ++i)
            if (!finite(k.position[i]) || !finite(k.bg[i])) return fail(c, HGS_E_INVALID, "camera %d: position/bg not finite", v);
    }
    HIP_TRY(c, hipSetDevice(c->device));
    // tile layout: views in order, row-major tiles within a view
    const int tw = c->ropts.tile_w, th = c->ropts.tile_h;
    uint64_t tiles = 0, max_tiles = 1;
    std::vector<uint32_t> tile_base(n);
    for (int v = 0; v < n; ++v) {
        tile_base[v] = (uint32_t)tiles;
        const uint64_t t = (uint64_t)((cams[v].width + tw - 1) / tw) * ((cams[v].height + th - 1) / th);
        tiles += t;
        max_tiles = std::max(max_tiles, t);
    }
    if (tiles >= (1ull << 31) || !pair_keys_fit(n, max_tiles)) return fail(c, HGS_E_UNSUPPORTED, "too many tiles");
    // same view count and image sizes as before: the tile layout, its device
    // table and a captured render stay valid (camera poses live in device
    // memory uploaded before each render)
    bool same_layout = (int)c->cams.size() == n;
    for (int v = 0; same_layout && v < n; ++v)
        same_layout = c->cams[v].width == cams[v].width && c->cams[v].height == cams[v].height;
    hgs_status s;
    if ((s = ensure(c, c->views, sizeof(ViewDev) * n)) || (s = ensure(c, c->tile_view, tiles * 4)) ||
        (s = ensure(c, c->ranges, tiles * sizeof(uint2))))
        return s;
    if ((int)c->cams.size() < n || !c->views_host) {
        if (c->views_host) {
            HIP_TRY(c, hipEventSynchronize(c->views_copied));
            (void)hipHostFree(c->views_host);
        }
        c->views_host = nullptr;
        HIP_TRY(c, hipHostMalloc((void**)&c->views_host, sizeof(ViewDev) * n, hipHostMallocDefault));
    } else {
        HIP_TRY(c, hipEventSynchronize(c->views_copied));
    }
    for (int v = 0; v < n; ++v) {
        const hgs_camera& k = cams[v];
        ViewDev d{};
        for (int i = 0; i < 3; ++i) d.o[i] = (double)k.position[i];
        for (int i = 0; i < 9; ++i) d.R[i] = (double)k.R[i];
        d.fx = k.fx; d.fy = k.fy; d.cx = k.cx; d.cy = k.cy;
        d.W = (double)k.width; d.H = (double)k.height; d.znear = k.znear;
        d.f2 = 2.0 * std::max(d.fx, d.fy);
        d.tau2 = (double)c->tau * (double)c->tau;
        d.tau = (double)c->tau;
        {
            // same arithmetic order as the device node test (no contraction:
            // these are single products and sums)
            volatile double a = d.fx * d.fx, b = d.cx * d.cx;
            d.nl = a + b;
            const double cxw = d.cx - d.W;
            volatile double b2 = cxw * cxw;
            d.nr = a + b2;
            volatile double e = d.fy * d.fy, f = d.cy * d.cy;
            d.nt = e + f;
            const double cyh = d.cy - d.H;
            volatile double f2 = cyh * cyh;
            d.nb = e + f2;
        }
        d.xlo = (-d.cx - 0.15 * d.W) / d.fx;
        d.xhi = (d.W - d.cx + 0.15 * d.W) / d.fx;
        d.ylo = (-d.cy - 0.15 * d.H) / d.fy;
        d.yhi = (d.H - d.cy + 0.15 * d.H) / d.fy;
        for (int i = 0; i < 3; ++i) d.bg[i] = k.bg[i];
        d.width = k.width; d.height = k.height;
        d.tiles_x = (k.width + tw - 1) / tw;
        d.tiles_y = (k.height + th - 1) / th;
        d.tile_base = tile_base[v];
        d.keep_node = -1;
        d.rgb = d.depth = d.alpha = nullptr;
        c->views_host[v] = d;
    }
    c->cams.assign(cams, cams + n);
    c->total_tiles = (uint32_t)tiles;
    c->tile_abs = tile_base;
    if ((s = plan_passes(c, same_layout ? c->want_passes : 1, !same_layout))) return s;
    c->views_dirty = true;
    c->last_valid = false;
    if (c->loaded) {
        initial_caps(c);
        if ((s = alloc_work(c))) return s;
    }
    return HGS_OK;
}

hgs_status hgs_set_lod(hgs_ctx* c, int32_t mode, float tau) {
    if (!c) return HGS_E_INVALID;
    if (mode < HGS_LOD_ALL_LEAVES || mode > HGS_LOD_LEARNED) return fail(c, HGS_E_INVALID, "unknown LOD mode %d", mode);
    if (!(tau > 0.f) || !finite(tau)) return fail(c, HGS_E_INVALID, "tau must be a positive number");
    if (mode == HGS_LOD_LEARNED && !c->mlp_loaded) return fail(c, HGS_E_STATE, "learned LOD needs hgs_load_lod_mlp first");
    invalidate_graph(c);
    c->lod_mode = mode;
    c->tau = tau;
    if (c->views_host) HIP_TRY(c, hipEventSynchronize(c->views_copied));
    for (size_t v = 0; c->views_host && v < c->cams.size(); ++v) {
        c->views_host[v].tau2 = (double)tau * (double)tau;
        c->views_host[v].tau = (double)tau;
    }
    c->views_dirty = true;
    return HGS_OK;
}

namespace {

// Tile layout of the views already set, for a new tile shape: per-view tile
// counts, the views' tile bases and the tile -> view table (the device
// mirror of the views is uploaded again before the next render).
hgs_status relayout_tiles(hgs_ctx* c) {
    const int V = (int)c->cams.size();
    if (V == 0) return HGS_OK;
    const int tw = c->ropts.tile_w, th = c->ropts.tile_h;
    uint64_t tiles = 0, max_tiles = 1;
    std::vector<uint32_t> base(V);
    for (int v = 0; v < V; ++v) {
        base[v] = (uint32_t)tiles;
        const uint64_t t = (uint64_t)((c->cams[v].width + tw - 1) / tw) * ((c->cams[v].height + th - 1) / th);
        tiles += t;
        max_tiles = std::max(max_tiles, t);
    }
    if (tiles >= (1ull << 31) || !pair_keys_fit(V, max_tiles)) return fail(c, HGS_E_UNSUPPORTED, "too many tiles");
    hgs_status s;
    if ((s = ensure(c, c->tile_view, tiles * 4)) || (s = ensure(c, c->ranges, tiles * sizeof(uint2)))) return s;
    HIP_TRY(c, hipEventSynchronize(c->views_copied));
    for (int v = 0; v < V; ++v) {
        c->views_host[v].tiles_x = (c->cams[v].width + tw - 1) / tw;
        c->views_host[v].tiles_y = (c->cams[v].height + th - 1) / th;
    }
    c->total_tiles = (uint32_t)tiles;
    c->tile_abs = base;
    c->last_valid = false;
    return plan_passes(c, c->want_passes, true);
}

}  // namespace

hgs_status hgs_set_option(hgs_ctx* c, int32_t opt, int64_t val) {
    if (!c) return HGS_E_INVALID;
    invalidate_graph(c);
    switch (opt) {
        case HGS_OPT_SYNC_CHECK: c->sync_check = val != 0; return HGS_OK;
        case HGS_OPT_AUTO_REGROW: c->auto_regrow = val != 0; return HGS_OK;
        case HGS_OPT_COUNT_NALG: c->ropts.count_nalg = val != 0; return HGS_OK;
        case HGS_OPT_BATCH_DEPTH:
            if (val != 64 && val != 128 && val != 256) return fail(c, HGS_E_INVALID, "batch depth must be 64, 128 or 256");
            c->ropts.batch = (int)val;
            return HGS_OK;
        case HGS_OPT_USE_GRAPH: c->use_graph = val != 0; return HGS_OK;
        case HGS_OPT_PERSISTENT: c->ropts.persistent = val != 0; return HGS_OK;
        case HGS_OPT_EXACT_TILES: c->ropts.exact_tiles = val != 0; return HGS_OK;
        case HGS_OPT_LOD_BLEND: c->ropts.lod_blend = val != 0; return HGS_OK;
        case HGS_OPT_KEEP_STATE:
            if (val != 0 && (c->ropts.tile_w != kTile || c->ropts.tile_h != kTile))
                return fail(c, HGS_E_UNSUPPORTED, "kept pixel states need %dx%d tiles", kTile, kTile);
            c->ropts.keep_state = val != 0;
            return HGS_OK;
        case HGS_OPT_TILE_SHAPE: {
            const int tw = (int)(val >> 16), th = (int)(val & 0xffff);
            if (val < 0 || !tile_shape_ok(tw, th, 1) || !tile_shape_ok(tw, th, c->ropts.px))
                return fail(c, HGS_E_INVALID, "tile shape %dx%d is not one of 8x8, 16x8, 16x16, 32x8, 32x16 "
                            "(or does not allow %d pixels per thread)", tw, th, c->ropts.px);
            if (c->ropts.keep_state && (tw != kTile || th != kTile))
                return fail(c, HGS_E_UNSUPPORTED, "kept pixel states need %dx%d tiles", kTile, kTile);
            if (tw == c->ropts.tile_w && th == c->ropts.tile_h) return HGS_OK;
            c->ropts.tile_w = tw;
            c->ropts.tile_h = th;
            return relayout_tiles(c);
        }
        case HGS_OPT_PIXELS_PER_THREAD:
            if (!tile_shape_ok(c->ropts.tile_w, c->ropts.tile_h, (int)val))
                return fail(c, HGS_E_INVALID, "%lld pixels per thread: 1, 2 or 4, at least 64 threads per %dx%d tile",
                            (long long)val, c->ropts.tile_w, c->ropts.tile_h);
            c->ropts.px = (int)val;
            return HGS_OK;
        case HGS_OPT_LANES: {
            if (val != 1 && val != 2) return fail(c, HGS_E_INVALID, "lanes must be 1 or 2");
            if (val == 2 && !c->lane_stream) {
                HIP_TRY(c, hipSetDevice(c->device));
                HIP_TRY(c, hipStreamCreateWithFlags(&c->lane_stream, hipStreamNonBlocking));
                HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
                HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
            }
            c->lanes = (int)val;
            invalidate_graph(c);
            if (c->lanes == 1) {
                HIP_TRY(c, hipDeviceSynchronize());
                release_work(c->w[1]);
            }
            if (c->loaded && !c->cams.empty()) {
                hgs_status st = alloc_work(c);
                if (st) return st;
            }
            if (!c->cams.empty()) return plan_passes(c, c->lanes, false);
            return HGS_OK;
        }
        case HGS_OPT_PASS_VIEWS:
            if (val < 0 || val > kMaxViews) return fail(c, HGS_E_INVALID, "views per pass must be 0..%d", kMaxViews);
            c->pass_views = (int)val;
            if (!c->cams.empty()) return plan_passes(c, 1, true);
            return HGS_OK;
        case HGS_OPT_SORT_DIGIT_BITS:
            if (val < 6 || val > 11) return fail(c, HGS_E_INVALID, "digit bits must be 6..11");
            c->sort_digit_bits = (int)val;
            return HGS_OK;
        case HGS_OPT_STAGE_TIMING: {
            hgs_status s = harvest_events(c);
            if (s) return s;
            c->stage_timing = val != 0;
            for (double& a : c->acc_ms) a = 0;
            c->acc_n = 0;
            c->bwd_ms[0] = c->bwd_ms[1] = 0;
            c->bwd_n = 0;
            return HGS_OK;
        }
        case HGS_OPT_INITIAL_CAPACITY: {
            if (val < 0 || val > 0x7fffffff) return fail(c, HGS_E_INVALID, "capacity out of range");
            c->forced_cap = (uint32_t)val;
            if (c->forced_cap) {
                // shrink: drop the work buffers so they are re-made at this size
                HIP_TRY(c, hipDeviceSynchronize());
                for (Work& w : c->w) release_work(w);
                c->frontier_cap = c->cut_cap = c->pair_cap = 0;
                if (c->loaded && !c->cams.empty()) {
                    initial_caps(c);
                    hgs_status s = alloc_work(c);
                    if (s) return s;
                }
            }
            return HGS_OK;
        }
        default: return fail(c, HGS_E_INVALID, "unknown option %d", opt);
    }
}

hgs_status hgs_render(hgs_ctx* c, void* stream, const hgs_output* outs) {
    if (!c) return HGS_E_INVALID;
    if (!c->loaded) return fail(c, HGS_E_STATE, "no scene loaded");
    if (c->cams.empty()) return fail(c, HGS_E_STATE, "no cameras set");
    if (!outs) return fail(c, HGS_E_INVALID, "outs is NULL");
    for (size_t v = 0; v < c->cams.size(); ++v)
        if (!outs[v].rgb) return fail(c, HGS_E_INVALID, "view %zu: rgb output is NULL", v);
    if (c->lod_mode == HGS_LOD_LEARNED && !c->mlp_loaded) return fail(c, HGS_E_STATE, "learned LOD without a network");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    hgs_status st;
    if ((st = upload_views(c, s, outs))) return st;
    if (c->ropts.keep_state) {
        void* before = c->px_state.p;
        if ((st = ensure(c, c->px_state, (size_t)c->total_tiles * kTilePx * sizeof(uint2)))) return st;
        if (c->px_state.p != before) invalidate_graph(c);
    }
    c->regrows = 0;
    for (int attempt = 0; attempt < 16; ++attempt) {
        if (c->use_graph && !c->stage_timing) {
            if (!c->graph_valid) {
                invalidate_graph(c);
                if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                enqueue_render(c, c->cap_stream);
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(c->cap_stream, &g);
                if (ce != hipSuccess) return fail(c, HGS_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
                c->graph = g;
                HIP_TRY(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
                c->graph_valid = true;
            }
            HIP_TRY(c, hipGraphLaunch(c->gexec, s));
            ++c->graph_launches;
        } else {
            enqueue_render(c, s);
        }
        HIP_TRY(c, hipGetLastError());
        c->last_valid = true;
        if (!c->sync_check) return HGS_OK;
        if ((st = read_counters(c, s))) return st;
        uint64_t need_sum = 0;
        const Counters k = merge_passes(c, &need_sum);
        if (!k.overflow) return HGS_OK;
        c->last_valid = false;
        if (!c->auto_regrow) {
            grow_from(c, k);
            return fail(c, HGS_E_CAPACITY, "work buffers overflowed (bits %u); capacities grown", k.overflow);
        }
        const int np = n_passes(c);
        const bool too_big = (uint64_t)k.need_cut >= kEntryLimit || (uint64_t)k.need_pairs > kPairLimit ||
                             (uint64_t)k.need_frontier > kPairLimit;
        if (too_big && np < (int)c->cams.size()) {
            // a pass outgrew the index space: more, smaller passes
            const uint64_t est = (3 * need_sum) / (2 * kEntryLimit) + 1;
            if ((st = plan_passes(c, (int)std::max<uint64_t>(2 * np, est), false))) return st;
            ++c->regrows;
        } else if ((st = grow_from(c, k))) {
            return st;
        }
        if ((st = upload_views(c, s, outs))) return st;
    }
    const Counters k = merge_passes(c, nullptr);
    return fail(c, HGS_E_CAPACITY, "work buffers kept overflowing (bits %u; need cut %u, pairs %u, frontier %u; "
                "caps %u, %u, %u; %d passes)", k.overflow, k.need_cut, k.need_pairs, k.need_frontier, c->cut_cap,
                c->pair_cap, c->frontier_cap, n_passes(c));
}

hgs_status hgs_check(hgs_ctx* c) {
    if (!c) return HGS_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpy(c->ctr_host, c->counters.p, sizeof(Counters) * n_passes(c), hipMemcpyDeviceToHost));
    const Counters k = merge_passes(c, nullptr);
    if (k.overflow) {
        c->last_valid = false;
        hgs_status s = grow_from(c, k);
        if (s) return s;
        return fail(c, HGS_E_CAPACITY, "work buffers overflowed (bits %u); capacities grown", k.overflow);
    }
    return HGS_OK;
}

hgs_status hgs_get_cut(hgs_ctx* c, int32_t view, int32_t* ids, int64_t cap, int64_t* count) {
    if (!c || !count) return HGS_E_INVALID;
    if (!c->last_valid) return fail(c, HGS_E_STATE, "no valid render");
    if (view < 0 || view >= (int)c->cams.size()) return fail(c, HGS_E_INVALID, "view out of range");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    const int last = n_passes(c) - 1, vb = c->pass_v0[last];
    if (view < vb)
        return fail(c, HGS_E_STATE, "view %d was rendered in an earlier pass of the batch; only the last pass "
                    "(views %d..%d) keeps its intermediates", view, vb, (int)c->cams.size() - 1);
    HIP_TRY(c, hipMemcpy(c->ctr_host, c->counters.p, sizeof(Counters) * (last + 1), hipMemcpyDeviceToHost));
    const uint32_t m = std::min(c->ctr_host[last].cut, c->cut_cap);
    const uint32_t vrel = (uint32_t)(view - vb);
    std::vector<uint2> e(m);
    if (m) HIP_TRY(c, hipMemcpy(e.data(), c->w[c->last_lane].cut.p, (size_t)m * sizeof(uint2), hipMemcpyDeviceToHost));
    int64_t k = 0;
    for (uint32_t i = 0; i < m; ++i)
        if (e[i].y == vrel) {
            if (ids && k < cap) ids[k] = (int32_t)e[i].x;
            ++k;
        }
    *count = k;
    return HGS_OK;
}

hgs_status hgs_get_projected(hgs_ctx* c, int32_t view, float* out, int64_t cap, int64_t* count) {
    if (!c || !count) return HGS_E_INVALID;
    if (!c->last_valid) return fail(c, HGS_E_STATE, "no valid render");
    if (view < 0 || view >= (int)c->cams.size()) return fail(c, HGS_E_INVALID, "view out of range");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    const int last = n_passes(c) - 1, vb = c->pass_v0[last];
    if (view < vb)
        return fail(c, HGS_E_STATE, "view %d was rendered in an earlier pass of the batch; only the last pass "
                    "(views %d..%d) keeps its intermediates", view, vb, (int)c->cams.size() - 1);
    HIP_TRY(c, hipMemcpy(c->ctr_host, c->counters.p, sizeof(Counters) * (last + 1), hipMemcpyDeviceToHost));
    const uint32_t m = std::min(c->ctr_host[last].cut, c->cut_cap);
    const uint32_t vrel = (uint32_t)(view - vb);
    std::vector<uint2> e(m);
    std::vector<Proj> p(m);
    std::vector<uint32_t> nt(m);
    if (m) {
        const Work& W = c->w[c->last_lane];
        HIP_TRY(c, hipMemcpy(e.data(), W.cut.p, (size_t)m * sizeof(uint2), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(p.data(), W.proj.p, (size_t)m * sizeof(Proj), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(nt.data(), W.ntiles.p, (size_t)m * 4, hipMemcpyDeviceToHost));
    }
    int64_t k = 0;
    for (uint32_t i = 0; i < m; ++i) {
        if (e[i].y != vrel) continue;
        if (out && k < cap) {
            float* o = out + 12 * k;
            const Proj& q = p[i];
            const double A = (double)q.p * q.p, B = (double)q.p * q.r, C = (double)q.r * q.r + (double)q.s * q.s;
            o[0] = (float)q.u; o[1] = (float)q.v; o[2] = (float)A; o[3] = (float)B; o[4] = (float)C;
            o[5] = q.c0; o[6] = q.c1; o[7] = q.c2; o[8] = q.z; o[9] = q.opacity;
            o[10] = (float)nt[i];
            o[11] = q.p > 0.f ? 1.f : 0.f;
        }
        ++k;
    }
    *count = k;
    return HGS_OK;
}

hgs_status hgs_get_stats(hgs_ctx* c, hgs_stats* out) {
    if (!c || !out) return HGS_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    const int np = n_passes(c);
    HIP_TRY(c, hipMemcpy(c->ctr_host, c->counters.p, sizeof(Counters) * np, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    for (int g = 0; g < np; ++g) {
        const Counters& k = c->ctr_host[g];
        out->cut_size += std::min(k.cut, c->cut_cap);
        out->visible += k.visible;
        out->pairs += std::min(k.pairs, c->pair_cap);
        out->n_alg += (int64_t)k.nalg;
        out->n_eval += (int64_t)k.neval;
        out->visited += (int64_t)k.visited;
    }
    out->passes = np;
    out->tiles = c->total_tiles;
    out->regrows = c->regrows;
    hgs_status s = harvest_events(c);
    if (s) return s;
    out->timed_renders = c->acc_n;
    out->graph_launches = c->graph_launches;
    out->ms_cut = c->acc_ms[0];
    out->ms_project = c->acc_ms[1];
    out->ms_sort = c->acc_ms[2];
    out->ms_composite = c->acc_ms[3];
    out->ms_total = c->acc_ms[4];
    out->timed_backwards = c->bwd_n;
    out->ms_bwd_composite = c->bwd_ms[0];
    out->ms_bwd_total = c->bwd_ms[1];
    return HGS_OK;
}

hgs_status hgs_autotune(hgs_ctx* c, void* stream, const char* cache_path, int32_t reps, hgs_plan* out) {
    if (!c) return HGS_E_INVALID;
    if (reps < 1 || reps > 1000) return fail(c, HGS_E_INVALID, "reps must be 1..1000");
    if (!c->loaded || c->cams.empty()) return fail(c, HGS_E_STATE, "autotune needs a scene and cameras");
    if (c->lod_mode == HGS_LOD_LEARNED && !c->mlp_loaded) return fail(c, HGS_E_STATE, "learned LOD without a network");
    HIP_TRY(c, hipSetDevice(c->device));
    const std::string key = plan_key(c);
    hgs_plan best{};
    if (read_plan(cache_path, key, &best) &&
        (!c->ropts.keep_state || (best.tile_w == kTile && best.tile_h == kTile))) {
        hgs_status st;
        if ((st = hgs_set_option(c, HGS_OPT_PIXELS_PER_THREAD, 1)) ||
            (st = hgs_set_option(c, HGS_OPT_TILE_SHAPE, ((int64_t)best.tile_w << 16) | best.tile_h)) ||
            (st = hgs_set_option(c, HGS_OPT_PIXELS_PER_THREAD, best.pixels_per_thread)) ||
            (st = hgs_set_option(c, HGS_OPT_BATCH_DEPTH, best.batch_depth)) ||
            (st = hgs_set_option(c, HGS_OPT_PERSISTENT, best.persistent)) ||
            (st = hgs_set_option(c, HGS_OPT_SORT_DIGIT_BITS, best.sort_digit_bits)))
            return st;
        best.lanes = c->lanes;
        best.from_cache = 1;
        if (out) *out = best;
        return HGS_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    // internal outputs for every view
    const int V = (int)c->cams.size();
    size_t px = 0;
    for (const hgs_camera& k : c->cams) px += (size_t)k.width * k.height;
    DevMem buf;
    hgs_status st = ensure(c, buf, px * 5 * sizeof(float));
    if (st) return st;
    std::vector<hgs_output> outs(V);
    {
        float* p = static_cast<float*>(buf.p);
        for (int v = 0; v < V; ++v) {
            const size_t n = (size_t)c->cams[v].width * c->cams[v].height;
            outs[v].rgb = p;
            outs[v].depth = p + 3 * n;
            outs[v].alpha = p + 4 * n;
            p += 5 * n;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool graph = c->use_graph, timing = c->stage_timing, sync = c->sync_check;
    auto restore = [&]() {
        c->use_graph = graph;
        c->sync_check = sync;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        release(buf);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        restore();
        return fail(c, HGS_E_HIP, "event creation failed");
    }
    if (timing && (st = hgs_set_option(c, HGS_OPT_STAGE_TIMING, 0))) {
        restore();
        return st;
    }
    c->use_graph = false;
    c->sync_check = true;
    invalidate_graph(c);
    // a plan: tile shape, pixels per thread, batch depth, persistent, digit width
    auto apply = [&](int tw, int th, int px, int batch, int pers, int digits) -> hgs_status {
        c->ropts.px = 1;
        if (tw != c->ropts.tile_w || th != c->ropts.tile_h) {
            c->ropts.tile_w = tw;
            c->ropts.tile_h = th;
            hgs_status r = relayout_tiles(c);
            if (r) return r;
        }
        c->ropts.px = px;
        c->ropts.batch = batch;
        c->ropts.persistent = pers != 0;
        c->sort_digit_bits = digits;
        return HGS_OK;
    };
    auto run = [&](int tw, int th, int px, int batch, int pers, int digits, double* ms) -> hgs_status {
        hgs_status r = apply(tw, th, px, batch, pers, digits);
        return r ? r : time_plan(c, s, outs.data(), reps, e0, e1, ms);
    };
    double ms_default = 0.0;
    if ((st = run(kTile, kTile, 1, 256, 0, 8, &ms_default))) {
        restore();
        return st;
    }
    best = hgs_plan{256, 0, 8, 0, ms_default, ms_default, c->lanes, 0, kTile, kTile, 1, 0};
    // compositor choices: every supported tile shape and pixels per thread
    // (kept pixel states: the default shape only), the batch depths a tile's
    // threads can stage (one entry each), persistent tiles for the default
    // shape
    const int shapes[5][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 8}, {32, 16}};
    const int batches[3] = {64, 128, 256};
    for (const auto& sh : shapes)
        for (int px = 1; px <= 4; px *= 2) {
            if (!tile_shape_ok(sh[0], sh[1], px)) continue;
            const bool deflt = sh[0] == kTile && sh[1] == kTile && px == 1;
            if (c->ropts.keep_state && !deflt) continue;
            for (int b : batches) {
                if (b > sh[0] * sh[1] / px) continue;
                for (int pers = 0; pers < (deflt ? 2 : 1); ++pers) {
                    if (deflt && b == 256 && pers == 0) continue;
                    double ms;
                    if ((st = run(sh[0], sh[1], px, b, pers, best.sort_digit_bits, &ms))) {
                        restore();
                        return st;
                    }
                    if (ms < best.ms) {
                        best.tile_w = sh[0];
                        best.tile_h = sh[1];
                        best.pixels_per_thread = px;
                        best.batch_depth = b;
                        best.persistent = pers;
                        best.ms = ms;
                    }
                }
            }
        }
    for (int d = 6; d <= 11; ++d) {
        if (d == best.sort_digit_bits) continue;
        double ms;
        if ((st = run(best.tile_w, best.tile_h, best.pixels_per_thread, best.batch_depth, best.persistent, d, &ms))) {
            restore();
            return st;
        }
        if (ms < best.ms) { best.sort_digit_bits = d; best.ms = ms; }
    }
    if ((st = apply(best.tile_w, best.tile_h, best.pixels_per_thread, best.batch_depth, best.persistent,
                    best.sort_digit_bits))) {
        restore();
        return st;
    }
    c->last_valid = false;           // the last render went to internal buffers
    restore();
    invalidate_graph(c);
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(c, HGS_E_INVALID, "cannot append to plan cache %s", cache_path);
        std::fprintf(f, "%s %d %d %d %.6f %.6f %d %d %d %d\n", key.c_str(), best.batch_depth, best.persistent,
                     best.sort_digit_bits, best.ms, best.ms_default, best.lanes, best.tile_w, best.tile_h,
                     best.pixels_per_thread);
        std::fclose(f);
    }
    if (out) *out = best;
    return HGS_OK;
}

hgs_status hgs_sort_pairs(hgs_ctx* c, void* stream, uint32_t* keys, uint32_t* vals, int64_t n, int32_t key_bits) {
    if (!c || (!keys && n > 0) || (!vals && n > 0)) return HGS_E_INVALID;
    if (n < 0 || n >= (int64_t)0xF0000000ll) return fail(c, HGS_E_INVALID, "n out of range");
    if (key_bits < 1 || key_bits > 32) return fail(c, HGS_E_INVALID, "key_bits must be 1..32");
    if (n == 0) return HGS_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    hgs_status st;
    if ((st = ensure(c, c->sort_k, (size_t)n * 4)) || (st = ensure(c, c->sort_v, (size_t)n * 4)) ||
        (st = ensure(c, c->sort_n, 4)) || (st = ensure(c, c->sort_hist, kSortHistBytes)))
        return st;
    const uint32_t nn = (uint32_t)n;
    HIP_TRY(c, hipMemcpyAsync(c->sort_n.p, &nn, 4, hipMemcpyHostToDevice, s));
    SortArgs a{};
    a.keys[0] = keys;
    a.keys[1] = P<uint32_t>(c->sort_k);
    a.vals[0] = vals;
    a.vals[1] = P<uint32_t>(c->sort_v);
    a.count = P<uint32_t>(c->sort_n);
    a.cap = nn;
    a.key_bits = key_bits;
    a.max_digit_bits = c->sort_digit_bits;
    a.hist = P<uint32_t>(c->sort_hist);
    const int r = launch_sort(a, s);
    if (r == 1) {
        HIP_TRY(c, hipMemcpyAsync(keys, a.keys[1], (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(vals, a.vals[1], (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    return HGS_OK;
}

hgs_status hgs_sort_pairs_noalloc(hgs_ctx* c, void* stream, uint32_t* keys, uint32_t* vals, int64_t n,
                                  int32_t key_bits) {
    if (!c || (!keys && n > 0) || (!vals && n > 0)) return HGS_E_INVALID;
    if (n < 0 || n > (int64_t)kStaticSortMax)
        return fail(c, HGS_E_INVALID, "n = %lld is outside 0..%u, the pairs the static scratch area holds",
                    (long long)n, kStaticSortMax);
    if (key_bits < 1 || key_bits > 32) return fail(c, HGS_E_INVALID, "key_bits must be 1..32");
    if (n == 0) return HGS_OK;
    if (!c->scratch) return fail(c, HGS_E_STATE, "no scratch address for device %d", c->device);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    uint8_t* base = static_cast<uint8_t*>(c->scratch);
    SortArgs a{};
    a.keys[0] = keys;
    a.keys[1] = reinterpret_cast<uint32_t*>(base);
    a.vals[0] = vals;
    a.vals[1] = reinterpret_cast<uint32_t*>(base + kScratchPing);
    uint32_t* count = reinterpret_cast<uint32_t*>(base + 2 * kScratchPing);
    a.count = count;
    a.cap = (uint32_t)n;
    a.key_bits = key_bits;
    a.max_digit_bits = c->sort_digit_bits;
    a.hist = reinterpret_cast<uint32_t*>(base + kScratchHistOff);
    a.hist_stride = kStaticSortGroups;
    // the count of the previous call is still there: every call writes its own
    k_set_count<<<1, 64, 0, s>>>(count, (uint32_t)n);
    if (launch_sort(a, s) == 1) {
        const uint32_t grid = std::min<uint32_t>((uint32_t)((n + 255) / 256), 2048u);
        k_copy_pairs<<<grid, 256, 0, s>>>(a.keys[1], a.vals[1], keys, vals, (uint32_t)n);
    }
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_set_keep_nodes(hgs_ctx* c, int32_t n, const int32_t* nodes) {
    if (!c) return HGS_E_INVALID;
    if (n != (int32_t)c->cams.size() || !nodes) return fail(c, HGS_E_INVALID, "need one keep node per view");
    for (int v = 0; v < n; ++v)
        if (nodes[v] < -1 || nodes[v] >= c->n) return fail(c, HGS_E_INVALID, "keep node %d out of range", nodes[v]);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipEventSynchronize(c->views_copied));
    for (int v = 0; v < n; ++v) c->views_host[v].keep_node = nodes[v];
    c->views_dirty = true;
    return HGS_OK;
}

hgs_status hgs_lod_candidates(hgs_ctx* c, void* stream, float s_hi, uint32_t* entries, float* features, int32_t* rects,
                              int64_t cap, int64_t* count) {
    if (!c || !count) return HGS_E_INVALID;
    if (!c->loaded || !c->hier) return fail(c, HGS_E_STATE, "candidates need a hierarchical scene");
    if (c->cams.empty()) return fail(c, HGS_E_STATE, "no cameras set");
    if (!(s_hi > 0.f)) return fail(c, HGS_E_INVALID, "s_hi must be positive");
    if (cap < 0 || cap > 0xF0000000ll || (cap > 0 && (!entries || !features || !rects)))
        return fail(c, HGS_E_INVALID, "bad candidate buffers");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    hgs_status st;
    // the views' output pointers are not used by the cut; keep the mirror current
    std::vector<hgs_output> none(c->cams.size());
    for (size_t v = 0; v < none.size(); ++v) {
        none[v].rgb = c->views_host[v].rgb;
        none[v].depth = c->views_host[v].depth;
        none[v].alpha = c->views_host[v].alpha;
    }
    if ((st = upload_views(c, s, none.data()))) return st;
    for (int attempt = 0; attempt < 8; ++attempt) {
        Counters* ctr = P<Counters>(c->counters);
        k_reset<<<1, 64, 0, s>>>(ctr);
        CutArgs ca{};
        ca.bound = P<float4>(c->bound);
        ca.child = P<int2>(c->child);
        ca.leaf_ids = P<int32_t>(c->leaf_ids);
        ca.n_leaves = c->n_leaves;
        ca.n_nodes = c->n;
        ca.level_offset_host = c->level_offset.data();
        ca.n_levels = c->n_levels;
        ca.mode = HGS_LOD_THRESHOLD;
        ca.flat = false;
        ca.views = P<ViewDev>(c->views);
        ca.n_views = (int)c->cams.size();
        ca.frontier[0] = P<uint2>(c->w[0].frontier[0]);
        ca.frontier[1] = P<uint2>(c->w[0].frontier[1]);
        ca.frontier_cap = c->frontier_cap;
        ca.cut = P<uint2>(c->w[0].cut);
        ca.cut_cap = c->cut_cap;
        ca.scan_tmp = P<uint4>(c->w[0].scan_tmp);
        ca.dec = P<uint8_t>(c->w[0].dec);
        ca.ctr = ctr;
        ca.mlp = nullptr;
        ca.s_hi = s_hi;
        ca.cand = reinterpret_cast<uint2*>(entries);
        ca.cand_cap = (uint32_t)cap;
        launch_cut(ca, s);
        if (cap > 0) {
            LodMlpDev g = mlp_geometry(c);
            launch_lod_features(ca.cand, &ctr->cand, ca.views, &g, features, reinterpret_cast<int4*>(rects), s);
        }
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipMemcpyAsync(c->ctr_host, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        const Counters k = *c->ctr_host;
        if (k.overflow & (kOvFrontier | kOvCut)) {
            if ((st = grow_from(c, k))) return st;
            continue;
        }
        *count = (k.overflow & kOvCand) ? (int64_t)k.need_cand : (int64_t)k.cand;
        if (k.overflow & kOvCand) return fail(c, HGS_E_CAPACITY, "%lld candidates exceed the buffers", (long long)*count);
        return HGS_OK;
    }
    return fail(c, HGS_E_CAPACITY, "work buffers kept overflowing");
}

hgs_status hgs_load_lod_mlp(hgs_ctx* c, const uint16_t* bf16, const float* mean, const float* stdv, float p_star,
                            float s_hi) {
    if (!c) return HGS_E_INVALID;
    if (!c->loaded || !c->hier) return fail(c, HGS_E_STATE, "the learned cut needs a hierarchical scene");
    if (!bf16 || !mean || !stdv) return fail(c, HGS_E_INVALID, "NULL network arrays");
    if (!(p_star >= 0.f && p_star <= 1.f) || !(s_hi > 0.f)) return fail(c, HGS_E_INVALID, "bad p_star or s_hi");
    for (int i = 0; i < kMlpIn; ++i)
        if (!(stdv[i] > 0.f) || !finite(mean[i])) return fail(c, HGS_E_INVALID, "bad feature normalisation");
    for (int i = 0; i < kMlpParams; ++i) {
        const float w = bf16_to_f32_host(bf16[i]);
        if (!finite(w)) return fail(c, HGS_E_INVALID, "non-finite weight %d", i);
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hgs_status st;
    if ((st = ensure(c, c->mlp_w, kMlpParams * sizeof(uint16_t))) || (st = ensure(c, c->mlp_dev, sizeof(LodMlpDev))) ||
        (st = ensure(c, c->mlp_w32, kMlpParams * sizeof(float))))
        return st;
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(c->mlp_w.p, bf16, kMlpParams * sizeof(uint16_t), hipMemcpyHostToDevice));
    // the same weights widened to FP32 (exact), read by the cut's network pass
    std::vector<float> w32(kMlpParams);
    for (int i = 0; i < kMlpParams; ++i) w32[i] = bf16_to_f32_host(bf16[i]);
    HIP_TRY(c, hipMemcpy(c->mlp_w32.p, w32.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    LodMlpDev m = mlp_geometry(c);
    m.w = P<uint16_t>(c->mlp_w);
    for (int i = 0; i < kMlpIn; ++i) {
        m.mean[i] = mean[i];
        m.inv_std[i] = 1.f / stdv[i];
    }
    m.p_star = p_star;
    m.s_hi = s_hi;
    HIP_TRY(c, hipMemcpy(c->mlp_dev.p, &m, sizeof(LodMlpDev), hipMemcpyHostToDevice));
    invalidate_graph(c);
    c->mlp_host = m;
    c->s_hi = s_hi;
    c->mlp_loaded = true;
    return HGS_OK;
}

hgs_status hgs_mlp_forward(hgs_ctx* c, void* stream, const float* feats, int64_t n, const uint16_t* w, const float* mean,
                           const float* stdv, float* logits) {
    if (!c) return HGS_E_INVALID;
    if (n < 0 || n > 0x7fffffffll || (n > 0 && (!feats || !w || !logits)) || !mean || !stdv)
        return fail(c, HGS_E_INVALID, "bad arguments");
    for (int i = 0; i < kMlpIn; ++i)
        if (!(stdv[i] > 0.f)) return fail(c, HGS_E_INVALID, "bad feature normalisation");
    if (n == 0) return HGS_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    launch_mlp_forward(feats, (uint32_t)n, mean, stdv, w, logits, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_mlp_train_step(hgs_ctx* c, void* stream, const float* feats, const float* labels, int64_t n,
                              const float* mean, const float* stdv, float* master, uint16_t* w, float* adam_m,
                              float* adam_v, int32_t step, float lr, float* grad_out, float* loss_out) {
    if (!c) return HGS_E_INVALID;
    if (n <= 0 || n > (1ll << 24) || !feats || !labels || !mean || !stdv || !w)
        return fail(c, HGS_E_INVALID, "bad arguments");
    if (lr > 0.f && (!master || !adam_m || !adam_v || step < 1)) return fail(c, HGS_E_INVALID, "Adam needs state and step >= 1");
    if (lr < 0.f || !finite(lr)) return fail(c, HGS_E_INVALID, "lr must be >= 0");
    for (int i = 0; i < kMlpIn; ++i)
        if (!(stdv[i] > 0.f)) return fail(c, HGS_E_INVALID, "bad feature normalisation");
    HIP_TRY(c, hipSetDevice(c->device));
    hgs_status st;
    if ((st = ensure(c, c->train_scratch, mlp_train_scratch_floats((uint32_t)n) * sizeof(float)))) return st;
    launch_mlp_train_step(feats, labels, (uint32_t)n, mean, stdv, master, w, adam_m, adam_v, step, lr, grad_out,
                          loss_out, P<float>(c->train_scratch), (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_mlp_backward(hgs_ctx* c, void* stream, const float* feats, const float* labels, int64_t n,
                            const float* mean, const float* stdv, const uint16_t* w, float* grad_out,
                            float* loss_out) {
    if (!c) return HGS_E_INVALID;
    if (!grad_out) return fail(c, HGS_E_INVALID, "grad_out is required");
    return hgs_mlp_train_step(c, stream, feats, labels, n, mean, stdv, nullptr, const_cast<uint16_t*>(w), nullptr,
                              nullptr, 0, 0.f, grad_out, loss_out);
}

hgs_status hgs_mlp_adam(hgs_ctx* c, void* stream, const float* grad, float* master, uint16_t* w, float* adam_m,
                        float* adam_v, int32_t step, float lr) {
    if (!c) return HGS_E_INVALID;
    if (!grad || !master || !w || !adam_m || !adam_v) return fail(c, HGS_E_INVALID, "null argument");
    if (step < 1) return fail(c, HGS_E_INVALID, "step counts from 1");
    if (!(lr > 0.f) || !finite(lr)) return fail(c, HGS_E_INVALID, "lr must be > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_mlp_adam(grad, master, w, adam_m, adam_v, step, lr, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_mlp_bf16_from_master(hgs_ctx* c, void* stream, const float* master, uint16_t* w) {
    if (!c || !master || !w) return HGS_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    launch_bf16_from_master(master, w, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_feature_stats(hgs_ctx* c, void* stream, const float* feats, int64_t n, float* mean_std) {
    if (!c || !mean_std || n < 0 || n > 0x7fffffffll || (n > 0 && !feats)) return HGS_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    launch_feat_stats(feats, (uint32_t)n, mean_std, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_stream_copy(hgs_ctx* c, void* stream, const void* src, void* dst, int64_t bytes) {
    if (!c) return HGS_E_INVALID;
    if (bytes < 0 || bytes % 16 || (bytes && (!src || !dst)) || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(c, HGS_E_INVALID, "bytes must be a multiple of 16 and both pointers 16-byte aligned");
    if (bytes == 0) return HGS_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    launch_stream_copy(src, dst, (size_t)bytes, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_downsample2x(hgs_ctx* c, void* stream, const float* src, int32_t width, int32_t height, float* dst) {
    if (!c || !src || !dst || width < 1 || height < 1 || width > 8192 || height > 8192)
        return fail(c, HGS_E_INVALID, "bad downsample arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_downsample2x(src, width, height, dst, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

namespace {

// Check n region descriptors and copy them to the context's device buffer
// (after the stream's previous work, which may still read it).
hgs_status upload_regions(hgs_ctx* c, hipStream_t s, int64_t n, const hgs_region* regions) {
    std::vector<RegionDev> r((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const hgs_region& q = regions[i];
        if (!q.img || !q.ref || q.w < 1 || q.h < 1 || q.x0 < 0 || q.y0 < 0 || q.x0 + q.w > q.ref_w ||
            q.y0 + q.h > q.ref_h)
            return fail(c, HGS_E_INVALID, "region %lld is outside its reference", (long long)i);
        r[i] = RegionDev{q.img, q.ref, q.w, q.h, q.ref_w, q.ref_h, q.x0, q.y0};
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hgs_status st;
    HIP_TRY(c, hipStreamSynchronize(s));   // the descriptor buffer is reused
    if ((st = ensure(c, c->region_dev, sizeof(RegionDev) * (size_t)n))) return st;
    HIP_TRY(c, hipMemcpy(c->region_dev.p, r.data(), sizeof(RegionDev) * (size_t)n, hipMemcpyHostToDevice));
    return HGS_OK;
}

}  // namespace

hgs_status hgs_region_mse(hgs_ctx* c, void* stream, int32_t n, const hgs_region* regions, float* out) {
    if (!c || n < 0 || (n > 0 && (!regions || !out))) return HGS_E_INVALID;
    if (n == 0) return HGS_OK;
    hipStream_t s = (hipStream_t)stream;
    hgs_status st = upload_regions(c, s, n, regions);
    if (st) return st;
    launch_region_mse(P<RegionDev>(c->region_dev), n, out, s);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_lod_labels(hgs_ctx* c, void* stream, int32_t n, const hgs_region* regions, float label_db,
                          float* labels, float* drop_db) {
    if (!c || n < 0 || (n > 0 && (!regions || !labels))) return HGS_E_INVALID;
    if (!std::isfinite(label_db)) return fail(c, HGS_E_INVALID, "label_db must be finite");
    if (n > 0x3fffffff) return fail(c, HGS_E_INVALID, "too many candidates");
    if (n == 0) return HGS_OK;
    hipStream_t s = (hipStream_t)stream;
    hgs_status st = upload_regions(c, s, 2 * (int64_t)n, regions);
    if (st) return st;
    launch_lod_labels(P<RegionDev>(c->region_dev), n, (double)label_db, labels, drop_db, s);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_set_surfaces(hgs_ctx* c, int32_t n, const hgs_surface* surfaces) {
    if (!c || n < 0 || (n > 0 && !surfaces)) return HGS_E_INVALID;
    for (int i = 0; i < n; ++i) {
        const hgs_surface& q = surfaces[i];
        if (q.kind < 0 || q.kind > 2 || q.pattern < 0 || q.pattern > 3) return fail(c, HGS_E_INVALID, "surface %d: bad kind", i);
        for (int k = 0; k < 3; ++k)
            if (!finite(q.o[k]) || !finite(q.a[k]) || !finite(q.b[k]) || !finite(q.col[k]))
                return fail(c, HGS_E_INVALID, "surface %d: not finite", i);
    }
    static_assert(sizeof(hgs_surface) == sizeof(SurfaceDev), "surface layout");
    HIP_TRY(c, hipSetDevice(c->device));
    hgs_status st;
    if ((st = ensure(c, c->surf, sizeof(SurfaceDev) * (size_t)(n > 0 ? n : 1)))) return st;
    HIP_TRY(c, hipDeviceSynchronize());
    if (n) HIP_TRY(c, hipMemcpy(c->surf.p, surfaces, sizeof(SurfaceDev) * (size_t)n, hipMemcpyHostToDevice));
    c->n_surf = n;
    return HGS_OK;
}

hgs_status hgs_slice_occupancy(hgs_ctx* c, void* stream, const hgs_slice_grid* grid, uint8_t* occ, uint8_t* map) {
    if (!c) return HGS_E_INVALID;
    if (!c->loaded) return fail(c, HGS_E_STATE, "no scene");
    if (!grid || (!occ && !map) || !grid->heights) return fail(c, HGS_E_INVALID, "NULL grid, heights or outputs");
    const hgs_slice_grid& g = *grid;
    if (g.nx < 1 || g.ny < 1 || g.nx > 16384 || g.ny > 16384) return fail(c, HGS_E_INVALID, "grid must be 1..16384 cells per side");
    if (g.n_planes < 1 || g.n_planes > 256) return fail(c, HGS_E_INVALID, "need 1..256 planes");
    if (!(g.cell > 0.0) || !std::isfinite(g.cell) || !std::isfinite(g.x0) || !std::isfinite(g.y0))
        return fail(c, HGS_E_INVALID, "cell size must be positive and the corner finite");
    if (!(g.rho_min > 0.f && g.rho_min < 1.f)) return fail(c, HGS_E_INVALID, "rho_min must be in (0, 1)");
    for (int k = 0; k < g.n_planes; ++k)
        if (!finite(g.heights[k])) return fail(c, HGS_E_INVALID, "plane %d height not finite", k);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    SliceArgs a{};
    a.geo = P<float4>(c->geo);
    a.ids = c->hier ? P<int32_t>(c->leaf_ids) : nullptr;
    a.n = (uint32_t)(c->hier ? c->n_leaves : c->n);
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.cell = g.cell;
    a.nx = g.nx;
    a.ny = g.ny;
    a.n_planes = g.n_planes;
    for (int k = 0; k < g.n_planes; ++k) a.heights[k] = g.heights[k];
    a.rho_min = g.rho_min;
    a.occ = occ;
    a.map = map;
    launch_slice(a, s);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_disc_collision(hgs_ctx* c, void* stream, const uint8_t* map, double x0, double y0, double cell,
                              int32_t nx, int32_t ny, int64_t n, const double* xy, double radius, uint8_t* out) {
    if (!c) return HGS_E_INVALID;
    if (nx < 1 || ny < 1 || nx > 16384 || ny > 16384) return fail(c, HGS_E_INVALID, "grid must be 1..16384 cells per side");
    if (n < 0 || (n > 0 && (!map || !xy || !out))) return fail(c, HGS_E_INVALID, "bad query arrays");
    if (!(cell > 0.0) || !std::isfinite(cell) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(c, HGS_E_INVALID, "cell size must be positive and the corner finite");
    if (!(radius >= 0.0) || !std::isfinite(radius)) return fail(c, HGS_E_INVALID, "radius must be finite and >= 0");
    HIP_TRY(c, hipSetDevice(c->device));
    DiscArgs d{map, x0, y0, cell, nx, ny, n, xy, radius, out};
    launch_disc_collision(d, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

namespace {

hgs_status check_grid(hgs_ctx* c, int32_t nx, int32_t ny) {
    if (nx < 1 || ny < 1 || nx > 16384 || ny > 16384) return fail(c, HGS_E_INVALID, "grid must be 1..16384 cells per side");
    if ((int64_t)nx * ny > (int64_t)1 << 24) return fail(c, HGS_E_INVALID, "grid must hold at most 2^24 cells");
    return HGS_OK;
}

constexpr int kNavBatch = 32;          // relaxation rounds between convergence checks (settled rounds return at once)
constexpr int64_t kNavMaxRounds = 1 << 22;

}  // namespace

hgs_status hgs_navigable_map(hgs_ctx* c, void* stream, const uint8_t* map, double x0, double y0, double cell,
                             int32_t nx, int32_t ny, double radius, uint8_t* nav) {
    if (!c) return HGS_E_INVALID;
    if (hgs_status s = check_grid(c, nx, ny)) return s;
    if (!map || !nav) return fail(c, HGS_E_INVALID, "map and nav must be device buffers");
    if (!(cell > 0.0) || !std::isfinite(cell) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(c, HGS_E_INVALID, "cell size must be positive and the corner finite");
    if (!(radius >= 0.0) || !std::isfinite(radius)) return fail(c, HGS_E_INVALID, "radius must be finite and >= 0");
    HIP_TRY(c, hipSetDevice(c->device));
    NavArgs a{map, x0, y0, cell, nx, ny, radius, nav};
    launch_navigable(a, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_distance_fields(hgs_ctx* c, void* stream, const uint8_t* nav, int32_t nx, int32_t ny,
                               int32_t n_goals, const int32_t* goals, uint64_t* dist, int64_t* rounds) {
    if (!c) return HGS_E_INVALID;
    if (hgs_status s = check_grid(c, nx, ny)) return s;
    if (n_goals < 1 || n_goals > 65535) return fail(c, HGS_E_INVALID, "n_goals must be 1..65535");
    if (!nav || !goals || !dist) return fail(c, HGS_E_INVALID, "nav, goals and dist are required");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int T = dist_tile();
    const int tx = (nx + T - 1) / T, ty = (ny + T - 1) / T;
    const size_t tiles = (size_t)tx * ty;
    hgs_status s;
    if ((s = ensure(c, c->nav_goals, (size_t)n_goals * 4)) || (s = ensure(c, c->nav_flags, 2 * tiles * n_goals)) ||
        (s = ensure(c, c->nav_active, kNavBatch * 4)))
        return s;
    if (!c->nav_active_host)
        HIP_TRY(c, hipHostMalloc((void**)&c->nav_active_host, kNavBatch * 4, hipHostMallocDefault));
    HIP_TRY(c, hipMemcpyAsync(c->nav_goals.p, goals, (size_t)n_goals * 4, hipMemcpyHostToDevice, st));
    DistArgs d{};
    d.nav = nav;
    d.nx = nx;
    d.ny = ny;
    d.tiles_x = tx;
    d.tiles_y = ty;
    d.n_goals = n_goals;
    d.goals = P<int32_t>(c->nav_goals);
    d.dist = dist;
    d.flags[0] = P<uint8_t>(c->nav_flags);
    d.flags[1] = P<uint8_t>(c->nav_flags) + tiles * n_goals;
    d.active = P<uint32_t>(c->nav_active);
    launch_dist_init(d, st);
    HIP_TRY(c, hipGetLastError());
    // rounds in batches; a round in which no tile changed is a fixed point
    int64_t done = -1;
    for (int64_t r0 = 0; r0 < kNavMaxRounds && done < 0; r0 += kNavBatch) {
        launch_dist_rounds(d, (int)(r0 & 1), kNavBatch, st);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipMemcpyAsync(c->nav_active_host, c->nav_active.p, kNavBatch * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        for (int k = 0; k < kNavBatch; ++k)
            if (c->nav_active_host[k] == 0) {
                done = r0 + k + 1;
                break;
            }
    }
    if (done < 0) return fail(c, HGS_E_UNSUPPORTED, "distance fields did not settle within %lld rounds", (long long)kNavMaxRounds);
    if (rounds) *rounds = done;
    return HGS_OK;
}

hgs_status hgs_trace_paths(hgs_ctx* c, void* stream, const uint8_t* nav, int32_t nx, int32_t ny,
                           const uint64_t* dist, int32_t n_goals, int64_t n, const int32_t* starts,
                           const int32_t* slots, int32_t cap, int32_t* paths, int32_t* lengths) {
    if (!c) return HGS_E_INVALID;
    if (hgs_status s = check_grid(c, nx, ny)) return s;
    if (n_goals < 1 || n_goals > 65535) return fail(c, HGS_E_INVALID, "n_goals must be 1..65535");
    if (n < 0 || cap < 0) return fail(c, HGS_E_INVALID, "n and cap must be >= 0");
    if (n > 0 && (!nav || !dist || !starts || !slots || !lengths || (cap > 0 && !paths)))
        return fail(c, HGS_E_INVALID, "bad query arrays");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t stride = ((int64_t)nx * ny + 15) / 16 * 16;
    if (n > 0) {
        if (hgs_status s = ensure(c, c->nav_steps, (size_t)n_goals * stride)) return s;
    }
    TraceArgs a{nav, nx, ny, dist, n_goals, n, starts, slots, cap, paths, lengths, P<uint8_t>(c->nav_steps), stride};
    launch_trace(a, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_render_backward(hgs_ctx* c, void* stream, const hgs_image_grad* grads, const hgs_scene_grad* out) {
    if (!c || !grads || !out) return HGS_E_INVALID;
    if (!c->last_valid) return fail(c, HGS_E_STATE, "backward needs a completed render");
    if (n_passes(c) != 1) return fail(c, HGS_E_STATE, "backward needs a render done in one pass");
    if (c->last_blend) return fail(c, HGS_E_UNSUPPORTED, "backward of a blended render is not supported");
    if (!c->last_default_tiles)
        return fail(c, HGS_E_UNSUPPORTED, "backward needs a render binned to %dx%d tiles", kTile, kTile);
    if (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh)
        return fail(c, HGS_E_INVALID, "every gradient array is required");
    const int nv = (int)c->cams.size();
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipEventSynchronize(c->dimg_copied));    // the previous copy is done with the mirror
    for (int v = 0; v < nv; ++v) c->dimg_host[v] = ImgGrad{grads[v].rgb, grads[v].depth, grads[v].alpha};
    hipStream_t st = (hipStream_t)stream;
    hgs_status s;
    if ((s = ensure(c, c->egrad, (size_t)c->cut_cap * kEntryGrad * sizeof(float))) ||
        (s = ensure(c, c->brec, (size_t)c->cut_cap * kEntryRec * sizeof(float))) ||
        (s = ensure(c, c->dimg, (size_t)nv * sizeof(ImgGrad))))
        return s;
    HIP_TRY(c, hipMemcpyAsync(c->dimg.p, c->dimg_host, (size_t)nv * sizeof(ImgGrad), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipEventRecord(c->dimg_copied, st));
    BwdArgs b{};
    Work& W = c->w[c->last_lane];
    b.vals = P<uint32_t>(W.pval[c->last_pair_buf]);
    b.ranges = P<uint2>(c->ranges);
    b.total_tiles = pass_tile0(c, 1) - pass_tile0(c, 0);
    b.proj = P<Proj>(W.proj);
    b.cut_cap = c->cut_cap;
    b.views = P<ViewDev>(c->views);
    b.tile_view = P<uint32_t>(c->tile_view);
    b.dimg = P<ImgGrad>(c->dimg);
    b.egrad = P<float>(c->egrad);
    b.state = c->last_keep ? P<uint2>(c->px_state) : nullptr;
    ProjBwdArgs p{};
    p.cut = P<uint2>(W.cut);
    p.cut_cap = c->cut_cap;
    p.geo = P<float4>(c->geo);
    p.sh = P<float>(c->sh);
    p.n = c->n;
    p.sh_degree = c->sh_degree;
    p.views = P<ViewDev>(c->views);
    p.egrad = b.egrad;
    p.ctr = P<Counters>(c->counters);
    p.rec = P<float>(c->brec);
    SortArgs sa{};
    sa.keys[0] = P<uint32_t>(W.dkey[0]);
    sa.keys[1] = P<uint32_t>(W.dkey[1]);
    sa.vals[0] = P<uint32_t>(W.dval[0]);
    sa.vals[1] = P<uint32_t>(W.dval[1]);
    sa.count = &p.ctr->cut;
    sa.cap = c->cut_cap;
    sa.key_bits = bits_for((uint32_t)c->n);
    sa.max_digit_bits = c->sort_digit_bits;
    sa.hist = P<uint32_t>(W.hist);
    GatherArgs ga{};
    ga.cap = c->cut_cap;
    ga.ctr = p.ctr;
    ga.rec = p.rec;
    ga.sh_degree = c->sh_degree;
    ga.g_means = out->means;
    ga.g_scales = out->scales;
    ga.g_quats = out->quats;
    ga.g_opacity = out->opacity;
    ga.g_sh = out->sh;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (c->stage_timing) {
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) e = nullptr;
        if (ev[0]) HIP_TRY(c, hipEventRecord(ev[0], st));
    }
    launch_backward_composite(b, p.ctr, st);
    if (ev[1]) HIP_TRY(c, hipEventRecord(ev[1], st));
    launch_backward_params(p, sa, ga, st);
    if (ev[2]) HIP_TRY(c, hipEventRecord(ev[2], st));
    if (ev[0] && ev[1] && ev[2]) {
        c->bwd_ev.push_back({ev[0], ev[1], ev[2]});
    } else {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_render_surfaces(hgs_ctx* c, void* stream, int32_t view, int32_t ss, float* rgb) {
    if (!c || !rgb) return HGS_E_INVALID;
    if (view < 0 || view >= (int32_t)c->cams.size()) return fail(c, HGS_E_INVALID, "view out of range");
    if (ss < 1 || ss > 4) return fail(c, HGS_E_INVALID, "supersampling must be 1..4");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_surfaces(P<SurfaceDev>(c->surf), c->n_surf, c->views_host[view], ss, rgb, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return HGS_OK;
}

}  // extern "C"
