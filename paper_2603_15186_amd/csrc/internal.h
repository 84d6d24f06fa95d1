// Internal declarations shared by the renderer's translation units: device
// data layouts, per-view parameters, counters and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "hgs.h"
#include "validate.h"

namespace hgs {

constexpr int kTile = 16;                 // default tile edge in pixels (the backward pass's tile)
constexpr int kTilePx = kTile * kTile;    // pixels per default tile
constexpr int kMaxViews = 4096;
// Cut entries are addressed by 28-bit indices: the depth-sorted values
// carry the entry index in the low 28 bits and min(tile count, 15) in the
// top 4, so the pair-count scan reads tile counts in depth order without
// gathering them (15: look the count up).
constexpr int kNtShift = 28;
constexpr uint32_t kEntryMask = (1u << kNtShift) - 1u;
constexpr uint32_t kNtSat = 15u;

// Overflow bits in Counters::overflow.
constexpr uint32_t kOvFrontier = 1u;
constexpr uint32_t kOvCut = 2u;
constexpr uint32_t kOvPairs = 4u;
constexpr uint32_t kOvCand = 8u;
constexpr uint32_t kOvDepth = 16u;        // a depth key outside the range the pass's key width assumed

// Per-view parameters, resident in device memory.  FP64 copies of the
// extrinsics and intrinsics feed the cut and the projection; the compositor
// reads the image layout and output pointers.
struct ViewDev {
    double o[3];
    double R[9];
    double fx, fy, cx, cy, W, H, znear;
    double f2, tau2;                 // cut: 2 max(fx, fy) and tau^2
    double tau;                      // LOD threshold, pixels (transition blending)
    double nl, nr, nt, nb;           // squared lengths of the side-plane normals
    double xlo, xhi, ylo, yhi;       // Jacobian clamp range of x/z and y/z
    float bg[3];
    int32_t width, height, tiles_x, tiles_y;
    uint32_t tile_base;              // first tile id of this view within its pass
    int32_t keep_node;               // >= 0: never refine this node (label renders)
    float* rgb;
    float* depth;
    float* alpha;
};

// Views do not change while a kernel runs.  When every active lane of a
// wave works on the same view (the usual case for view-major frontiers and
// cuts; node-grouped ones are served from views staged in LDS), f gets a
// copy of that view read through the constant
// address space at a wave-uniform index, so its fields arrive by scalar
// loads instead of one vector gather per field; otherwise f gets the lane's
// own view.  Either way f sees the same values.
typedef const uint64_t __attribute__((address_space(4))) ConstWord;
static_assert(sizeof(ViewDev) % 8 == 0, "views are copied in 8-byte words");

// View v read through the constant address space (v wave-uniform: scalar
// loads), word by word into a local copy.
__device__ __forceinline__ ViewDev view_uniform(const ViewDev* views, uint32_t v) {
    ConstWord* src = (ConstWord*)(views + v);
    uint64_t w[sizeof(ViewDev) / 8];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(ViewDev) / 8); ++k) w[k] = src[k];
    ViewDev V;
    __builtin_memcpy(&V, w, sizeof V);
    return V;
}

template <class F>
__device__ __forceinline__ auto on_view(const ViewDev* views, uint32_t v, F&& f) {
    const uint32_t v0 = __builtin_amdgcn_readfirstlane(v);
    if (__ballot(v != v0) == 0) {
        const ViewDev V = view_uniform(views, v0);
        return f(V);
    }
    return f(views[v]);
}

// A copy of view v (the lane's own), read by scalar loads when every active
// lane of the wave asks for the same view.
__device__ __forceinline__ ViewDev load_view(const ViewDev* views, uint32_t v) {
    const uint32_t v0 = __builtin_amdgcn_readfirstlane(v);
    if (__ballot(v != v0) == 0) return view_uniform(views, v0);
    return views[v];
}

// Projected Gaussian, one per cut entry (48 bytes).  The conic is kept as
// the factors of q = (p dx + r dy)^2 + (s dy)^2, which evaluates a sum of
// squares instead of a cancelling quadratic form.
struct alignas(16) Proj {
    double u, v;                     // 2D mean, pixels
    float p, r, s;                   // conic factors
    float opacity;
    float c0, c1, c2;                // clamped RGB
    float z;                         // camera-space depth
};

// Where an entry bins: its tile rectangle and its view's tile layout
// (16 bytes, so the depth-ordered emission gathers one record).
struct alignas(16) BinRec {
    ushort4 rc;                      // tile rectangle x0, y0, x1, y1 (inclusive)
    uint32_t tile_base;              // sort key of the view's first tile: view << key_shift
    uint16_t tiles_x;
    uint16_t height;                 // image height in pixels
};

// Device counters of one render.
constexpr int kCutLevels = 64;       // hierarchy levels at most (scene validation enforces it)

struct Counters {
    uint32_t frontier[2];            // frontier sizes (ping, pong)
    uint32_t cut;                    // cut entries written so far
    uint32_t pairs;                  // total (tile, Gaussian) pairs
    uint32_t overflow;               // kOv* bits
    uint32_t need_frontier;          // largest frontier requested
    uint32_t need_cut;               // cut entries requested
    uint32_t need_pairs;             // pairs requested
    uint32_t visible;                // cut entries with at least one tile
    uint32_t tile_queue;             // persistent compositor work counter
    uint32_t cand;                   // learned-LOD candidates collected
    uint32_t need_cand;
    unsigned long long nalg;         // evaluated (pixel, Gaussian) pairs with q <= 9
    unsigned long long neval;        // (pixel, list entry) slots the compositor walked
    unsigned long long visited;      // (node, view) pairs the cut tested, over all levels
};

// Options of the compositor and binning.
struct RenderOpts {
    int batch = 256;
    bool count_nalg = false;
    bool persistent = false;
    bool exact_tiles = true;
    bool lod_blend = false;
    bool keep_state = false;         // compositor keeps each pixel's stop position and final T
    int tile_w = kTile, tile_h = kTile;   // binning and compositing tile (8x8 .. 32x16)
    int px = 1;                      // pixels per compositor thread (1, 2 or 4)
};

// Tile shapes the binning and the compositor support, and the pixels per
// compositor thread each allows (a workgroup of tile_w * tile_h / px
// threads, at least one wave64).
bool tile_shape_ok(int tile_w, int tile_h, int px);

// ---------------------------------------------------------------- launchers

// Scan scratch needs (uint2 / uint32 elements).
constexpr int kScanBlocks = 1024;
constexpr int kCutBlocks = 4096;     // workgroups of a cut level's count and emit passes
constexpr int kSortBlocks = 1024;
constexpr int kSortBins = 2048;          // widest radix digit: 11 bits
constexpr int kSortGroup = 8192;         // histogram groups of the radix sort: multiples of this size,
constexpr int kSortMaxGroups = 8192;     // at most this many groups per sort
// histogram buffer: per-group counts of every digit, then the digit totals
constexpr size_t kSortHistBytes = (size_t)kSortBins * (kSortMaxGroups + 1) * 4;

// Threshold / all-leaves / flat cut for all views.  Writes (node, view)
// entries to `cut` and the count to ctr->cut.
struct CutArgs {
    const float4* bound;
    const int2* child;               // (first_child, child_count)
    const int32_t* leaf_ids;         // ascending leaf ids (all-leaves mode)
    int64_t n_leaves;
    int64_t n_nodes;
    const int64_t* level_offset_host;
    int n_levels;
    int mode;                        // HGS_LOD_*
    bool flat;
    const ViewDev* views;
    int n_views;
    uint2* frontier[2];
    uint32_t frontier_cap;
    uint2* cut;
    uint32_t cut_cap;
    uint4* scan_tmp;                 // kScanBlocks + 1 entries
    uint8_t* dec;                    // frontier_cap bytes: per-entry decisions
    Counters* ctr;
    // learned refinement (nullptr = off); candidate band for it and for
    // candidate collection: refined by the threshold and s <= s_hi pixels
    const void* mlp;
    float p_star;                    // learned cut: 0 refines every candidate (the threshold cut)
    const float* mlp_w32;            // learned cut: the network's weights widened to FP32
    double s_hi;
    uint2* cand;                     // nullptr: do not collect candidates
    uint32_t cand_cap;
    // children of a node's views laid out child-major in the frontier
    // (node-grouped), else in plain parent order with view-major roots
    bool group_children;
};
void launch_cut(const CutArgs& a, hipStream_t s);

// Raw learned-LOD features (8 floats) and screen footprint (x0, y0, x1, y1
// pixel bounds of the node's bounding-sphere projection, clipped) of
// candidate (node, view) entries.
void launch_lod_features(const uint2* cand, const uint32_t* count, const ViewDev* views, const void* mlp_geom,
                         float* feats, int4* rects, hipStream_t s);

struct ProjectArgs {
    const uint2* cut;
    uint32_t cut_cap;
    const float4* geo;               // [n*3]
    const float* sh;                 // [g][k][c]: the 3 K coefficients of a Gaussian contiguous
    int64_t n;
    int sh_degree;
    const ViewDev* views;
    Proj* proj;
    // depth keys: the FP32 depth's bits minus depth_base; binned depths lie
    // in [depth_base, depth_top] (bit patterns), else kOvDepth is raised
    uint32_t* depth_key;
    uint32_t depth_base, depth_top;
    int view_shift;                  // > 0: the key also holds the entry's view << view_shift
    uint32_t* depth_val;
    uint32_t* ntiles;
    BinRec* bins;
    bool exact_tiles;
    Counters* ctr;
    // transition blending (blend false: off): parent ids, bounding spheres
    // and (first child, child count) of every node
    bool blend;
    const int32_t* parent;
    const float4* bound;
    const int2* child;
    int tile_w, tile_h;              // tile shape in pixels
    int key_shift;                   // pair sort keys: view << key_shift | tile within the view
    // the pass's views staged in LDS (at most kProjectLdsViews; for
    // node-grouped cuts, whose waves span several views)
    bool lds_views;
    int n_views;
};
constexpr int kProjectLdsViews = 64;
void launch_project(const ProjectArgs& a, hipStream_t s);

// keys[i] = view of the depth-sorted entry order[i] (order: index | tiles
// << 28), read from the cut, so that a stable pass on them groups the
// entries by view.
void launch_view_keys(const uint32_t* order, const uint2* cut, const uint32_t* count, uint32_t cap, uint32_t* keys,
                      hipStream_t s);

// Pair emission in depth order: offsets = exclusive scan of ntiles over the
// depth-sorted entries.
struct EmitArgs {
    const uint32_t* order;           // depth-sorted entries (index | min(tiles, 15) << 28)
    const uint32_t* ntiles;
    const BinRec* bins;
    const Proj* proj;
    uint32_t cut_cap;
    uint32_t* offsets;               // scratch [cut_cap]
    uint32_t* keys;
    uint32_t* vals;
    uint32_t pair_cap;
    bool exact_tiles;
    uint4* scan_tmp;
    Counters* ctr;
    int tile_w, tile_h;              // tile shape in pixels
};
void launch_emit(const EmitArgs& a, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low key_bits bits.
// count: device pointer to n (clamped to cap).  Ping-pong buffers; returns
// the index (0 or 1) of the buffer pair that holds the result.
struct SortArgs {
    uint32_t* keys[2];
    uint32_t* vals[2];
    const uint32_t* count;
    uint32_t cap;
    int key_bits;
    int max_digit_bits = 11;         // 6..11
    uint32_t* hist;                  // kSortBins * (hist_stride + 1) counts
    uint32_t hist_stride = kSortMaxGroups;   // per-digit row of hist: at least the sort's group count
};
int launch_sort(const SortArgs& a, hipStream_t s);

struct CompositeArgs {
    const uint32_t* keys;            // pair sort keys (view << key_shift | tile within the view), grouped
    const uint32_t* vals;            // entry indices
    uint32_t pair_cap;
    uint32_t cut_cap;
    uint2* ranges;                   // [total_tiles]
    uint32_t total_tiles;
    int key_shift;
    const Proj* proj;
    const ViewDev* views;
    const uint32_t* tile_view;       // [total_tiles] view of each global tile
    int n_views;
    RenderOpts opts;
    Counters* ctr;
    // per pixel of the pass, [tile][256 pixels]: (list position where the
    // pixel stopped, or the list length; final transmittance bits); null: not kept
    uint2* state;
};
void launch_ranges(const CompositeArgs& a, hipStream_t s);
void launch_composite(const CompositeArgs& a, hipStream_t s);

void launch_reset_counters(Counters* c, hipStream_t s);

// GS-slice occupancy (slice.hip): occ[k][j][i] and map[j][i] bytes (either
// may be null), cell (i, j) = [x0 + i cell, x0 + (i+1) cell] x [y0 + j cell,
// y0 + (j+1) cell].
struct SliceArgs {
    const float4* geo;               // [n_nodes * 3]
    const int32_t* ids;              // Gaussians to slice (null: 0..n-1)
    uint32_t n;
    double x0, y0, cell;
    int nx, ny, n_planes;
    double rho_min;
    float heights[256];              // plane heights (passed by value)
    uint8_t* occ;
    uint8_t* map;
};
void launch_slice(const SliceArgs& a, hipStream_t s);

// Disc robots against a 2D map (slice.hip).
struct DiscArgs {
    const uint8_t* map;              // [ny][nx], nonzero = occupied
    double x0, y0, cell;
    int nx, ny;
    int64_t n;
    const double* xy;                // n (x, y) pairs
    double radius;
    uint8_t* out;                    // n flags
};
void launch_disc_collision(const DiscArgs& d, hipStream_t s);

// backward pass (backward.hip)
constexpr int kEntryGrad = 12;       // floats per cut entry: u, v, p, r, s, opacity, rgb, depth, 2 spare
struct ImgGrad {
    const float* rgb;                // [3][h][w] or null
    const float* depth;              // [h][w] or null
    const float* alpha;              // [h][w] or null
};
struct BwdArgs {
    const uint32_t* vals;            // tile-sorted entry indices
    const uint2* ranges;
    uint32_t total_tiles;
    const Proj* proj;
    uint32_t cut_cap;
    const ViewDev* views;
    const uint32_t* tile_view;
    const ImgGrad* dimg;             // per view of the pass
    float* egrad;                    // [cut_cap][kEntryGrad]
    const uint2* state;              // the forward's kept pixel states (CompositeArgs::state); null: replay
};
struct ProjBwdArgs {
    const uint2* cut;
    uint32_t cut_cap;
    const float4* geo;
    const float* sh;                 // [g][k][c]
    int64_t n;
    int sh_degree;
    const ViewDev* views;
    const float* egrad;
    const Counters* ctr;
    const uint32_t* order;           // entry at each position of the Gaussian-sorted order
    float* rec;                      // [cut_cap][kEntryRec]: per-entry parameter gradients, in that order
};
constexpr int kEntryRec = 20;        // mean 3, scale 3, quaternion 4, opacity, colour 3, direction 3, pad
struct GatherArgs {
    const uint32_t* keys;            // Gaussian ids of the entries, ascending
    uint32_t cap;
    const Counters* ctr;
    const float* rec;
    int sh_degree;
    float* g_means;                  // [n][3]
    float* g_scales;                 // [n][3]
    float* g_quats;                  // [n][4]
    float* g_opacity;                // [n]
    float* g_sh;                     // [n][K][3]
};
void launch_backward_composite(const BwdArgs& b, const Counters* ctr, hipStream_t s);
void launch_backward_params(ProjBwdArgs p, SortArgs sa, GatherArgs ga, hipStream_t s);

// shortest-path planning (nav.hip)
struct NavArgs {
    const uint8_t* map;              // [ny][nx], nonzero = occupied
    double x0, y0, cell;
    int nx, ny;
    double radius;
    uint8_t* nav;                    // [ny][nx]: 1 navigable, 0 not
};
struct DistArgs {
    const uint8_t* nav;              // [ny][nx], nonzero = navigable
    int nx, ny, tiles_x, tiles_y;
    int n_goals;
    const int32_t* goals;            // device [n_goals] cell indices
    uint64_t* dist;                  // [n_goals][ny][nx]: a | b << 32, ~0 unreached
    uint8_t* flags[2];               // [n_goals][tiles]: tile changed in the last round
    uint32_t* active;                // per round of a batch: tiles that changed
};
struct TraceArgs {
    const uint8_t* nav;
    int nx, ny;
    const uint64_t* dist;
    int n_goals;
    int64_t n;
    const int32_t* starts;           // device [n] cell indices
    const int32_t* slots;            // device [n] field index
    int32_t cap;
    int32_t* paths;                  // device [n][cap]
    int32_t* lengths;                // device [n]
    uint8_t* steps;                  // scratch [n_goals][stride]: each cell's move
    int64_t stride;                  // bytes per goal: nx * ny rounded up to 16
};
int dist_tile();
void launch_navigable(const NavArgs& a, hipStream_t s);
void launch_dist_init(const DistArgs& d, hipStream_t s);
void launch_dist_rounds(const DistArgs& d, int round0, int n_rounds, hipStream_t s);
void launch_trace(const TraceArgs& a, hipStream_t s);

// learned-LOD network (mlp.hip)
void launch_mlp_forward(const float* feats, uint32_t n, const float* mean, const float* stdv, const uint16_t* w,
                        float* logits, hipStream_t s);
size_t mlp_train_scratch_floats(uint32_t n);
void launch_mlp_train_step(const float* feats, const float* labels, uint32_t n, const float* mean, const float* stdv,
                           float* master, uint16_t* w, float* m, float* v, int step, float lr, float* grad_out,
                           float* loss_out, float* scratch, hipStream_t s);
void launch_mlp_adam(const float* grad, float* master, uint16_t* w, float* m, float* v, int step, float lr,
                     hipStream_t s);
void launch_bf16_from_master(const float* master, uint16_t* w, hipStream_t s);
void launch_feat_stats(const float* f, uint32_t n, float* out, hipStream_t s);

// image helpers (imgutil.hip)
struct RegionDev {
    const float* img;                // planar [3][h][w]
    const float* ref;                // planar [3][ref_h][ref_w]
    int32_t w, h, ref_w, ref_h, x0, y0;
};
void launch_downsample2x(const float* src, int W, int H, float* dst, hipStream_t s);
// dst = src, `bytes` (a multiple of 16) of 16-byte aligned device memory
void launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// ground-truth surfaces of synthetic scenes (surfaces.hip); layout of
// hgs_surface
struct SurfaceDev {
    int32_t kind;                    // 0 rectangle, 1 cylinder side, 2 disk
    int32_t pattern;                 // 0 none, 1 boards, 2 tiles, 3 wall stripes
    float o[3], a[3], b[3];
    float col[3];
    float r, h;
};
void launch_surfaces(const SurfaceDev* surf, int ns, const ViewDev& V, int ss, float* out, hipStream_t s);
void launch_region_mse(const RegionDev* reg, int n, float* out, hipStream_t s);
// labels[i], drop_db[i] (may be null) from regions 2i (refined) and 2i + 1 (kept)
void launch_lod_labels(const RegionDev* reg, int n, double label_db, float* labels, float* drop_db, hipStream_t s);

}  // namespace hgs
