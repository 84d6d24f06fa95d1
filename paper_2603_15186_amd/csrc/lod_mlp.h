// Learned level-of-detail refinement: per-node features and the 8-32-32-1
// MLP (BF16 weights, FP32 accumulation) that decides whether a node the
// projected-size rule would refine is refined.  The threshold rule stays the
// fallback: nodes outside the candidate band follow it unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace hgs {

constexpr int kMlpIn = 8, kMlpH = 32;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;   // 1377
// Parameter offsets: W1[32][8], b1[32], W2[32][32], b2[32], W3[32], b3.
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH,
              kOffB2 = kOffW2 + kMlpH * kMlpH, kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpH;

struct LodMlpDev {
    const uint16_t* w;            // kMlpParams BF16 values
    float mean[kMlpIn];
    float inv_std[kMlpIn];
    float p_star;                 // refine iff sigmoid(out) >= p_star
    float s_hi;                   // candidates: projected size <= s_hi pixels
    const float4* nodefeat;       // (normal x, y, z, child colour variance)
    const int32_t* parent;
    const float4* bound;
    const float4* geo;            // geo[3k].w = opacity
    const int2* child;
    const int64_t* level_offset;  // device copy, n_levels + 1 entries
    int n_levels;
};

// Geometry of a node's bounding sphere seen from a view, FP64 in a fixed
// order without contraction (the cut's decisions depend on it exactly).
struct NodeGeom {
    double dx, dy, dz;            // c - o
    double px, py, pz;            // camera-space centre
    double r;                     // radius
    double d2;                    // |c - o|^2
};

__device__ __forceinline__ void node_geometry(const ViewDev& V, float4 b, NodeGeom* g) {
#pragma clang fp contract(off)
    g->dx = (double)b.x - V.o[0];
    g->dy = (double)b.y - V.o[1];
    g->dz = (double)b.z - V.o[2];
    g->r = (double)b.w;
    g->px = (V.R[0] * g->dx + V.R[1] * g->dy) + V.R[2] * g->dz;
    g->py = (V.R[3] * g->dx + V.R[4] * g->dy) + V.R[5] * g->dz;
    g->pz = (V.R[6] * g->dx + V.R[7] * g->dy) + V.R[8] * g->dz;
    g->d2 = (g->dx * g->dx + g->dy * g->dy) + g->dz * g->dz;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// The 8 raw features of node k seen from view V (before standardisation):
// log projected size, log depth, opacity, child count, child colour
// variance, |cos| between the view ray and the node's thinnest axis, level,
// log projected size of the parent.
__device__ __forceinline__ void lod_features(const LodMlpDev& m, const ViewDev& V, int k, float4 b,
                                             const NodeGeom& g, int level, float f[kMlpIn]) {
    const double dist = sqrt(g.d2);
    const double inv = 1.0 / (dist > 1e-9 ? dist : 1e-9);
    const double size = V.f2 * g.r * inv;
    f[0] = (float)log(size > 1e-6 ? size : 1e-6);
    f[1] = (float)log(g.pz > V.znear ? g.pz : V.znear);
    f[2] = m.geo[3 * (int64_t)k].w;
    f[3] = (float)m.child[k].y;
    const float4 nf = m.nodefeat[k];
    f[4] = nf.w;
    f[5] = (float)fabs((g.dx * nf.x + g.dy * nf.y + g.dz * nf.z) * inv);
    f[6] = (float)level;
    const int p = m.parent[k];
    if (p >= 0) {
        const float4 pb = m.bound[p];
        const double qx = (double)pb.x - V.o[0], qy = (double)pb.y - V.o[1], qz = (double)pb.z - V.o[2];
        const double pd = sqrt(qx * qx + qy * qy + qz * qz);
        const double ps = V.f2 * (double)pb.w / (pd > 1e-9 ? pd : 1e-9);
        f[7] = (float)log(ps > 1e-6 ? ps : 1e-6);
    } else {
        f[7] = f[0];
    }
}

// Forward pass on standardised features; returns the logit.
__device__ __forceinline__ float lod_mlp_logit(const uint16_t* __restrict__ w, const float x[kMlpIn]) {
    float h1[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float acc = bf16_to_f32(w[kOffB1 + j]);
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) acc = fmaf(bf16_to_f32(w[kOffW1 + j * kMlpIn + i]), x[i], acc);
        h1[j] = acc > 0.f ? acc : 0.f;
    }
    float out = bf16_to_f32(w[kOffB3]);
    for (int j = 0; j < kMlpH; ++j) {
        float acc = bf16_to_f32(w[kOffB2 + j]);
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) acc = fmaf(bf16_to_f32(w[kOffW2 + j * kMlpH + i]), h1[i], acc);
        acc = acc > 0.f ? acc : 0.f;
        out = fmaf(bf16_to_f32(w[kOffW3 + j]), acc, out);
    }
    return out;
}

// Forward pass with the weights already widened to FP32; same arithmetic as
// lod_mlp_logit.  W is a pointer type: a constant-address-space pointer lets
// uniform weight reads go through the scalar cache.
template <class W>
__device__ __forceinline__ float lod_mlp_logit_f32(W w, const float x[kMlpIn]) {
    float h1[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float acc = w[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) acc = fmaf(w[kOffW1 + j * kMlpIn + i], x[i], acc);
        h1[j] = acc > 0.f ? acc : 0.f;
    }
    float out = w[kOffB3];
#pragma unroll 4
    for (int j = 0; j < kMlpH; ++j) {
        float acc = w[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) acc = fmaf(w[kOffW2 + j * kMlpH + i], h1[i], acc);
        acc = acc > 0.f ? acc : 0.f;
        out = fmaf(w[kOffW3 + j], acc, out);
    }
    return out;
}

// For a candidate node (the threshold rule refines it and its projected
// size is at most s_hi): does the learned cut refine it?  Yes iff the
// network's probability reaches p_star.  sw: the weights as FP32.
template <class W>
__device__ __forceinline__ bool lod_mlp_expand(const LodMlpDev& m, W sw, const ViewDev& V, int k, float4 b,
                                               const NodeGeom& g, int level) {
    float f[kMlpIn];
    lod_features(m, V, k, b, g, level, f);
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) f[i] = (f[i] - m.mean[i]) * m.inv_std[i];
    const float z = lod_mlp_logit_f32(sw, f);
    const float p = 1.f / (1.f + __expf(-z));
    return p >= m.p_star;
}

}  // namespace hgs
