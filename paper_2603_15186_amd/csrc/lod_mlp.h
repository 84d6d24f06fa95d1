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
    // per node, three float4: (thinnest axis x, y, z, children's colour
    // variance), the parent's bounding sphere (radius < 0: none), (opacity,
    // child count, 0, 0); one gather per candidate
    const float4* nodefeat;
    const float4* bound;
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
    // The features only feed the network, whose decisions are compared with
    // a 1e-3 margin on the logit: single precision (the hardware log2 and
    // reciprocal square root, a few ulp) is far inside it.  The differences
    // to the camera come from the FP64 geometry.
    constexpr float kLn2 = 0.69314718055994531f;
    const float inv = __builtin_amdgcn_rsqf(fmaxf((float)g.d2, 1e-18f));      // 1 / max(|c - o|, 1e-9)
    const float f2 = (float)V.f2;
    f[0] = kLn2 * __log2f(fmaxf(f2 * (float)g.r * inv, 1e-6f));
    f[1] = kLn2 * __log2f((float)(g.pz > V.znear ? g.pz : V.znear));
    const float4 nf = m.nodefeat[3 * (int64_t)k], pb = m.nodefeat[3 * (int64_t)k + 1],
                 oc = m.nodefeat[3 * (int64_t)k + 2];
    f[2] = oc.x;
    f[3] = oc.y;
    f[4] = nf.w;
    f[5] = fabsf(((float)g.dx * nf.x + (float)g.dy * nf.y + (float)g.dz * nf.z) * inv);
    f[6] = (float)level;
    if (pb.w >= 0.f) {
        const float qx = (float)((double)pb.x - V.o[0]), qy = (float)((double)pb.y - V.o[1]),
                    qz = (float)((double)pb.z - V.o[2]);
        const float pinv = __builtin_amdgcn_rsqf(fmaxf(qx * qx + qy * qy + qz * qz, 1e-18f));
        f[7] = kLn2 * __log2f(fmaxf(f2 * pb.w * pinv, 1e-6f));
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

// The same network for the 64 candidates of a wave on the matrix cores
// (FP32 MFMA 16x16x4, FP32 products and sums): candidates are the N
// dimension, hidden units the M dimension, so a layer's accumulators
// (lane l, register r: hidden unit 4 (l / 16) + r of a 16-unit tile,
// candidate l % 16 of a 16-candidate tile) are the next layer's B operand
// as they stand, with the weights loaded in the matching K order.  x: the
// wave's standardised features, candidate c's at x[c * kMlpXStride + i].
// Every lane of the wave takes part; returns the logit of the lane's own
// candidate (lane c: candidate c).
constexpr int kMlpXStride = kMlpIn + 1;
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float lod_mlp_logit_mfma(const float* __restrict__ w, const float* x) {
    const int l = __lane_id();
    const int lr = l & 15, lg = l >> 4;
    mlp_f4 h1[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) h1[m][t] = mlp_f4{0.f, 0.f, 0.f, 0.f};
    // layer 1: H1^T (32 x 64) = W1 (32 x 8) X^T (8 x 64)
#pragma unroll
    for (int s = 0; s < kMlpIn / 4; ++s) {
        float a[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) a[m] = w[kOffW1 + (16 * m + lr) * kMlpIn + 4 * s + lg];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float b = x[(16 * t + lr) * kMlpXStride + 4 * s + lg];
#pragma unroll
            for (int m = 0; m < 2; ++m) h1[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b, h1[m][t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float bias = w[kOffB1 + 16 * m + 4 * lg + r];
#pragma unroll
            for (int t = 0; t < 4; ++t) h1[m][t][r] = fmaxf(h1[m][t][r] + bias, 0.f);
        }
    // layer 2: H2^T (32 x 64) = W2 (32 x 32) H1^T, one 16-unit output tile m
    // at a time, the K steps over (tile mp, register r); layer 3 takes each
    // tile's units as they come: every lane sums its four units per
    // candidate tile, then the four lane groups are added
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        mlp_f4 h2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) h2[t] = mlp_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mp = 0; mp < 2; ++mp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = w[kOffW2 + (16 * m + lr) * kMlpH + 16 * mp + 4 * lg + r];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    h2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, h1[mp][t][r], h2[t], 0, 0, 0);
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float bias = w[kOffB2 + 16 * m + 4 * lg + r], w3 = w[kOffW3 + 16 * m + 4 * lg + r];
#pragma unroll
            for (int t = 0; t < 4; ++t) part[t] = fmaf(w3, fmaxf(h2[t][r] + bias, 0.f), part[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        part[t] += __shfl_xor(part[t], 16, 64);
        part[t] += __shfl_xor(part[t], 32, 64);
    }
    const float z = lg == 0 ? part[0] : (lg == 1 ? part[1] : (lg == 2 ? part[2] : part[3]));
    return w[kOffB3] + z;
}

}  // namespace hgs
