// Ground-truth images of the synthetic buildings: ray casting of the exact
// surfaces the Gaussian leaves were drawn from (rectangles, cylinder sides,
// disks with their procedural colour patterns), supersampled.  These stand
// in for the posed photographs a scan is judged against; the Gaussian scene
// only approximates them.  Evaluation infrastructure for the learned cut,
// not part of the render path.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kChunk = 512;     // surfaces staged in LDS at a time

__device__ __forceinline__ float3 f3(const float* p) { return make_float3(p[0], p[1], p[2]); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Procedural colour factors of the generator: floor boards, ceiling tiles,
// walls with a skirting band and soft stripes.
__device__ __forceinline__ float pattern(int kind, float3 p) {
    const float twopi = 6.283185307179586f;
    if (kind == 1) return 0.85f + 0.15f * (sinf(twopi * p.x / 0.4f) > 0.f ? 1.f : (sinf(twopi * p.x / 0.4f) < 0.f ? -1.f : 0.f));
    if (kind == 2) {
        float m = fmodf(floorf(p.x / 0.6f) + floorf(p.y / 0.6f), 2.f);
        if (m < 0.f) m += 2.f;
        return 0.9f + 0.1f * m;
    }
    if (kind == 3) {
        const float zz = fmodf(p.z, 3.0f);
        return (zz >= 0.f ? zz : zz + 3.0f) < 0.12f ? 0.55f : 0.92f + 0.08f * sinf(twopi * (p.x + p.y) / 1.3f);
    }
    return 1.f;
}

// Nearest hit of the ray o + t d (t > tmin) with surface s; returns t or a
// negative value.
__device__ __forceinline__ float hit(const SurfaceDev& s, float3 o, float3 d, float tmin) {
    if (s.kind == 0) {                       // rectangle o + u a + v b
        const float3 so = f3(s.o), a = f3(s.a), b = f3(s.b);
        const float3 n = cross3(a, b);
        const float den = dot3(d, n);
        if (fabsf(den) < 1e-12f) return -1.f;
        const float t = dot3(sub3(so, o), n) / den;
        if (!(t > tmin)) return -1.f;
        const float3 p = make_float3(o.x + t * d.x - so.x, o.y + t * d.y - so.y, o.z + t * d.z - so.z);
        const float u = dot3(p, a) / dot3(a, a), v = dot3(p, b) / dot3(b, b);
        return (u >= 0.f && u <= 1.f && v >= 0.f && v <= 1.f) ? t : -1.f;
    }
    if (s.kind == 1) {                       // cylinder side: centre o.xy, base o.z, radius r, height h
        const float px = o.x - s.o[0], py = o.y - s.o[1];
        const float A = d.x * d.x + d.y * d.y;
        if (A < 1e-12f) return -1.f;
        const float B = px * d.x + py * d.y, C = px * px + py * py - s.r * s.r;
        const float disc = B * B - A * C;
        if (disc < 0.f) return -1.f;
        const float sq = sqrtf(disc);
        float t = (-B - sq) / A;
        for (int k = 0; k < 2; ++k) {
            if (t > tmin) {
                const float z = o.z + t * d.z;
                if (z >= s.o[2] && z <= s.o[2] + s.h) return t;
            }
            t = (-B + sq) / A;
        }
        return -1.f;
    }
    // disk: centre o, radius r, normal +z
    if (fabsf(d.z) < 1e-12f) return -1.f;
    const float t = (s.o[2] - o.z) / d.z;
    if (!(t > tmin)) return -1.f;
    const float x = o.x + t * d.x - s.o[0], y = o.y + t * d.y - s.o[1];
    return x * x + y * y <= s.r * s.r ? t : -1.f;
}

template <int SS>
__global__ __launch_bounds__(256) void k_surfaces(const SurfaceDev* __restrict__ surf, int ns, ViewDev V,
                                                  float* __restrict__ out) {
    constexpr int nsub = SS * SS;
    constexpr int ss = SS;
    __shared__ SurfaceDev s_surf[kChunk];
    const int W = V.width, H = V.height;
    const int px = blockIdx.x * 16 + threadIdx.x % 16, py = blockIdx.y * 16 + threadIdx.x / 16;
    const bool inside = px < W && py < H;
    const float3 o = make_float3((float)V.o[0], (float)V.o[1], (float)V.o[2]);
    float best_t[nsub];
    int best_s[nsub];
    float3 dirs[nsub];
#pragma unroll
    for (int k = 0; k < nsub; ++k) {
        const float sx = px + (k % ss + 0.5f) / ss, sy = py + (k / ss + 0.5f) / ss;
        const float cx = (sx - (float)V.cx) / (float)V.fx, cy = (sy - (float)V.cy) / (float)V.fy;
        // world direction = R^T (cx, cy, 1)
        dirs[k] = make_float3((float)V.R[0] * cx + (float)V.R[3] * cy + (float)V.R[6],
                              (float)V.R[1] * cx + (float)V.R[4] * cy + (float)V.R[7],
                              (float)V.R[2] * cx + (float)V.R[5] * cy + (float)V.R[8]);
        best_t[k] = 3.4e38f;
        best_s[k] = -1;
    }
    for (int base = 0; base < ns; base += kChunk) {
        const int cnt = min(kChunk, ns - base);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += 256) s_surf[i] = surf[base + i];
        __syncthreads();
        if (inside) {
            for (int i = 0; i < cnt; ++i) {
#pragma unroll
                for (int k = 0; k < nsub; ++k) {
                    const float t = hit(s_surf[i], o, dirs[k], (float)V.znear);
                    if (t > 0.f && t < best_t[k]) {
                        best_t[k] = t;
                        best_s[k] = base + i;
                    }
                }
            }
        }
    }
    if (!inside) return;
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < nsub; ++k) {
        if (best_s[k] < 0) {
            for (int c = 0; c < 3; ++c) acc[c] += V.bg[c];
            continue;
        }
        const SurfaceDev& s = surf[best_s[k]];
        const float3 p = make_float3(o.x + best_t[k] * dirs[k].x, o.y + best_t[k] * dirs[k].y, o.z + best_t[k] * dirs[k].z);
        const float f = pattern(s.pattern, p);
        for (int c = 0; c < 3; ++c) acc[c] += fminf(fmaxf(s.col[c] * f, 0.f), 1.f);
    }
    const size_t plane = (size_t)W * H, i = (size_t)py * W + px;
    for (int c = 0; c < 3; ++c) out[c * plane + i] = acc[c] / nsub;
}

}  // namespace

void launch_surfaces(const SurfaceDev* surf, int ns, const ViewDev& V, int ss, float* out, hipStream_t s) {
    dim3 grid((V.width + 15) / 16, (V.height + 15) / 16);
    switch (ss) {
        case 1: k_surfaces<1><<<grid, 256, 0, s>>>(surf, ns, V, out); break;
        case 2: k_surfaces<2><<<grid, 256, 0, s>>>(surf, ns, V, out); break;
        case 3: k_surfaces<3><<<grid, 256, 0, s>>>(surf, ns, V, out); break;
        default: k_surfaces<4><<<grid, 256, 0, s>>>(surf, ns, V, out); break;
    }
}

}  // namespace hgs
