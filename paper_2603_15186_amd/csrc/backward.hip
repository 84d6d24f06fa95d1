// Backward pass of the renderer: gradients of a loss, given its gradients
// with respect to the output images (RGB, raw depth D = sum w z, alpha =
// 1 - T), with respect to the Gaussians' means, scales, rotations,
// opacities and SH coefficients (the optimisation behind the paper's scene
// reconstruction, Sec. III-B).
//
// Compositing (one 256-thread workgroup per 16x16 tile, a pixel per thread,
// a 16-lane quarter-wave per 4x4 block as in the forward compositor): the
// tile's depth-ordered entries are staged in LDS in batches and listed per
// block exactly as the forward stages and lists them.  Where each pixel
// stopped and its final transmittance T_N come from the forward compositor
// when the render kept them; else the pixel replays the forward recurrence
// over its block's list with the same single-precision operations.  It then
// walks the lists back to front, recovering T
// before entry i as T_{i+1} / (1 - alpha_i), with
//   dL/dalpha_i = sum_c gC_c (c_ic T_i - B_c / (1 - alpha_i))
//               + gD (z_i T_i - B_D / (1 - alpha_i)) + gA T_N / (1 - alpha_i)
// where B holds what lies behind entry i (T_N bg for the colour).  Through
// alpha = o e^{-q/2} (no gradient where capped at 0.99) and q = t1^2 + t2^2,
// t1 = p dx + r dy, t2 = s dy, each pixel yields ten numbers per entry
// (2D mean, conic factors p r s, opacity, colour, depth); the 16 lanes of a
// block, which walk the same entry, sum them with shuffles, blocks add them
// in LDS, and one global atomic add per number and tile lands them in a
// per-entry buffer.
//
// Projection (FP64): the cut entries are sorted by Gaussian (the radix sort
// of the binning); one thread per entry in that order takes the chain rule
// from the 2D mean, the conic factors of Sigma' = T T^T + 0.3 I
// (T = J W R S), the camera depth and the colour back to the Gaussian's
// mean, scale, rotation and opacity, written as a per-entry record (in the
// sorted order) with the entry's colour gradient and view direction.  One
// thread per Gaussian then sums its run of records, forming the SH
// coefficients' gradients sum g_c Y_k(d) on the way: no scattered atomics on
// the parameter arrays.
#include "blocks.h"
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = kTilePx;
constexpr int kB = 128;                         // entries staged per batch
constexpr int kNG = 10;                         // per-entry gradient numbers

struct BwdShared {
    StageA a[kB + 1];
    StageB b[kB + 1];
    StageC c[kB + 1];
    float2 uv[kB];                              // tile-relative 2D means
    float io[kB];                               // inverse opacities
    uint32_t entry[kB];
    float acc[kNG][kB];
    alignas(16) uint16_t idx[kBlocks * kB];
    uint32_t wc[(kNT / kWave) * kBlocks];
    uint32_t n[kBlocks];
    uint32_t maxlast;
};

// Q of a staged entry at pixel centre (fx, fy) by the compositor's own
// operations (its factors scaled by kS as the compositor stages them,
// -log2(o) folded into the row term), so that alpha and the stop decisions
// here are the forward pass's bit for bit.
__device__ __forceinline__ float compositor_q(const StageA& A, const StageB& B, float fx, float fy) {
    const float t1 = fmaf(kS * A.p, fx, fmaf(kS * A.r, fy, kS * A.c1));
    const float t2 = fmaf(kS * A.s, fy, kS * B.c2);
    return fmaf(t1, t1, fmaf(t2, t2, -B.lo));
}

// Stage entries [base, base + cnt) of the tile's list and build each 4x4
// block's list of staged offsets (16 B units, depth order), padded with the
// empty record up to a multiple of four of its wave's longest list.
// Returns this lane's block list length and writes the padded length.
__device__ __forceinline__ uint32_t stage_lists(const BwdArgs& a, BwdShared& S, uint32_t base, uint32_t cnt,
                                                double dx0, double dy0, int w, int lane, int gid, int k,
                                                uint32_t* n_step_out) {
    uint32_t m = 0;
    const int j = threadIdx.x;
    if (j < (int)cnt) {
        const uint32_t e = a.vals[base + j];
        const Proj P = a.proj[e < a.cut_cap ? e : 0u];
        const float u = (float)(P.u - dx0), v = (float)(P.v - dy0);
        S.a[j] = StageA{P.p, P.r, -fmaf(P.p, u, P.r * v), P.s};
        S.b[j] = StageB{-P.s * v, __log2f(P.opacity), P.z, P.c0};
        S.c[j] = StageC{P.c1, P.c2};
        S.uv[j] = make_float2(u, v);
        S.io[j] = 1.f / P.opacity;
        S.entry[j] = e;
        m = block_mask(u, v, P.p, P.r, P.s);
    }
    uint32_t pre[kBlocks];
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) {
        const uint64_t bal = __ballot((m >> b) & 1u);
        pre[b] = (uint32_t)__popcll(bal & lanemask_lt());
        if (lane == 0) S.wc[w * kBlocks + b] = (uint32_t)__popcll(bal);
    }
    __syncthreads();
    if (threadIdx.x < kBlocks) {
        uint32_t t = 0;
#pragma unroll
        for (int ww = 0; ww < kNT / kWave; ++ww) {
            const uint32_t c = S.wc[ww * kBlocks + threadIdx.x];
            S.wc[ww * kBlocks + threadIdx.x] = t;
            t += c;
        }
        S.n[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kBlocks; ++b)
        if ((m >> b) & 1u) S.idx[b * kB + S.wc[w * kBlocks + b] + pre[b]] = (uint16_t)(j * 16);
    const uint32_t n_mine = S.n[gid];
    const uint32_t n_wave = __builtin_amdgcn_readfirstlane(
        max(max(S.n[w * 4], S.n[w * 4 + 1]), max(S.n[w * 4 + 2], S.n[w * 4 + 3])));
    const uint32_t n_step = (n_wave + 3u) & ~3u;
    uint16_t* list = S.idx + gid * kB;
    for (uint32_t p = n_mine + (uint32_t)k; p < n_step; p += 16) list[p] = (uint16_t)(kB * 16);
    __syncthreads();
    *n_step_out = n_step;
    return n_mine;
}

// Sum over the 16 lanes of a DPP row, left in every lane of the row: lane
// pairs (quad_perm 1,0,3,2), quad pairs (2,3,0,1), then the mirrored half
// row and the mirrored row.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float group_sum(float x) {
    x += dpp_f<0xb1>(x);      // quad_perm [1, 0, 3, 2]
    x += dpp_f<0x4e>(x);      // quad_perm [2, 3, 0, 1]
    x += dpp_f<0x141>(x);     // row_half_mirror
    x += dpp_f<0x140>(x);     // row_mirror
    return x;
}

// Batches of 128 entries and a register budget of eight waves per SIMD: the
// reverse walk is a chain of row reductions and LDS adds whose latency only
// more resident waves hide.
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(8))) void k_composite_bwd(BwdArgs a) {
    __shared__ BwdShared S;
    const uint32_t tile = blockIdx.x;
    const uint32_t view = a.tile_view[tile];
    const ViewDev& V = a.views[view];
    const ImgGrad G = a.dimg[view];
    const uint32_t local = tile - V.tile_base;
    const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int g = lane >> 4, k = lane & 15;
    const int gid = w * 4 + g;
    const int lx = g * 4 + (k & 3), ly = w * 4 + (k >> 2);
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < V.width && py < V.height;
    const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
    const double dx0 = (double)x0, dy0 = (double)y0;
    const uint2 rg = a.ranges[tile];
    const uint32_t n = rg.y - rg.x;
    if (threadIdx.x == 0) {
        S.a[kB] = StageA{0.f, 0.f, 0.f, 0.f};
        S.b[kB] = StageB{0.f, -__builtin_inff(), 0.f, 0.f};
        S.c[kB] = StageC{0.f, 0.f};
        S.maxlast = 0;
    }

    // 1. where the pixel stopped and its final transmittance: kept by the
    // forward compositor, else a forward replay over the block lists (the
    // forward's operations)
    float T = 1.f;
    bool live = inside;
    uint32_t last = n;
    if (a.state) {
        const uint2 st = a.state[(size_t)tile * kNT + threadIdx.x];
        last = st.x;
        T = __uint_as_float(st.y);
        __syncthreads();                            // S.maxlast is set
    }
    for (uint32_t b0 = 0; !a.state && b0 < n; b0 += kB) {
        const uint32_t cnt = min((uint32_t)kB, n - b0);
        uint32_t n_step;
        stage_lists(a, S, rg.x + b0, cnt, dx0, dy0, w, lane, gid, k, &n_step);
        const uint16_t* list = S.idx + gid * kB;
        for (uint32_t p = 0; p < n_step; ++p) {
            const uint32_t off = list[p];
            const StageA A = *reinterpret_cast<const StageA*>(reinterpret_cast<const char*>(S.a) + off);
            const StageB B = *reinterpret_cast<const StageB*>(reinterpret_cast<const char*>(S.b) + off);
            const float Q = compositor_q(A, B, fx, fy);
            const float al = fminf(0.99f, __builtin_amdgcn_exp2f(-Q));
            const float Tn = T - al * T;
            const bool add = live && Q <= entry_qmax(-B.lo);
            if (add && Tn < 1e-4f) {
                live = false;
                last = b0 + off / 16;
            }
            T = add && live ? Tn : T;
            if ((p & 3u) == 3u && __ballot(live) == 0) break;
        }
        if (__syncthreads_count(live ? 1 : 0) == 0) break;
    }
    if (!inside) last = 0;
    atomicMax(&S.maxlast, last);

    // 2. back to front over the same lists
    const size_t plane = (size_t)V.width * V.height;
    const size_t pix = (size_t)py * V.width + px;
    float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
    if (inside) {
        gC0 = G.rgb ? G.rgb[pix] : 0.f;
        gC1 = G.rgb ? G.rgb[plane + pix] : 0.f;
        gC2 = G.rgb ? G.rgb[2 * plane + pix] : 0.f;
        gD = G.depth ? G.depth[pix] : 0.f;
        gA = G.alpha ? G.alpha[pix] : 0.f;
    }
    const float TN = T;
    float Tc = T;
    float B0 = T * V.bg[0], B1 = T * V.bg[1], B2 = T * V.bg[2], BD = 0.f;
    for (int i = threadIdx.x; i < kNG * kB; i += kNT) (&S.acc[0][0])[i] = 0.f;
    __syncthreads();
    const uint32_t maxlast = S.maxlast;
    const int nb = (int)((maxlast + kB - 1) / kB);
    for (int bi = nb - 1; bi >= 0; --bi) {
        const uint32_t b0 = (uint32_t)bi * kB;
        const uint32_t cnt = min((uint32_t)kB, n - b0);
        uint32_t n_step;
        stage_lists(a, S, rg.x + b0, cnt, dx0, dy0, w, lane, gid, k, &n_step);
        const uint16_t* list = S.idx + gid * kB;
        for (int p = (int)n_step - 1; p >= 0; --p) {
            const uint32_t off = list[p];
            const uint32_t j = off / 16;
            float gr[kNG];
#pragma unroll
            for (int t = 0; t < kNG; ++t) gr[t] = 0.f;
            bool has = false;
            if (j < kB && b0 + j < last) {
                const StageA A = S.a[j];
                const StageB B = S.b[j];
                const StageC C = S.c[j];
                const float t1 = fmaf(A.p, fx, fmaf(A.r, fy, A.c1));
                const float t2 = fmaf(A.s, fy, B.c2);
                const float Q = compositor_q(A, B, fx, fy);
                const float al0 = fminf(0.99f, __builtin_amdgcn_exp2f(-Q));
                const float al = Q <= entry_qmax(-B.lo) ? al0 : 0.f;
                if (al > 0.f) {
                    has = true;
                    const float iom = __builtin_amdgcn_rcpf(1.f - al);
                    const float Ti = Tc * iom;
                    const float c0 = B.col0, c1 = C.col1, c2 = C.col2, z = B.z;
                    const float wgt = al * Ti;
                    const float dLda = gC0 * (c0 * Ti - B0 * iom) + gC1 * (c1 * Ti - B1 * iom) +
                                       gC2 * (c2 * Ti - B2 * iom) + gD * (z * Ti - BD * iom) + gA * TN * iom;
                    gr[6] = gC0 * wgt;
                    gr[7] = gC1 * wgt;
                    gr[8] = gC2 * wgt;
                    gr[9] = gD * wgt;
                    B0 = fmaf(c0, wgt, B0);
                    B1 = fmaf(c1, wgt, B1);
                    B2 = fmaf(c2, wgt, B2);
                    BD = fmaf(z, wgt, BD);
                    Tc = Ti;
                    if (al0 < 0.99f) {
                        const float gq = -0.5f * al * dLda;
                        const float2 uv = S.uv[j];
                        const float dx = fx - uv.x, dy = fy - uv.y;
                        gr[0] = gq * (-2.f * t1 * A.p);
                        gr[1] = gq * (-2.f * (t1 * A.r + t2 * A.s));
                        gr[2] = gq * (2.f * t1 * dx);
                        gr[3] = gq * (2.f * t1 * dy);
                        gr[4] = gq * (2.f * t2 * dy);
                        gr[5] = dLda * al * S.io[j];
                    }
                }
            }
            // the 16 lanes of a block share the entry: sum them when any
            // contributes (a block-uniform branch)
            const uint32_t gbits = (uint32_t)(__ballot(has) >> (16 * g)) & 0xffffu;
            if (gbits) {
#pragma unroll
                for (int t = 0; t < kNG; ++t) {
                    const float sum = group_sum(gr[t]);
                    if (k == 0 && sum != 0.f) atomicAdd(&S.acc[t][j], sum);
                }
            }
        }
        __syncthreads();
        const int jj = threadIdx.x;
        if (jj < (int)cnt) {
            const uint32_t e = S.entry[jj];
            if (e < a.cut_cap) {
                float* dst = a.egrad + (size_t)e * kEntryGrad;
#pragma unroll
                for (int t = 0; t < kNG; ++t) {
                    const float x = S.acc[t][jj];
                    if (x != 0.f) atomicAdd(dst + t, x);
                    S.acc[t][jj] = 0.f;
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_zero_egrad(float* g, const Counters* ctr, uint32_t cap) {
    const uint64_t n = (uint64_t)min(ctr->cut, cap) * kEntryGrad;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        g[i] = 0.f;
}

// Real SH basis (as in the projection) and its gradient with respect to the
// direction's components, FP64.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(double x, double y, double z, double Y[16], double dY[16][3]) {
    constexpr int deg = DEG;
    constexpr double k00 = 0.28209479177387814, k1 = 0.48860251190291992;
    constexpr double k2a = 1.0925484305920792, k2b = 0.31539156525252005, k2c = 0.54627421529603959;
    constexpr double k3a = 0.59004358992664352, k3b = 2.8906114426405538, k3c = 0.45704579946446572,
                     k3d = 0.3731763325901154, k3e = 1.4453057213202769;
    for (int k = 0; k < 16; ++k) Y[k] = dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    Y[0] = k00;
    if (deg >= 1) {
        Y[1] = -k1 * y; dY[1][1] = -k1;
        Y[2] = k1 * z; dY[2][2] = k1;
        Y[3] = -k1 * x; dY[3][0] = -k1;
    }
    if (deg >= 2) {
        Y[4] = k2a * x * y; dY[4][0] = k2a * y; dY[4][1] = k2a * x;
        Y[5] = -k2a * y * z; dY[5][1] = -k2a * z; dY[5][2] = -k2a * y;
        Y[6] = k2b * (3.0 * z * z - 1.0); dY[6][2] = 6.0 * k2b * z;
        Y[7] = -k2a * x * z; dY[7][0] = -k2a * z; dY[7][2] = -k2a * x;
        Y[8] = k2c * (x * x - y * y); dY[8][0] = 2.0 * k2c * x; dY[8][1] = -2.0 * k2c * y;
    }
    if (deg >= 3) {
        Y[9] = -k3a * y * (3.0 * x * x - y * y);
        dY[9][0] = -6.0 * k3a * x * y; dY[9][1] = -k3a * (3.0 * x * x - 3.0 * y * y);
        Y[10] = k3b * x * y * z;
        dY[10][0] = k3b * y * z; dY[10][1] = k3b * x * z; dY[10][2] = k3b * x * y;
        Y[11] = -k3c * y * (5.0 * z * z - 1.0);
        dY[11][1] = -k3c * (5.0 * z * z - 1.0); dY[11][2] = -10.0 * k3c * y * z;
        Y[12] = k3d * z * (5.0 * z * z - 3.0);
        dY[12][2] = k3d * (15.0 * z * z - 3.0);
        Y[13] = -k3c * x * (5.0 * z * z - 1.0);
        dY[13][0] = -k3c * (5.0 * z * z - 1.0); dY[13][2] = -10.0 * k3c * x * z;
        Y[14] = k3e * z * (x * x - y * y);
        dY[14][0] = 2.0 * k3e * x * z; dY[14][1] = -2.0 * k3e * y * z; dY[14][2] = k3e * (x * x - y * y);
        Y[15] = -k3a * x * (x * x - 3.0 * y * y);
        dY[15][0] = -k3a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = 6.0 * k3a * x * y;
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(ProjBwdArgs a) {
    const uint32_t m = min(a.ctr->cut, a.cut_cap);
    constexpr int K = (DEG + 1) * (DEG + 1);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
        const uint32_t i = a.order[p];
        const float* eg = a.egrad + (size_t)i * kEntryGrad;
        double gin[kNG];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kNG; ++k) {
            gin[k] = eg[k];
            any = any || gin[k] != 0.0;
        }
        float4* rec0 = reinterpret_cast<float4*>(a.rec + (size_t)p * kEntryRec);
        for (int t = 0; t < kEntryRec / 4; ++t) rec0[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (!any) continue;
        const uint2 e = a.cut[i];
        const ViewDev& V = a.views[e.y];
        const int64_t g = e.x;
        const float4 g0 = a.geo[3 * g], g1 = a.geo[3 * g + 1], g2 = a.geo[3 * g + 2];
        const double dx = (double)g0.x - V.o[0], dy = (double)g0.y - V.o[1], dz = (double)g0.z - V.o[2];
        const double tx = (V.R[0] * dx + V.R[1] * dy) + V.R[2] * dz;
        const double ty = (V.R[3] * dx + V.R[4] * dy) + V.R[5] * dz;
        const double tz = (V.R[6] * dx + V.R[7] * dy) + V.R[8] * dz;
        if (!(tz > V.znear)) continue;
        const double iz = 1.0 / tz;
        const double xr0 = tx * iz, yr0 = ty * iz;
        const bool xcl = xr0 < V.xlo || xr0 > V.xhi, ycl = yr0 < V.ylo || yr0 > V.yhi;
        const double xr = fmin(fmax(xr0, V.xlo), V.xhi), yr = fmin(fmax(yr0, V.ylo), V.yhi);
        double M[2][3];
        for (int j = 0; j < 3; ++j) {
            M[0][j] = V.fx * iz * (V.R[j] - xr * V.R[6 + j]);
            M[1][j] = V.fy * iz * (V.R[3 + j] - yr * V.R[6 + j]);
        }
        double qw = g1.x, qx = g1.y, qy = g1.z, qz = g1.w;
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const double R[3][3] = {{1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)},
                                {2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx)},
                                {2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
        const double sc[3] = {g2.x, g2.y, g2.z};
        double MR[2][3], Tm[2][3];
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 3; ++k) {
                MR[r][k] = M[r][0] * R[0][k] + M[r][1] * R[1][k] + M[r][2] * R[2][k];
                Tm[r][k] = MR[r][k] * sc[k];
            }
        const double s00 = Tm[0][0] * Tm[0][0] + Tm[0][1] * Tm[0][1] + Tm[0][2] * Tm[0][2] + 0.3;
        const double s01 = Tm[0][0] * Tm[1][0] + Tm[0][1] * Tm[1][1] + Tm[0][2] * Tm[1][2];
        const double s11 = Tm[1][0] * Tm[1][0] + Tm[1][1] * Tm[1][1] + Tm[1][2] * Tm[1][2] + 0.3;
        const double det = s00 * s11 - s01 * s01;
        if (!(det > 0.0)) continue;
        // conic factors p = sqrt(s11 / det), r = -s01 / sqrt(det s11),
        // s = 1 / sqrt(s11) and their derivatives
        const double gp = gin[2], gr = gin[3], gs = gin[4];
        const double pp = sqrt(s11 / det), idet2 = 1.0 / (det * det);
        const double mm = det * s11, im12 = 1.0 / sqrt(mm), im32 = im12 / mm;
        const double h00 = gp * (0.5 / pp) * (-s11 * s11 * idet2) + gr * 0.5 * s01 * im32 * s11 * s11;
        const double h01 = gp * (0.5 / pp) * (2.0 * s11 * s01 * idet2) + gr * (-im12 - s01 * s01 * s11 * im32);
        const double h11 = gp * (0.5 / pp) * (-s01 * s01 * idet2) + gr * 0.5 * s01 * im32 * (det + s00 * s11) +
                           gs * (-0.5 / (s11 * sqrt(s11)));
        // Sigma' = T T^T: dL/dT
        double gT[2][3];
        for (int k = 0; k < 3; ++k) {
            gT[0][k] = 2.0 * h00 * Tm[0][k] + h01 * Tm[1][k];
            gT[1][k] = 2.0 * h11 * Tm[1][k] + h01 * Tm[0][k];
        }
        double gsc[3], gMR[2][3];
        for (int k = 0; k < 3; ++k) {
            gsc[k] = gT[0][k] * MR[0][k] + gT[1][k] * MR[1][k];
            gMR[0][k] = gT[0][k] * sc[k];
            gMR[1][k] = gT[1][k] * sc[k];
        }
        double gR[3][3], gM[2][3];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) gR[j][k] = M[0][j] * gMR[0][k] + M[1][j] * gMR[1][k];
        for (int r = 0; r < 2; ++r)
            for (int j = 0; j < 3; ++j) gM[r][j] = gMR[r][0] * R[j][0] + gMR[r][1] * R[j][1] + gMR[r][2] * R[j][2];
        // quaternion: dL/d(normalised q), then through the normalisation
        const double gw = 2.0 * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] +
                                 qx * gR[2][1]);
        const double gx = 2.0 * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2.0 * qx * gR[1][1] - qw * gR[1][2] +
                                 qz * gR[2][0] + qw * gR[2][1] - 2.0 * qx * gR[2][2]);
        const double gy = 2.0 * (-2.0 * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] +
                                 qz * gR[1][2] - qw * gR[2][0] + qz * gR[2][1] - 2.0 * qy * gR[2][2]);
        const double gz = 2.0 * (-2.0 * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] -
                                 2.0 * qz * gR[1][1] + qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
        const double qd = qw * gw + qx * gx + qy * gy + qz * gz;
        // camera-space mean: 2D mean, depth, Jacobian
        const double gu = gin[0], gv = gin[1];
        double gt0 = gu * V.fx * iz, gt1 = gv * V.fy * iz;
        double gt2 = -(gu * V.fx * tx + gv * V.fy * ty) * iz * iz + gin[9];
        const double iz2 = iz * iz;
        for (int j = 0; j < 3; ++j) {
            const double w0 = V.R[j], w1 = V.R[3 + j], w2 = V.R[6 + j];
            if (!xcl) {
                gt0 += gM[0][j] * (-V.fx * iz2 * w2);
                gt2 += gM[0][j] * (-V.fx * iz2 * w0 + 2.0 * V.fx * xr * iz2 * w2);
            } else {
                gt2 += gM[0][j] * (-V.fx * iz2 * (w0 - xr * w2));
            }
            if (!ycl) {
                gt1 += gM[1][j] * (-V.fy * iz2 * w2);
                gt2 += gM[1][j] * (-V.fy * iz2 * w1 + 2.0 * V.fy * yr * iz2 * w2);
            } else {
                gt2 += gM[1][j] * (-V.fy * iz2 * (w1 - yr * w2));
            }
        }
        double gmu[3];
        for (int j = 0; j < 3; ++j) gmu[j] = V.R[j] * gt0 + V.R[3 + j] * gt1 + V.R[6 + j] * gt2;
        // colour: SH coefficients and the view direction
        const double dn = sqrt(dx * dx + dy * dy + dz * dz), idn = 1.0 / dn;
        const double ux = dx * idn, uy = dy * idn, uz = dz * idn;
        double Y[16], dY[16][3];
        sh_basis_grad<DEG>(ux, uy, uz, Y, dY);
        double gdir[3] = {0.0, 0.0, 0.0};
        double gcm[3] = {0.0, 0.0, 0.0};                              // colour gradient, 0 where clamped
        for (int c = 0; c < 3; ++c) {
            const double gc = gin[6 + c];
            if (gc == 0.0) continue;
            double val = 0.5, d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double f = a.sh[((int64_t)g * K + k) * 3 + c];
                val += f * Y[k];
                d0 += f * dY[k][0];
                d1 += f * dY[k][1];
                d2 += f * dY[k][2];
            }
            if (val < 0.0 || val > 1.0) continue;                       // clamped colour
            gcm[c] = gc;
            gdir[0] += gc * d0;
            gdir[1] += gc * d1;
            gdir[2] += gc * d2;
        }
        const double dd = ux * gdir[0] + uy * gdir[1] + uz * gdir[2];
        gmu[0] += (gdir[0] - ux * dd) * idn;
        gmu[1] += (gdir[1] - uy * dd) * idn;
        gmu[2] += (gdir[2] - uz * dd) * idn;
        float4* rec = reinterpret_cast<float4*>(a.rec + (size_t)p * kEntryRec);
        rec[0] = make_float4((float)gmu[0], (float)gmu[1], (float)gmu[2], (float)gsc[0]);
        rec[1] = make_float4((float)gsc[1], (float)gsc[2], (float)((gw - qw * qd) / qn), (float)((gx - qx * qd) / qn));
        rec[2] = make_float4((float)((gy - qy * qd) / qn), (float)((gz - qz * qd) / qn), (float)gin[5], (float)gcm[0]);
        rec[3] = make_float4((float)gcm[1], (float)gcm[2], (float)ux, (float)uy);
        rec[4] = make_float4((float)uz, 0.f, 0.f, 0.f);
    }
}

// Entry records in Gaussian order: thread p starts a run when its key
// differs from the previous one and sums the run's records; the SH
// coefficients' gradients are sum_entries g_c Y_k(d_entry).  One thread per
// Gaussian, so the outputs are updated without atomics.
template <int DEG>
__global__ __launch_bounds__(256) void k_gather_bwd(GatherArgs a) {
    const uint32_t m = min(a.ctr->cut, a.cap);
    constexpr int K = (DEG + 1) * (DEG + 1);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
        const uint32_t key = a.keys[p];
        if (p > 0 && a.keys[p - 1] == key) continue;
        float acc[11];
#pragma unroll
        for (int t = 0; t < 11; ++t) acc[t] = 0.f;
        float sh[3 * K];
#pragma unroll
        for (int t = 0; t < 3 * K; ++t) sh[t] = 0.f;
        bool any = false;
        for (uint32_t q = p; q < m && a.keys[q] == key; ++q) {
            const float4* rec = reinterpret_cast<const float4*>(a.rec + (size_t)q * kEntryRec);
            const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3], r4 = rec[4];
            const float v[11] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z};
#pragma unroll
            for (int t = 0; t < 11; ++t) {
                acc[t] += v[t];
                any = any || v[t] != 0.f;
            }
            const float gc[3] = {r2.w, r3.x, r3.y};
            if (gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f) {
                any = true;
                double Y[16], dY[16][3];
                sh_basis_grad<DEG>(r3.z, r3.w, r4.x, Y, dY);
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) sh[k * 3 + c] += (float)(gc[c] * Y[k]);
            }
        }
        if (!any) continue;
        const size_t g = key;
#pragma unroll
        for (int t = 0; t < 3; ++t) a.g_means[3 * g + t] += acc[t];
#pragma unroll
        for (int t = 0; t < 3; ++t) a.g_scales[3 * g + t] += acc[3 + t];
#pragma unroll
        for (int t = 0; t < 4; ++t) a.g_quats[4 * g + t] += acc[6 + t];
        a.g_opacity[g] += acc[10];
#pragma unroll
        for (int t = 0; t < 3 * K; ++t) a.g_sh[g * 3 * K + t] += sh[t];
    }
}

__global__ void k_entry_keys(const uint2* cut, const Counters* ctr, uint32_t cap, uint32_t* keys, uint32_t* vals) {
    const uint32_t m = min(ctr->cut, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        keys[i] = cut[i].x;
        vals[i] = i;
    }
}

}  // namespace

void launch_backward_composite(const BwdArgs& b, const Counters* ctr, hipStream_t s) {
    k_zero_egrad<<<1024, 256, 0, s>>>(b.egrad, ctr, b.cut_cap);
    if (b.total_tiles) k_composite_bwd<<<b.total_tiles, kNT, 0, s>>>(b);
}

void launch_backward_params(ProjBwdArgs p, SortArgs sa, GatherArgs ga, hipStream_t s) {
    // the entries in Gaussian order: the chain rule reads each Gaussian's
    // parameters for its views in a row and writes the records in that
    // order, which the sum then reads sequentially
    k_entry_keys<<<2048, 256, 0, s>>>(p.cut, p.ctr, p.cut_cap, sa.keys[0], sa.vals[0]);
    const int r = launch_sort(sa, s);
    p.order = sa.vals[r];
    ga.keys = sa.keys[r];
    switch (p.sh_degree) {
        case 0: k_project_bwd<0><<<2048, 256, 0, s>>>(p); break;
        case 1: k_project_bwd<1><<<2048, 256, 0, s>>>(p); break;
        case 2: k_project_bwd<2><<<2048, 256, 0, s>>>(p); break;
        default: k_project_bwd<3><<<2048, 256, 0, s>>>(p); break;
    }
    switch (ga.sh_degree) {
        case 0: k_gather_bwd<0><<<2048, 256, 0, s>>>(ga); break;
        case 1: k_gather_bwd<1><<<2048, 256, 0, s>>>(ga); break;
        case 2: k_gather_bwd<2><<<2048, 256, 0, s>>>(ga); break;
        default: k_gather_bwd<3><<<2048, 256, 0, s>>>(ga); break;
    }
}

}  // namespace hgs
