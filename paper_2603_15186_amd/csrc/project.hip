// EWA projection of the cut's Gaussians with spherical-harmonic colour, and
// pair emission in depth order.
//
// Per cut entry (node, view): Sigma = R S S^T R^T (Supplementary Material of
// NavGSim), camera-space mean t = W (mu - o), first-order perspective
// Jacobian J at the mean (x/z and y/z clamped to the image's range widened
// by 15 % of its size per side), Sigma' = J W Sigma W^T J^T + 0.3 I, 2D mean (fx tx/tz + cx,
// fy ty/tz + cy), colour clamp(sum_k f_k Y_k(d) + 0.5, 0, 1).
//
// The geometry runs in FP64 (the pass is bound by HBM traffic; FP64 keeps
// the conic of edge-on sheets accurate).  Sigma' is formed as T T^T with
// T = J W R S (2x3), which is symmetric positive semidefinite by
// construction.  The depth key is the single-precision value of the FP64
// camera depth, whose three-term sum is evaluated in a fixed order with
// contraction disabled, so the depth order is an exact, reproducible result.
#include "device_util.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = 256;
// Binning covers q <= 9 (1 + kBinSlack): a superset of every pixel the
// compositor can take, whatever the rounding of its single-precision q.
constexpr double kBinSlack = 1e-3;

// Real spherical-harmonic basis (Condon-Shortley phase) up to degree 3 as
// Cartesian polynomials of the unit direction; index l*l + l + m.
// Constants: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) times the polynomial's
// normalising factor, e.g. 0.5 sqrt(1/pi), sqrt(3/(4 pi)), 0.5 sqrt(15/pi),
// 0.25 sqrt(5/pi), 0.25 sqrt(15/pi), 0.25 sqrt(35/(2 pi)), 0.5 sqrt(105/pi),
// 0.25 sqrt(21/(2 pi)), 0.25 sqrt(7/pi), 0.25 sqrt(105/pi).
// With Blend, coefficient f of node g becomes f_p + t (f_g - f_p) with f_p
// that of node pg (pg < 0: no blending).  The coefficients of a Gaussian are
// one contiguous run of 3 K floats ([k][c]), read with 16-byte loads when
// 3 K is a multiple of four.
template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t g, float f[3 * (DEG + 1) * (DEG + 1)]) {
    constexpr int NF = 3 * (DEG + 1) * (DEG + 1);
    const float* src = sh + g * NF;
    if constexpr (NF % 4 == 0) {
#pragma unroll
        for (int q = 0; q < NF / 4; ++q) {
            const float4 v = reinterpret_cast<const float4*>(src)[q];
            f[4 * q] = v.x;
            f[4 * q + 1] = v.y;
            f[4 * q + 2] = v.z;
            f[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NF; ++q) f[q] = src[q];
    }
}

template <bool Blend, int DEG>
__device__ __forceinline__ void sh_colour(const float* __restrict__ sh, int64_t g, int64_t pg, float t, float x,
                                          float y, float z, float rgb[3]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr float k00 = 0.28209479177387814f;
    constexpr float k1 = 0.48860251190291992f;
    constexpr float k2a = 1.0925484305920792f, k2b = 0.31539156525252005f, k2c = 0.54627421529603959f;
    constexpr float k3a = 0.59004358992664352f, k3b = 2.8906114426405538f, k3c = 0.45704579946446572f,
                    k3d = 0.3731763325901154f, k3e = 1.4453057213202769f;
    float Y[16];
    Y[0] = k00;
    if constexpr (DEG >= 1) {
        Y[1] = -k1 * y;
        Y[2] = k1 * z;
        Y[3] = -k1 * x;
    }
    if constexpr (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = k2a * x * y;
        Y[5] = -k2a * y * z;
        Y[6] = k2b * (3.f * zz - 1.f);
        Y[7] = -k2a * x * z;
        Y[8] = k2c * (xx - yy);
        if constexpr (DEG >= 3) {
            Y[9] = -k3a * y * (3.f * xx - yy);
            Y[10] = k3b * x * y * z;
            Y[11] = -k3c * y * (5.f * zz - 1.f);
            Y[12] = k3d * z * (5.f * zz - 3.f);
            Y[13] = -k3c * x * (5.f * zz - 1.f);
            Y[14] = k3e * z * (xx - yy);
            Y[15] = -k3a * x * (xx - 3.f * yy);
        }
    }
    float f[3 * K];
    load_sh<DEG>(sh, g, f);
    if (Blend && pg >= 0) {
        float fp[3 * K];
        load_sh<DEG>(sh, pg, fp);
#pragma unroll
        for (int q = 0; q < 3 * K; ++q) f[q] = fp[q] + t * (f[q] - fp[q]);
    }
    float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fmaf(f[3 * k + c], Y[k], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) rgb[c] = fminf(fmaxf(acc[c], 0.f), 1.f);
}

// Conic of a projected entry, rebuilt from its stored single-precision
// factors (the same inputs in the counting and the emitting pass).
__device__ __forceinline__ void conic_of(const Proj& p, double* A, double* B, double* C) {
    const double pp = p.p, rr = p.r, ss = p.s;
    *A = pp * pp;
    *B = pp * rr;
    *C = rr * rr + ss * ss;
}

// Tiles of one tile row that the ellipse q(d) <= Q reaches.  The ellipse
// meets the row's band of pixel-centre heights [yb0, yb1] (relative to the
// mean) in a convex set whose x-extent [xa, xb] is found in closed form: for
// a height dy the ellipse spans dx = (-B dy +- sqrt(A Q - det dy^2)) / A, a
// concave right end and convex left end whose extremes over the band sit at
// the clamped heights of the ellipse's rightmost and leftmost points.  A
// tile is reached iff its pixel-centre x-range overlaps [xa, xb]; the
// result is an interval of tiles (empty: lo > hi).
struct RowSpan {
    double A, B, C, det, Q, ey, ymax_at_x;   // ymax_at_x: height of the rightmost point
};

__device__ __forceinline__ RowSpan row_span_init(const Proj& p) {
    RowSpan r;
    conic_of(p, &r.A, &r.B, &r.C);
    r.det = r.A * r.C - r.B * r.B;
    r.Q = 9.0 * (1.0 + kBinSlack);
    // covariance = inverse conic: Sxx = C/det, Syy = A/det, Sxy = -B/det
    r.ey = sqrt(r.Q * r.A / r.det);
    const double sxx = r.C / r.det, sxy = -r.B / r.det;
    r.ymax_at_x = sxy * sqrt(r.Q / sxx);
    return r;
}

// x-extent [xa, xb] (absolute pixels) of the ellipse within the band of
// pixel-centre heights [ya, yb] (absolute); false if they do not meet.
__device__ __forceinline__ bool band_span(const RowSpan& r, double u, double v, double ya, double yb, double* xa,
                                          double* xb) {
    double y0 = fmax(ya - v, -r.ey);
    double y1 = fmin(yb - v, r.ey);
    if (y0 > y1) return false;
    const double yr = fmin(fmax(r.ymax_at_x, y0), y1);
    const double yl = fmin(fmax(-r.ymax_at_x, y0), y1);
    const double sr = fmax(r.A * r.Q - r.det * yr * yr, 0.0);
    const double sl = fmax(r.A * r.Q - r.det * yl * yl, 0.0);
    *xb = u + (-r.B * yr + sqrt(sr)) / r.A + 1e-7;
    *xa = u + (-r.B * yl - sqrt(sl)) / r.A - 1e-7;
    return true;
}

// Tiles [lo, hi] of tile row ty (tiles of tw x th pixels) that the ellipse
// reaches, within [tx_lo, tx_hi]; lo > hi when none.
__device__ __forceinline__ void row_tiles(const RowSpan& r, double u, double v, int ty, int tw, int th, int H,
                                          int tx_lo, int tx_hi, int* lo, int* hi) {
    double xa, xb;
    const double ya = ty * th + 0.5, yb = fmin((double)(ty * th + th - 1), (double)(H - 1)) + 0.5;
    if (!band_span(r, u, v, ya, yb, &xa, &xb)) {
        *lo = 1;
        *hi = 0;
        return;
    }
    // tile tx covers pixel centres [tw tx + 0.5, tw tx + tw - 0.5]
    const int a = (int)ceil((xa - (tw - 0.5)) / tw);
    const int b = (int)floor((xb - 0.5) / tw);
    *lo = a > tx_lo ? a : tx_lo;
    *hi = b < tx_hi ? b : tx_hi;
}

// Number of tiles of rect `rc` that the ellipse reaches (all of them when
// exact is false).
__device__ __forceinline__ uint32_t count_tiles(const Proj& p, ushort4 rc, int tw, int th, int H, bool exact) {
    const uint32_t all = (uint32_t)(rc.z - rc.x + 1) * (uint32_t)(rc.w - rc.y + 1);
    if (!exact || all <= 1) return all;
    const RowSpan r = row_span_init(p);
    uint32_t n = 0;
    for (int ty = rc.y; ty <= rc.w; ++ty) {
        int lo, hi;
        row_tiles(r, p.u, p.v, ty, tw, th, H, rc.x, rc.z, &lo, &hi);
        n += hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
    }
    return n;
}

// Rows of T = M R diag(s) for the Gaussian with quaternion (w, x, y, z) =
// q and scales sc, and the entries of T T^T.
__device__ __forceinline__ void proj_cov(const double M0[3], const double M1[3], float4 q, float4 sc, double* a00,
                                         double* a01, double* a11) {
    double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
    const double qi = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qi; qx *= qi; qy *= qi; qz *= qi;
    const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                          2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                          2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
    const double s[3] = {sc.x, sc.y, sc.z};
    double T0[3], T1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T0[k] = (M0[0] * Rq[k] + M0[1] * Rq[3 + k] + M0[2] * Rq[6 + k]) * s[k];
        T1[k] = (M1[0] * Rq[k] + M1[1] * Rq[3 + k] + M1[2] * Rq[6 + k]) * s[k];
    }
    *a00 = T0[0] * T0[0] + T0[1] * T0[1] + T0[2] * T0[2];
    *a01 = T0[0] * T1[0] + T0[1] * T1[1] + T0[2] * T1[2];
    *a11 = T1[0] * T1[0] + T1[1] * T1[1] + T1[2] * T1[2];
}

// Projected bounding-sphere size 2 max(fx, fy) r / |c - o| in pixels, FP64
// in the cut's order of operations.
__device__ __forceinline__ double sphere_size(const ViewDev& V, float4 b) {
#pragma clang fp contract(off)
    const double bx = (double)b.x - V.o[0], by = (double)b.y - V.o[1], bz = (double)b.z - V.o[2];
    const double d2 = (bx * bx + by * by) + bz * bz;
    return V.f2 * (double)b.w / sqrt(d2);
}

// Blend: level-of-detail transition blending.  Node g with parent p takes
// the weight t = clamp((s_p - tau) / (s_p - s_g), 0, 1) of the projected
// bounding-sphere sizes of p and g (t = 1 when s_g >= s_p), and is projected
// as the Gaussian with mean mu_p + t (mu_g - mu_p), covariance Sigma_p +
// t (Sigma_g - Sigma_p) (formed after projection as (1 - t) T_p T_p^T +
// t T_g T_g^T, positive semidefinite by construction) and SH coefficients
// interpolated alike.  Opacity: the first of p's children in the view's cut
// carries o_p + t (o_g - o_p), the others t o_g, so that at the refine
// decision (s_p = tau, t = 0 for every child) exactly one copy of p is drawn
// and, at the node's own decision (s_g = tau, t = 1), the node itself: the
// image is continuous across both.  The cut lists a parent's children that
// it holds next to each other in ascending order (they are decided in one
// level pass, in frontier order), so g is that first child unless the entry
// before it is a sibling of the same view.  The blended mean and depth key
// follow the same FP64 steps as the unblended ones.
template <bool Blend, int DEG>
__global__ __launch_bounds__(kNT) void k_project(ProjectArgs a) {
    constexpr int kWords = (int)(sizeof(ViewDev) / 8);
    __shared__ uint64_t s_view[kProjectLdsViews * kWords];
    const uint32_t m = min(a.ctr->cut, a.cut_cap);
    if (a.lds_views) {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(a.views);
        for (int k = threadIdx.x; k < a.n_views * kWords; k += kNT) s_view[k] = src[k];
        __syncthreads();
    }
    uint32_t vis = 0;
    for (uint32_t i = blockIdx.x * kNT + threadIdx.x; i < m; i += gridDim.x * kNT) {
        const uint2 e = a.cut[i];
        ViewDev V;
        if (a.lds_views) {
            uint64_t wd[kWords];
#pragma unroll
            for (int q = 0; q < kWords; ++q) wd[q] = s_view[e.y * kWords + q];
            __builtin_memcpy(&V, wd, sizeof V);
        } else {
            V = load_view(a.views, e.y);
        }
        const int64_t g = e.x;
        const float4 g0 = a.geo[3 * g], g1 = a.geo[3 * g + 1], g2 = a.geo[3 * g + 2];
        int64_t pg = -1;
        double t = 1.0;
        bool first = true;
        float4 p0 = g0;
        if (Blend) {
            const int32_t par = a.parent[g];
            if (par >= 0) {
                const double sp = sphere_size(V, a.bound[par]), sg = sphere_size(V, a.bound[g]);
                if (sg < sp) {
#pragma clang fp contract(off)
                    t = (sp - V.tau) / (sp - sg);
                    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                }
                if (i > 0) {
                    const uint2 q = a.cut[i - 1];
                    first = !(q.y == e.y && (int64_t)q.x >= (int64_t)a.child[par].x && (int64_t)q.x < g);
                }
                if (t < 1.0) {
                    pg = par;
                    p0 = a.geo[3 * pg];
                }
            }
        }
        double dx, dy, dz, tx, ty, tz;
        double op = g0.w;
        {
#pragma clang fp contract(off)
            double mx = g0.x, my = g0.y, mz = g0.z;
            if (Blend && pg >= 0) {
                mx = (double)p0.x + t * ((double)g0.x - (double)p0.x);
                my = (double)p0.y + t * ((double)g0.y - (double)p0.y);
                mz = (double)p0.z + t * ((double)g0.z - (double)p0.z);
                op = first ? (double)p0.w + t * ((double)g0.w - (double)p0.w) : t * (double)g0.w;
            }
            dx = mx - V.o[0];
            dy = my - V.o[1];
            dz = mz - V.o[2];
            tx = (V.R[0] * dx + V.R[1] * dy) + V.R[2] * dz;
            ty = (V.R[3] * dx + V.R[4] * dy) + V.R[5] * dz;
            tz = (V.R[6] * dx + V.R[7] * dy) + V.R[8] * dz;
        }
        Proj p = {};
        uint32_t ntiles = 0;
        ushort4 rc = make_ushort4(1, 1, 0, 0);
        const float zf = (float)tz;
        if (tz > V.znear) {
            const double iz = 1.0 / tz;
            double xr = tx * iz, yr = ty * iz;
            xr = fmin(fmax(xr, V.xlo), V.xhi);
            yr = fmin(fmax(yr, V.ylo), V.yhi);
            // M = J W (2x3)
            double M0[3], M1[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                M0[j] = V.fx * iz * (V.R[j] - xr * V.R[6 + j]);
                M1[j] = V.fy * iz * (V.R[3 + j] - yr * V.R[6 + j]);
            }
            double c00, c01, c11;
            proj_cov(M0, M1, g1, g2, &c00, &c01, &c11);
            if (Blend && pg >= 0) {
                double b00, b01, b11;
                proj_cov(M0, M1, a.geo[3 * pg + 1], a.geo[3 * pg + 2], &b00, &b01, &b11);
                const double u = 1.0 - t;
                c00 = u * b00 + t * c00;
                c01 = u * b01 + t * c01;
                c11 = u * b11 + t * c11;
            }
            const double s00 = c00 + 0.3;
            const double s01 = c01;
            const double s11 = c11 + 0.3;
            const double det = s00 * s11 - s01 * s01;
            if (det > 0.0) {
                const double u = V.fx * tx * iz + V.cx;
                const double v = V.fy * ty * iz + V.cy;
                // q = (p dx + r dy)^2 + (s dy)^2 with p^2 = s11/det,
                // p r = -s01/det, r^2 + s^2 = s00/det
                const double is11 = 1.0 / s11;
                p.u = u;
                p.v = v;
                p.p = (float)sqrt(s11 / det);
                p.r = (float)(-s01 / sqrt(det * s11));
                p.s = (float)sqrt(is11);
                p.opacity = (float)op;
                p.z = zf;
                // pixel-centre bounding box of q <= 9 (1 + slack)
                const double qm = 9.0 * (1.0 + kBinSlack);
                const double ex = sqrt(qm * s00) + 1e-6, ey = sqrt(qm * s11) + 1e-6;
                const double px0 = ceil(u - ex - 0.5), px1 = floor(u + ex - 0.5);
                const double py0 = ceil(v - ey - 0.5), py1 = floor(v + ey - 0.5);
                const double cx0 = fmax(px0, 0.0), cx1 = fmin(px1, (double)(V.width - 1));
                const double cy0 = fmax(py0, 0.0), cy1 = fmin(py1, (double)(V.height - 1));
                if (cx0 <= cx1 && cy0 <= cy1) {
                    rc = make_ushort4((unsigned short)((int)cx0 / a.tile_w), (unsigned short)((int)cy0 / a.tile_h),
                                      (unsigned short)((int)cx1 / a.tile_w), (unsigned short)((int)cy1 / a.tile_h));
                    ntiles = count_tiles(p, rc, a.tile_w, a.tile_h, V.height, a.exact_tiles);
                }
                if (ntiles > 0) {
                    const double id = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                    float rgb[3];
                    sh_colour<Blend, DEG>(a.sh, g, pg, (float)t, (float)(dx * id), (float)(dy * id),
                                          (float)(dz * id), rgb);
                    p.c0 = rgb[0];
                    p.c1 = rgb[1];
                    p.c2 = rgb[2];
                }
            }
        }
        a.proj[i] = p;
        BinRec br;
        br.rc = rc;
        br.tile_base = e.y << a.key_shift;
        br.tiles_x = (uint16_t)V.tiles_x;
        br.height = (uint16_t)V.height;
        a.bins[i] = br;
        a.ntiles[i] = ntiles;
        // positive depths order as their bit patterns, and so do their
        // offsets from depth_base; unbinned entries last
        uint32_t dk = 0xffffffffu;
        if (ntiles > 0) {
            const uint32_t bits = __float_as_uint(zf);
            if (bits < a.depth_base || bits > a.depth_top) atomicOr(&a.ctr->overflow, kOvDepth);
            dk = bits - a.depth_base;
            if (a.view_shift > 0) dk |= e.y << a.view_shift;
        }
        a.depth_key[i] = dk;
        a.depth_val[i] = i | (min(ntiles, kNtSat) << kNtShift);
        vis += ntiles > 0 ? 1u : 0u;
    }
    vis = wave_sum(vis);
    if (lane_id() == 0 && vis) atomicAdd(&a.ctr->visible, vis);
}

// ---------------------------------------------------------------- emission

struct ScanCtx {
    const uint32_t* order;
    const uint32_t* ntiles;
    const uint32_t* count;
    uint32_t cap;
    uint32_t* offsets;
    uint4* tmp;
    Counters* ctr;
    uint32_t pair_cap;
};

// Tile count of a depth-sorted value: carried in its top bits unless
// saturated.
__device__ __forceinline__ uint32_t tiles_of(const ScanCtx& c, uint32_t val, uint32_t n) {
    const uint32_t nt = val >> kNtShift, e = val & kEntryMask;
    return nt < kNtSat ? nt : (e < n ? c.ntiles[e] : 0u);
}

__device__ __forceinline__ void chunk_of(uint32_t n, int G, int b, uint32_t* lo, uint32_t* hi) {
    uint32_t chunk = ceil_div(n, (uint32_t)G);
    if (chunk < (uint32_t)kNT) chunk = kNT;
    chunk = ceil_div(chunk, (uint32_t)kNT) * kNT;
    uint64_t s = (uint64_t)b * chunk, e = s + chunk;
    *lo = (uint32_t)(s < n ? s : n);
    *hi = (uint32_t)(e < n ? e : n);
}

__global__ __launch_bounds__(kNT) void k_scan_reduce(ScanCtx c) {
    __shared__ uint32_t sh[kNT / kWave + 1];
    const uint32_t n = min(*c.count, c.cap);
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, &lo, &hi);
    uint32_t acc = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kNT) acc += tiles_of(c, c.order[i], n);
    uint32_t tot;
    block_excl_scan<kNT>(acc, sh, &tot);
    if (threadIdx.x == 0) c.tmp[blockIdx.x] = make_uint4(tot, 0, 0, 0);
}

// Exclusive scan of the G <= 4 * 1024 block counts (four consecutive ones
// per thread); the total is also summed in 64 bits so that pair counts
// beyond 2^32 are caught as overflow.
__global__ __launch_bounds__(1024) void k_scan_blocks(ScanCtx c, int G) {
    __shared__ uint32_t sh[1024 / kWave + 1];
    __shared__ unsigned long long sh64[1024 / kWave];
    const int t = threadIdx.x;
    uint32_t x[4], sum = 0;
    unsigned long long sum64 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        x[j] = b < G ? c.tmp[b].x : 0u;
        sum += x[j];
        sum64 += x[j];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<1024>(sum, sh, &tot);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        if (b < G) c.tmp[b].x = ex;
        ex += x[j];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) sum64 += __shfl_xor(sum64, o, kWave);
    if (lane_id() == 0) sh64[t / kWave] = sum64;
    __syncthreads();
    if (t == 0) {
        unsigned long long total = 0;
        for (int w = 0; w < 1024 / kWave; ++w) total += sh64[w];
        Counters* k = c.ctr;
        if (total > c.pair_cap) {
            k->overflow |= kOvPairs;
            const uint32_t need = (uint32_t)(total < 0xffffffffull ? total : 0xffffffffull);
            if (need > k->need_pairs) k->need_pairs = need;
        }
        k->pairs = total < c.pair_cap ? (uint32_t)total : c.pair_cap;
    }
}

__global__ __launch_bounds__(kNT) void k_scan_write(ScanCtx c) {
    __shared__ uint32_t sh[kNT / kWave + 1];
    const uint32_t n = min(*c.count, c.cap);
    uint32_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, &lo, &hi);
    if (lo >= hi) return;
    uint32_t off = c.tmp[blockIdx.x].x;
    for (uint32_t s = lo; s < hi; s += kNT) {
        const uint32_t i = s + threadIdx.x;
        uint32_t x = 0;
        if (i < hi) x = tiles_of(c, c.order[i], n);
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kNT>(x, sh, &tot);
        if (i < hi) c.offsets[i] = off + ex;
        off += tot;
    }
}

// Pairs of one depth-ordered entry, handed to put(k, tile) in order.
template <class F>
__device__ __forceinline__ void entry_tiles(const EmitArgs& a, uint32_t e, uint32_t nt, const BinRec& br, F put) {
    const ushort4 rc = br.rc;
    const uint32_t tw = br.tiles_x;
    const uint32_t all = (uint32_t)(rc.z - rc.x + 1) * (uint32_t)(rc.w - rc.y + 1);
    uint32_t k = 0;
    // the exact set is part of the rectangle: equal counts mean all of it
    if (!a.exact_tiles || nt == all) {
        for (int ty = rc.y; ty <= rc.w; ++ty)
            for (int tx = rc.x; tx <= rc.z; ++tx) put(k++, br.tile_base + (uint32_t)ty * tw + (uint32_t)tx);
        return;
    }
    const Proj p = a.proj[e];
    const RowSpan r = row_span_init(p);
    for (int ty = rc.y; ty <= rc.w; ++ty) {
        int lo, hi;
        row_tiles(r, p.u, p.v, ty, a.tile_w, a.tile_h, br.height, rc.x, rc.z, &lo, &hi);
        for (int tx = lo; tx <= hi; ++tx) put(k++, br.tile_base + (uint32_t)ty * tw + (uint32_t)tx);
    }
}

// Each workgroup expands 256 consecutive depth-ordered entries into their
// (tile, entry) pairs, which form one contiguous run of the pair arrays:
// the run is assembled in LDS and written out coalesced; pairs past the
// staging capacity are stored directly.
constexpr uint32_t kEmitStage = 2048;

__global__ __launch_bounds__(kNT) void k_emit(EmitArgs a) {
    __shared__ uint32_t s_key[kEmitStage];
    __shared__ uint32_t s_val[kEmitStage];
    __shared__ uint32_t s_base, s_end;
    const uint32_t m = min(a.ctr->cut, a.cut_cap);
    const uint32_t cap = a.pair_cap;
    for (uint32_t first = blockIdx.x * kNT; first < m; first += gridDim.x * kNT) {
        const uint32_t i = first + threadIdx.x;
        uint32_t e = 0, nt = 0, pos = 0;
        if (i < m) {
            const uint32_t val = a.order[i];
            e = val & kEntryMask;
            nt = val >> kNtShift;
            if (nt == kNtSat) nt = e < m ? a.ntiles[e] : 0u;
            pos = a.offsets[i];
        }
        if (threadIdx.x == 0) {
            s_base = pos;
            s_end = pos;
        }
        __syncthreads();
        const uint32_t base = s_base;
        if (nt) {
            atomicMax(&s_end, pos + nt);
            const BinRec br = a.bins[e];
            const uint32_t lp = pos - base;
            entry_tiles(a, e, nt, br, [&](uint32_t k, uint32_t tile) {
                const uint32_t L = lp + k;
                if (L < kEmitStage) {
                    s_key[L] = tile;
                    s_val[L] = e;
                } else if (pos + k < cap) {
                    a.keys[pos + k] = tile;
                    a.vals[pos + k] = e;
                }
            });
        }
        __syncthreads();
        const uint32_t len = min(s_end - base, kEmitStage);
        for (uint32_t q = threadIdx.x; q < len; q += kNT) {
            if (base + q < cap) {
                a.keys[base + q] = s_key[q];
                a.vals[base + q] = s_val[q];
            }
        }
        __syncthreads();
    }
}

}  // namespace

__global__ void k_view_keys(const uint32_t* __restrict__ order, const uint2* __restrict__ cut, const uint32_t* count,
                            uint32_t cap, uint32_t* __restrict__ keys) {
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t e = order[i] & kEntryMask;
        keys[i] = e < n ? cut[e].y : 0u;
    }
}

template <bool Blend>
void launch_project_b(const ProjectArgs& a, hipStream_t s) {
    switch (a.sh_degree) {
        case 0: k_project<Blend, 0><<<4096, kNT, 0, s>>>(a); break;
        case 1: k_project<Blend, 1><<<4096, kNT, 0, s>>>(a); break;
        case 2: k_project<Blend, 2><<<4096, kNT, 0, s>>>(a); break;
        default: k_project<Blend, 3><<<4096, kNT, 0, s>>>(a); break;
    }
}

void launch_project(const ProjectArgs& a, hipStream_t s) {
    if (a.blend)
        launch_project_b<true>(a, s);
    else
        launch_project_b<false>(a, s);
}

void launch_view_keys(const uint32_t* order, const uint2* cut, const uint32_t* count, uint32_t cap, uint32_t* keys,
                      hipStream_t s) {
    k_view_keys<<<2048, 256, 0, s>>>(order, cut, count, cap, keys);
}

void launch_emit(const EmitArgs& a, hipStream_t s) {
    const int G = kCutBlocks;
    static_assert(kCutBlocks <= 4 * 1024, "the block scan takes four counts per thread");
    ScanCtx c;
    c.order = a.order;
    c.ntiles = a.ntiles;
    c.count = &a.ctr->cut;
    c.cap = a.cut_cap;
    c.offsets = a.offsets;
    c.tmp = a.scan_tmp;
    c.ctr = a.ctr;
    c.pair_cap = a.pair_cap;
    k_scan_reduce<<<G, kNT, 0, s>>>(c);
    k_scan_blocks<<<1, 1024, 0, s>>>(c, G);
    k_scan_write<<<G, kNT, 0, s>>>(c);
    k_emit<<<8192, kNT, 0, s>>>(a);
}

}  // namespace hgs
