// GS-slice occupancy: the scene's Gaussians cut by horizontal planes,
// rasterised into a 2D grid per plane and into their union (the collision
// map of Sec. III-C).
//
// Per Gaussian, in FP64: the inverse covariance C = R diag(1/s^2) R^T; the
// slice at height z is a 2D Gaussian with amplitude exp(-lambda (z-mu_z)^2/2),
// centre (mu_x, mu_y) - (z - mu_z)(alpha, beta) and inverse covariance the xy
// block of C, where (alpha, beta) solves the 2x2 system of that block with
// right-hand side (c_xz, c_yz) and lambda = c_zz - (alpha, beta) . (c_xz, c_yz)
// (Supplementary derivation; the printed second exponent's missing -1/2 is
// restored).  The Gaussian is solid where o a(z) exp(-q/2) >= rho_min, i.e.
// inside q <= 2 ln(o a(z) / rho_min); a cell (closed square) is marked when
// that ellipse meets it, found from the least value of q over the square:
// zero if the centre is inside, else the least over the four edges, each at
// the clamped stationary point of a 1D quadratic.
//
// One thread per Gaussian walks the planes and the cells of each ellipse's
// bounding box; marks are byte stores of 1 (concurrent stores agree).
// Gaussians that reach no plane (floor and ceiling sheets, other floors) are
// dropped after a cheap vertical test, before the FP64 slice algebra.
#include "device_util.h"
#include "grid.h"
#include "internal.h"

namespace hgs {

namespace {

constexpr int kNT = 256;

__global__ void k_fill_zero(uint4* p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_fill_zero_tail(uint8_t* p, size_t from, size_t n) {
    for (size_t i = from + blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Least of q(d) = a dx^2 + 2 b dx dy + c dy^2 over the square
// [qx0, qx0 + w] x [qy0, qy0 + w], d = point - centre (m).
__device__ __forceinline__ double square_min(double a, double b, double c, double mx, double my, double qx0,
                                             double qy0, double w) {
    const double lx = qx0 - mx, hx = qx0 + w - mx;     // x-range of d
    const double ly = qy0 - my, hy = qy0 + w - my;
    if (lx <= 0.0 && hx >= 0.0 && ly <= 0.0 && hy >= 0.0) return 0.0;
    double best = 1e300;
    const double ex[2] = {lx, hx}, ey[2] = {ly, hy};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double dx = ex[s];
        const double dy = fmin(fmax(-b * dx / c, ly), hy);
        best = fmin(best, (a * dx + 2.0 * b * dy) * dx + c * dy * dy);
        const double ey0 = ey[s];
        const double dx2 = fmin(fmax(-b * ey0 / a, lx), hx);
        best = fmin(best, (a * dx2 + 2.0 * b * ey0) * dx2 + c * ey0 * ey0);
    }
    return best;
}

__global__ __launch_bounds__(kNT) void k_slice(SliceArgs s) {
    for (uint32_t t = blockIdx.x * kNT + threadIdx.x; t < s.n; t += gridDim.x * kNT) {
        const int64_t g = s.ids ? (int64_t)s.ids[t] : (int64_t)t;
        const float4 g0 = s.geo[3 * g], g1 = s.geo[3 * g + 1], g2 = s.geo[3 * g + 2];
        // rotation of the normalised quaternion (w, x, y, z); columns = axes
        double qw = g1.x, qx = g1.y, qy = g1.z, qz = g1.w;
        const double qi = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= qi; qx *= qi; qy *= qi; qz *= qi;
        const double R[3][3] = {{1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)},
                                {2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx)},
                                {2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
        // vertical reach: o exp(-dz^2 / (2 Sigma_zz)) >= rho_min needs
        // dz^2 <= 2 Sigma_zz ln(o / rho_min) (lambda = 1 / Sigma_zz); planes
        // beyond it (with a relative margin) cannot be solid
        const double o = g0.w;
        if (!(o >= s.rho_min)) continue;
        const double szz = R[2][0] * R[2][0] * ((double)g2.x * g2.x) + R[2][1] * R[2][1] * ((double)g2.y * g2.y) +
                           R[2][2] * R[2][2] * ((double)g2.z * g2.z);
        const double reach2 = 2.0 * szz * log(o / s.rho_min) * (1.0 + 1e-6) + 1e-12;
        bool any = false;
        for (int k = 0; k < s.n_planes; ++k) {
            const double dz = (double)s.heights[k] - (double)g0.z;
            any = any || dz * dz <= reach2;
        }
        if (!any) continue;
        const double iv[3] = {1.0 / ((double)g2.x * g2.x), 1.0 / ((double)g2.y * g2.y), 1.0 / ((double)g2.z * g2.z)};
        double C[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                C[i][j] = R[i][0] * iv[0] * R[j][0] + R[i][1] * iv[1] * R[j][1] + R[i][2] * iv[2] * R[j][2];
        const double a = C[0][0], b = C[0][1], c = C[1][1];
        const double det = a * c - b * b;
        const double al = (C[0][2] * c - C[1][2] * b) / det;
        const double be = (C[1][2] * a - C[0][2] * b) / det;
        const double lam = C[2][2] - al * C[0][2] - be * C[1][2];
        for (int k = 0; k < s.n_planes; ++k) {
            const double dz = (double)s.heights[k] - (double)g0.z;
            if (dz * dz > reach2) continue;
            const double A = o * exp(-0.5 * lam * dz * dz);
            if (!(A >= s.rho_min)) continue;
            const double r2 = 2.0 * log(A / s.rho_min);
            const double mx = (double)g0.x - al * dz, my = (double)g0.y - be * dz;
            // bounding box of the ellipse (half-extents r sqrt(c/det), r sqrt(a/det)), one cell wider
            const double hx = sqrt(r2 * c / det) + s.cell, hy = sqrt(r2 * a / det) + s.cell;
            const double fi0 = floor((mx - hx - s.x0) / s.cell), fi1 = floor((mx + hx - s.x0) / s.cell);
            const double fj0 = floor((my - hy - s.y0) / s.cell), fj1 = floor((my + hy - s.y0) / s.cell);
            // off the grid (or not finite): nothing to mark
            if (!(fi1 >= 0.0 && fi0 <= (double)(s.nx - 1) && fj1 >= 0.0 && fj0 <= (double)(s.ny - 1))) continue;
            const int i0 = (int)fmax(fi0, 0.0), i1 = (int)fmin(fi1, (double)(s.nx - 1));
            const int j0 = (int)fmax(fj0, 0.0), j1 = (int)fmin(fj1, (double)(s.ny - 1));
            uint8_t* plane = s.occ ? s.occ + (size_t)k * s.nx * s.ny : nullptr;
            for (int j = j0; j <= j1; ++j) {
                const double qy0 = s.y0 + (double)j * s.cell;
                for (int i = i0; i <= i1; ++i) {
                    const double qx0 = s.x0 + (double)i * s.cell;
                    if (square_min(a, b, c, mx, my, qx0, qy0, s.cell) <= r2) {
                        const size_t cidx = (size_t)j * s.nx + i;
                        if (plane) plane[cidx] = 1;
                        if (s.map) s.map[cidx] = 1;
                    }
                }
            }
        }
    }
}

// Disc robots against a map: thread per query.
__global__ __launch_bounds__(kNT) void k_disc_collision(DiscArgs d) {
    for (int64_t q = blockIdx.x * (int64_t)kNT + threadIdx.x; q < d.n; q += (int64_t)gridDim.x * kNT)
        d.out[q] = disc_hits(d.map, d.x0, d.y0, d.cell, d.nx, d.ny, d.xy[2 * q], d.xy[2 * q + 1], d.radius) ? 1 : 0;
}

void zero_bytes(uint8_t* p, size_t n, hipStream_t st) {
    if (!p || n == 0) return;
    const size_t n16 = (reinterpret_cast<uintptr_t>(p) % 16 == 0) ? n / 16 : 0;
    if (n16) k_fill_zero<<<1024, 256, 0, st>>>(reinterpret_cast<uint4*>(p), n16);
    const size_t rest = n - n16 * 16;
    if (rest) k_fill_zero_tail<<<(unsigned)((rest + 255) / 256 < 4096 ? (rest + 255) / 256 : 4096), 256, 0, st>>>(
        p, n16 * 16, n);
}

}  // namespace

void launch_disc_collision(const DiscArgs& d, hipStream_t st) {
    if (d.n == 0) return;
    const int64_t blocks = (d.n + kNT - 1) / kNT;
    k_disc_collision<<<(unsigned)(blocks < 4096 ? blocks : 4096), kNT, 0, st>>>(d);
}

void launch_slice(const SliceArgs& a, hipStream_t st) {
    zero_bytes(a.occ, (size_t)a.n_planes * a.nx * a.ny, st);
    zero_bytes(a.map, (size_t)a.nx * a.ny, st);
    if (a.n) k_slice<<<2048, kNT, 0, st>>>(a);
}

}  // namespace hgs
