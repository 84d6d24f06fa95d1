/*
 * FP64 CPU oracle of the GS-slice occupancy map.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): the test-suite may load it, the
 * renderer never does, and the two share no code.
 *
 * What it follows (NavGSim, arXiv 2603.15186, Sec. III-C and the
 * Supplementary derivation of Gaussian slicing): a Gaussian with inverse
 * covariance C = Sigma^-1 = R S^-1 S^-T R^T, cut by the horizontal plane at
 * height z, is the 2D Gaussian
 *     exp(-1/2 lambda (z - mu_z)^2) exp(-1/2 (x - mu(z))^T C_xy (x - mu(z)))
 * with C_xy the xy block of C, (alpha, beta) the solution of
 *     alpha c_xx + beta c_xy = c_xz,   alpha c_xy + beta c_yy = c_yz,
 * lambda = c_zz - alpha^2 c_xx - beta^2 c_yy - 2 alpha beta c_xy and
 * mu(z) = (mu_x, mu_y) - (z - mu_z) (alpha, beta).  (The printed second
 * exponent lacks the factor -1/2; it is read as the conditional Gaussian.)
 *
 * Occupancy (the paper combines the slices into a 2D map without fixing the
 * rule; the reading used): on plane z, Gaussian g is solid where its
 * opacity-weighted slice o a(z) exp(-q/2) is at least rho_min, i.e. inside
 * the ellipse q <= r^2 = 2 ln(o a(z) / rho_min) when o a(z) >= rho_min.  A
 * grid cell (a closed square) is occupied on a plane when some Gaussian's
 * solid ellipse meets it; the map is the union over the planes.
 *
 * The meeting test is exact: the minimum of the convex quadratic q over the
 * square is 0 when the centre lies in it, else the least of the minima on
 * its four edges, each at the clamped stationary point of a 1D quadratic.
 * Decisions within a relative margin `amb` of their threshold are reported
 * as undecided (value 2), so an independent implementation may take either
 * side there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Inverse covariance entries and slice parameters of one Gaussian:
 * out = (alpha, beta, lambda, cxx, cxy, cyy). */
static void slice_params(const float* s, const float* q, double out[6]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double nq = sqrt(w * w + x * x + y * y + z * z);
    w /= nq; x /= nq; y /= nq; z /= nq;
    /* columns of R are the Gaussian's axes */
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    const double is[3] = {1.0 / ((double)s[0] * s[0]), 1.0 / ((double)s[1] * s[1]), 1.0 / ((double)s[2] * s[2])};
    double C[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += R[3 * i + k] * is[k] * R[3 * j + k];
            C[3 * i + j] = acc;
        }
    const double cxx = C[0], cxy = C[1], cxz = C[2], cyy = C[4], cyz = C[5], czz = C[8];
    const double det = cxx * cyy - cxy * cxy;
    const double alpha = (cxz * cyy - cyz * cxy) / det;
    const double beta = (cyz * cxx - cxz * cxy) / det;
    out[0] = alpha;
    out[1] = beta;
    out[2] = czz - alpha * alpha * cxx - beta * beta * cyy - 2.0 * alpha * beta * cxy;
    out[3] = cxx;
    out[4] = cxy;
    out[5] = cyy;
}

void or_slice_params(int64_t n, const float* scales, const float* quats, double* out) {
    for (int64_t i = 0; i < n; i++) slice_params(scales + 3 * i, quats + 4 * i, out + 6 * i);
}

/* Minimum of q(p) = (p - m)^T [[a, b], [b, c]] (p - m) over [x0, x1] x [y0, y1]. */
static double box_min(double a, double b, double c, double mx, double my, double x0, double x1, double y0,
                      double y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0;
    double best = INFINITY;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int e = 0; e < 2; e++) {
        /* edge x = xs[e]: q = a dx^2 + 2 b dx dy + c dy^2, least at dy = -b dx / c */
        const double dx = xs[e] - mx;
        double dy = -b * dx / c;
        dy = fmin(fmax(dy, y0 - my), y1 - my);
        best = fmin(best, a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
        /* edge y = ys[e] */
        const double ey = ys[e] - my;
        double ex = -b * ey / a;
        ex = fmin(fmax(ex, x0 - mx), x1 - mx);
        best = fmin(best, a * ex * ex + 2.0 * b * ex * ey + c * ey * ey);
    }
    return best;
}

/* occ[k][j][i] (k < n_planes, j < ny, i < nx): 0 free, 1 occupied, 2
 * undecided; cell (i, j) is [x0 + i cell, x0 + (i+1) cell] x [y0 + j cell,
 * y0 + (j+1) cell]. */
void or_slice_occupancy(int64_t n, const float* means, const float* scales, const float* quats,
                        const float* opacity, double x0, double y0, double cell, int32_t nx, int32_t ny,
                        int32_t n_planes, const float* heights, double rho_min, double amb, int8_t* occ) {
    double* P = (double*)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
    or_slice_params(n, scales, quats, P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < n_planes; k++) {
        int8_t* plane = occ + (size_t)k * nx * ny;
        for (int64_t t = 0; t < (int64_t)nx * ny; t++) plane[t] = 0;
        const double z = heights[k];
        for (int64_t g = 0; g < n; g++) {
            const double* p = P + 6 * g;
            const double dz = z - (double)means[3 * g + 2];
            const double A = (double)opacity[g] * exp(-0.5 * p[2] * dz * dz);
            if (A < rho_min * (1.0 - amb)) continue;
            const int borderline_amp = A <= rho_min * (1.0 + amb);
            const double r2 = borderline_amp ? 0.0 : 2.0 * log(A / rho_min);
            const double mx = (double)means[3 * g] - p[0] * dz, my = (double)means[3 * g + 1] - p[1] * dz;
            const double a = p[3], b = p[4], c = p[5];
            const double det = a * c - b * b;
            const double hx = sqrt(r2 * c / det) + cell, hy = sqrt(r2 * a / det) + cell;
            int64_t i0 = (int64_t)floor((mx - hx - x0) / cell), i1 = (int64_t)floor((mx + hx - x0) / cell);
            int64_t j0 = (int64_t)floor((my - hy - y0) / cell), j1 = (int64_t)floor((my + hy - y0) / cell);
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > nx - 1) i1 = nx - 1;
            if (j1 > ny - 1) j1 = ny - 1;
            for (int64_t j = j0; j <= j1; j++)
                for (int64_t i = i0; i <= i1; i++) {
                    const double qx0 = x0 + (double)i * cell, qy0 = y0 + (double)j * cell;
                    const double qm = box_min(a, b, c, mx, my, qx0, qx0 + cell, qy0, qy0 + cell);
                    int8_t* o = plane + (size_t)j * nx + i;
                    if (borderline_amp) {
                        if (qm <= amb && *o == 0) *o = 2;
                        continue;
                    }
                    const double tol = amb * (r2 > 1.0 ? r2 : 1.0);
                    if (qm <= r2 - tol) *o = 1;
                    else if (qm <= r2 + tol && *o == 0) *o = 2;
                }
        }
    }
    free(P);
}

/* Disc robots against a 2D occupancy map: query q at (x, y) with radius
 * rad collides (1) when some occupied cell's closed square lies within
 * distance rad of (x, y), else 0; 2 when the nearest occupied square is
 * within a relative margin amb of rad.  Cells outside the grid are free.
 * Every cell is examined (no search structure). */
void or_disc_collision(const uint8_t* map, double x0, double y0, double cell, int32_t nx, int32_t ny, int64_t n,
                       const double* xy, double rad, double amb, int8_t* out) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++) {
        const double x = xy[2 * q], y = xy[2 * q + 1];
        double best = INFINITY;
        for (int32_t j = 0; j < ny; j++)
            for (int32_t i = 0; i < nx; i++) {
                if (!map[(size_t)j * nx + i]) continue;
                const double ax = x0 + (double)i * cell, ay = y0 + (double)j * cell;
                const double dx = fmax(fmax(ax - x, 0.0), x - (ax + cell));
                const double dy = fmax(fmax(ay - y, 0.0), y - (ay + cell));
                const double d = sqrt(dx * dx + dy * dy);
                if (d < best) best = d;
            }
        out[q] = best <= rad * (1.0 - amb) ? 1 : (best <= rad * (1.0 + amb) ? 2 : 0);
    }
}
