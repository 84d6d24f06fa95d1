/*
 * FP64 CPU oracle of the hierarchical 3D Gaussian Splatting forward render.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow definition that the GPU
 * renderer is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the renderer never does, and the
 * two share no code, header, table or constant.
 *
 * What it follows (NavGSim, arXiv 2603.15186):
 *   - Sec. III-B: the scene is a tree of anisotropic Gaussians; level-of-detail
 *     rendering picks Gaussians from different levels of the tree.
 *   - Eq. (1) and the Supplementary Material: a Gaussian's density is
 *     exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) with Sigma = R S S^T R^T.
 *   - Sec. III-A: a view is defined by the camera intrinsics and extrinsics.
 * The paper defers everything else (projection, compositing, LOD metric) to
 * the hierarchical-3DGS work it builds on; the readings used here are listed
 * with the project's design notes: first-order (EWA) projection with a
 * 0.3 px^2 screen low-pass (Jacobian taken at the mean with x/z and y/z
 * clamped to the image's range widened by 15 % of its size per side), 3-sigma ellipse support q <= 9, front-to-back
 * compositing with alpha capped at 0.99f, skipped below 1/255f and a stop
 * before transmittance falls below 1e-4f, depth order by the camera-space z
 * of the mean stored in single precision with ties by ascending id, and a
 * projected-size threshold cut with sphere-frustum culling.
 *
 * Precision: everything in FP64.  The cut and the depth key are evaluated
 * with +, -, * only, in the order written, built with -ffp-contract=off, so
 * the node set and the depth order are exact results any IEEE FP64
 * implementation reproduces.  Compositing decisions that fall within a
 * relative margin of their threshold are forked: every branch is a valid
 * result, and the output lists them all (branch 0 takes the FP64 decision).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float position[3];
    float R[9];      /* world -> camera, rows: right, down, forward */
    float znear;
    float bg[3];
} or_camera;

/* Single-precision constants of the compositing rule, widened exactly. */
#define OR_ALPHA_CAP ((double)0.99f)
#define OR_ALPHA_MIN ((double)(1.0f / 255.0f))
#define OR_T_MIN ((double)1e-4f)
#define OR_LOWPASS 0.3
#define OR_Q_MAX 9.0

enum { OR_MODE_ALL_LEAVES = 0, OR_MODE_THRESHOLD = 1 };

/* ------------------------------------------------------------------------ */
/* Level-of-detail cut                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double o[3], R[9], fx, fy, cx, cy, W, H, znear, f2, tau2;
    double nl, nr, nt, nb;   /* squared plane-normal lengths */
} cut_cam;

static void cut_cam_init(cut_cam* k, const or_camera* c, float tau) {
    for (int i = 0; i < 3; i++) k->o[i] = (double)c->position[i];
    for (int i = 0; i < 9; i++) k->R[i] = (double)c->R[i];
    k->fx = c->fx; k->fy = c->fy; k->cx = c->cx; k->cy = c->cy;
    k->W = (double)c->width; k->H = (double)c->height; k->znear = c->znear;
    double f = k->fx > k->fy ? k->fx : k->fy;
    k->f2 = 2.0 * f;
    k->tau2 = (double)tau * (double)tau;
    double cxw = k->cx - k->W, cyh = k->cy - k->H;
    k->nl = k->fx * k->fx + k->cx * k->cx;
    k->nr = k->fx * k->fx + cxw * cxw;
    k->nt = k->fy * k->fy + k->cy * k->cy;
    k->nb = k->fy * k->fy + cyh * cyh;
}

/* Is the sphere (c, r) entirely outside the view frustum? */
static int cut_culled(const cut_cam* k, const double d[3], double r) {
    const double* R = k->R;
    double px = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
    double py = (R[3] * d[0] + R[4] * d[1]) + R[5] * d[2];
    double pz = (R[6] * d[0] + R[7] * d[1]) + R[8] * d[2];
    if (pz + r < k->znear) return 1;
    double rr = r * r;
    double eL = k->fx * px + k->cx * pz;
    if (eL < 0.0 && eL * eL > rr * k->nl) return 1;
    double eR = k->fx * px + (k->cx - k->W) * pz;
    if (eR > 0.0 && eR * eR > rr * k->nr) return 1;
    double eT = k->fy * py + k->cy * pz;
    if (eT < 0.0 && eT * eT > rr * k->nt) return 1;
    double eB = k->fy * py + (k->cy - k->H) * pz;
    if (eB > 0.0 && eB * eB > rr * k->nb) return 1;
    return 0;
}

/* Does the projected size 2 f r / |c - o| exceed tau (squared, no division)? */
static int cut_expand(const cut_cam* k, const double d[3], double r) {
    double a = k->f2 * r;
    double lhs = a * a;
    double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double rhs = k->tau2 * d2;
    return lhs > rhs;
}

typedef struct {
    const float* bound; const int32_t* first_child; const int32_t* child_count;
    const cut_cam* cam; int32_t* out; int64_t cap; int64_t count;
} cut_walk;

static void cut_visit(cut_walk* w, int32_t k) {
    const float* b = w->bound + 4 * (int64_t)k;
    double d[3] = {(double)b[0] - w->cam->o[0], (double)b[1] - w->cam->o[1],
                   (double)b[2] - w->cam->o[2]};
    double r = (double)b[3];
    if (cut_culled(w->cam, d, r)) return;
    int32_t nc = w->child_count[k];
    if (nc > 0 && cut_expand(w->cam, d, r)) {
        for (int32_t j = 0; j < nc; j++) cut_visit(w, w->first_child[k] + j);
        return;
    }
    if (w->count < w->cap) w->out[w->count] = k;
    w->count++;
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Node ids of the cut, ascending.  parent == NULL means a flat scene: every
 * Gaussian.  ALL_LEAVES: every leaf, no culling.  THRESHOLD: top-down from
 * the roots; a node whose bounding sphere is outside the frustum drops its
 * subtree; a leaf is emitted; an internal node is emitted unless its
 * projected size exceeds tau, in which case its children are visited.
 * Returns the count (entries beyond cap are not written). */
int64_t or_cut(int64_t n, const float* bound, const int32_t* parent,
               const int32_t* first_child, const int32_t* child_count,
               const or_camera* cam, int32_t mode, float tau, int32_t* out,
               int64_t cap) {
    int64_t cnt = 0;
    if (parent == NULL) {
        for (int64_t i = 0; i < n; i++) { if (cnt < cap) out[cnt] = (int32_t)i; cnt++; }
        return cnt;
    }
    if (mode == OR_MODE_ALL_LEAVES) {
        for (int64_t i = 0; i < n; i++)
            if (child_count[i] == 0) { if (cnt < cap) out[cnt] = (int32_t)i; cnt++; }
        return cnt;
    }
    cut_cam k;
    cut_cam_init(&k, cam, tau);
    cut_walk w = {bound, first_child, child_count, &k, out, cap, 0};
    for (int64_t i = 0; i < n; i++)
        if (parent[i] < 0) cut_visit(&w, (int32_t)i);
    int64_t m = w.count < cap ? w.count : cap;
    qsort(out, (size_t)m, sizeof(int32_t), cmp_i32);
    return w.count;
}

/* ------------------------------------------------------------------------ */
/* Learned level-of-detail cut                                               */
/* ------------------------------------------------------------------------ */

/* The learned refinement of the cut is this project's (the paper selects
 * Gaussians from the tree's levels, Sec. III-B, without a learned rule).
 * Definition: the threshold cut, except that a candidate, an internal node
 * the threshold refines whose projected size is at most s_hi pixels, is
 * refined only when the network's logit z of its 8 standardised features
 * reaches z* = logit(p*).  Features of node k seen from the camera (FP64):
 *   0 log of its projected size 2 f r / |c - o| (size at least 1e-6,
 *     distance at least 1e-9), 1 log of its camera-space depth (at least
 *     znear), 2 its opacity, 3 its child count, 4 the variance of its
 *     children's DC colour (C0^2 times the summed per-channel variance of
 *     the DC coefficients; 0 for fewer than two children), 5 |cos| between
 *     c - o and its thinnest axis (the rotation's column of the least scale,
 *     the first on ties), 6 its level, 7 log of its parent's projected size
 *     (its own for a root).
 * Network: 8 -> 32 -> 32 -> 1, ReLU, parameters W1[32][8], b1, W2[32][32],
 * b2, w3, b3 (the BF16 values, widened).  A candidate whose logit lies
 * within `margin` of z* is reported as undecided; the walk takes z >= z*. */
typedef struct {
    const double* w;
    const double* mean;
    const double* std;
    double z_star, s_hi, margin;
    const float* quats;
    const float* scales;
    const float* opacity;
    const float* sh;
    int K;
    const int32_t* parent;
    const int32_t* level;
} lod_net;

static double lod_logit(const lod_net* net, const cut_cam* k, const float* bound, const int32_t* first_child,
                        const int32_t* child_count, int32_t node) {
    const float* b = bound + 4 * (int64_t)node;
    const double dx = (double)b[0] - k->o[0], dy = (double)b[1] - k->o[1], dz = (double)b[2] - k->o[2];
    const double r = b[3];
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    const double dd = dist > 1e-9 ? dist : 1e-9;
    double f[8];
    const double size = k->f2 * r / dd;
    f[0] = log(size > 1e-6 ? size : 1e-6);
    const double pz = k->R[6] * dx + k->R[7] * dy + k->R[8] * dz;
    f[1] = log(pz > k->znear ? pz : k->znear);
    f[2] = net->opacity[node];
    const int32_t nc = child_count[node];
    f[3] = nc;
    double var = 0.0;
    if (nc > 1) {
        for (int c = 0; c < 3; c++) {
            double s1 = 0.0, s2 = 0.0;
            for (int32_t j = 0; j < nc; j++) {
                const double v = net->sh[((int64_t)(first_child[node] + j) * net->K) * 3 + c];
                s1 += v;
                s2 += v * v;
            }
            const double m = s1 / nc;
            var += s2 / nc - m * m;
        }
        var *= 0.28209479177387814 * 0.28209479177387814;
    }
    f[4] = var > 0.0 ? var : 0.0;
    {
        const float* q = net->quats + 4 * (int64_t)node;
        const float* sc = net->scales + 3 * (int64_t)node;
        const double qn = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
        const double qw = q[0] / qn, qx = q[1] / qn, qy = q[2] / qn, qz = q[3] / qn;
        const double Rq[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                              2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                              2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
        int a = 0;
        if (sc[1] < sc[a]) a = 1;
        if (sc[2] < sc[a]) a = 2;
        f[5] = fabs(dx * Rq[a] + dy * Rq[3 + a] + dz * Rq[6 + a]) / dd;
    }
    f[6] = net->level[node];
    const int32_t p = net->parent[node];
    if (p >= 0) {
        const float* pb = bound + 4 * (int64_t)p;
        const double qx = (double)pb[0] - k->o[0], qy = (double)pb[1] - k->o[1], qz = (double)pb[2] - k->o[2];
        const double pd = sqrt(qx * qx + qy * qy + qz * qz);
        const double ps = k->f2 * (double)pb[3] / (pd > 1e-9 ? pd : 1e-9);
        f[7] = log(ps > 1e-6 ? ps : 1e-6);
    } else {
        f[7] = f[0];
    }
    double x[8], h1[32];
    for (int i = 0; i < 8; i++) x[i] = (f[i] - net->mean[i]) / net->std[i];
    const double* W1 = net->w;
    const double* b1 = W1 + 32 * 8;
    const double* W2 = b1 + 32;
    const double* b2 = W2 + 32 * 32;
    const double* w3 = b2 + 32;
    const double b3 = w3[32];
    for (int j = 0; j < 32; j++) {
        double acc = b1[j];
        for (int i = 0; i < 8; i++) acc += W1[8 * j + i] * x[i];
        h1[j] = acc > 0.0 ? acc : 0.0;
    }
    double z = b3;
    for (int j = 0; j < 32; j++) {
        double acc = b2[j];
        for (int i = 0; i < 32; i++) acc += W2[32 * j + i] * h1[i];
        z += w3[j] * (acc > 0.0 ? acc : 0.0);
    }
    return z;
}

typedef struct {
    cut_walk base;
    const lod_net* net;
    int32_t* amb;
    int64_t amb_cap, amb_count;
    const int32_t* flip;      /* ascending undecided candidates to take the other way */
    int64_t n_flip, bad_flips;
} lcut_walk;

static void lcut_visit(lcut_walk* w, int32_t k) {
    const float* b = w->base.bound + 4 * (int64_t)k;
    const cut_cam* cam = w->base.cam;
    double d[3] = {(double)b[0] - cam->o[0], (double)b[1] - cam->o[1], (double)b[2] - cam->o[2]};
    double r = (double)b[3];
    if (cut_culled(cam, d, r)) return;
    int32_t nc = w->base.child_count[k];
    int expand = nc > 0 && cut_expand(cam, d, r);
    if (expand) {
        const double a = cam->f2 * r;
        const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (a * a <= (w->net->s_hi * w->net->s_hi) * d2) {
            const double z = lod_logit(w->net, cam, w->base.bound, w->base.first_child, w->base.child_count, k);
            if (fabs(z - w->net->z_star) <= w->net->margin) {
                if (w->amb_count < w->amb_cap) w->amb[w->amb_count] = k;
                w->amb_count++;
            }
            const int undecided = fabs(z - w->net->z_star) <= w->net->margin;
            expand = z >= w->net->z_star;
            if (w->n_flip && bsearch(&k, w->flip, (size_t)w->n_flip, sizeof(int32_t), cmp_i32)) {
                if (undecided) expand = !expand;
                else w->bad_flips++;
            }
        }
    }
    if (expand) {
        for (int32_t j = 0; j < nc; j++) lcut_visit(w, w->base.first_child[k] + j);
        return;
    }
    if (w->base.count < w->base.cap) w->base.out[w->base.count] = k;
    w->base.count++;
}

/* Learned cut (see above): node ids ascending in out (count returned),
 * undecided candidates reached ascending in amb (count in *n_amb).  Every
 * node of flip (ascending) that the walk reaches as an undecided candidate
 * takes the other decision, which is as valid; *bad_flips counts flip
 * nodes reached as decided candidates (left as decided). */
int64_t or_cut_learned(int64_t n, const float* bound, const int32_t* parent, const int32_t* first_child,
                       const int32_t* child_count, const int32_t* level, const float* quats, const float* scales,
                       const float* opacity, const float* sh, int32_t sh_degree, const double* w,
                       const double* mean, const double* std, double z_star, double s_hi, double margin,
                       const or_camera* cam, float tau, const int32_t* flip, int64_t n_flip, int32_t* out,
                       int64_t cap, int32_t* amb, int64_t amb_cap, int64_t* n_amb, int64_t* bad_flips) {
    cut_cam k;
    cut_cam_init(&k, cam, tau);
    lod_net net = {w, mean, std, z_star, s_hi, margin, quats, scales, opacity, sh,
                   (sh_degree + 1) * (sh_degree + 1), parent, level};
    lcut_walk lw = {{bound, first_child, child_count, &k, out, cap, 0}, &net, amb, amb_cap, 0, flip, n_flip, 0};
    for (int64_t i = 0; i < n; i++)
        if (parent[i] < 0) lcut_visit(&lw, (int32_t)i);
    int64_t m = lw.base.count < cap ? lw.base.count : cap;
    qsort(out, (size_t)m, sizeof(int32_t), cmp_i32);
    int64_t ma = lw.amb_count < amb_cap ? lw.amb_count : amb_cap;
    qsort(amb, (size_t)ma, sizeof(int32_t), cmp_i32);
    *n_amb = lw.amb_count;
    *bad_flips = lw.bad_flips;
    return lw.base.count;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics (Condon-Shortley phase), l <= 3                 */
/* ------------------------------------------------------------------------ */

static double factorial(int n) { double f = 1; for (int i = 2; i <= n; i++) f *= i; return f; }

/* Associated Legendre P_l^m(x) for 0 <= m <= l, including (-1)^m. */
static double assoc_legendre(int l, int m, double x) {
    double pmm = 1.0, s = sqrt((1.0 - x) * (1.0 + x)), fact = 1.0;
    for (int i = 1; i <= m; i++) { pmm *= -fact * s; fact += 2.0; }
    if (l == m) return pmm;
    double pmmp1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ll++) {
        pll = ((2.0 * ll - 1.0) * x * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmmp1; pmmp1 = pll;
    }
    return pll;
}

/* out[l*l + l + m] = Y_lm(d) for a unit direction d, l = 0..3. */
void or_sh_basis(const double d[3], double out[16]) {
    double ct = d[2];
    double phi = atan2(d[1], d[0]);
    for (int l = 0; l <= 3; l++) {
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, ct);
            double y;
            if (m == 0) y = K * P;
            else if (m > 0) y = sqrt(2.0) * K * P * cos(m * phi);
            else y = sqrt(2.0) * K * P * sin(am * phi);
            out[l * l + l + m] = y;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Projection                                                                */
/* ------------------------------------------------------------------------ */

enum {
    OP_VALID = 0, OP_U, OP_V, OP_A, OP_B, OP_C, OP_S00, OP_S01, OP_S11,
    OP_R, OP_G, OP_BL, OP_Z, OP_ZKEY, OP_OPAC, OP_TX, OP_TY, OP_STRIDE
};

static void matmul3(const double a[9], const double b[9], double c[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

static void transpose3(const double a[9], double t[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * j + i] = a[3 * i + j];
}

/* Camera of the projection (FP64 copies and the Jacobian clamp range). */
typedef struct {
    double Rv[9], o[3], fx, fy, cx, cy, xlo, xhi, ylo, yhi, znear;
} proj_cam;

static void proj_cam_init(proj_cam* k, const or_camera* cam) {
    for (int i = 0; i < 9; i++) k->Rv[i] = cam->R[i];
    for (int i = 0; i < 3; i++) k->o[i] = cam->position[i];
    k->fx = cam->fx; k->fy = cam->fy; k->cx = cam->cx; k->cy = cam->cy;
    /* Jacobian clamp: x/z within the image's tangent range widened by 15 %
     * of the image size on each side (1.3 x the half field of view when the
     * principal point is centred) */
    const double W = cam->width, H = cam->height;
    k->xlo = (-k->cx - 0.15 * W) / k->fx; k->xhi = (W - k->cx + 0.15 * W) / k->fx;
    k->ylo = (-k->cy - 0.15 * H) / k->fy; k->yhi = (H - k->cy + 0.15 * H) / k->fy;
    k->znear = cam->znear;
}

/* Sigma = R S S^T R^T of Gaussian g from its normalised quaternion. */
static void gauss_sigma(const float* scales, const float* quats, int64_t g, double Sig[9]) {
    double qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    double Rq[9] = {
        1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
        2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
        2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double S[9] = {0};
    for (int i = 0; i < 3; i++) S[4 * i] = (double)scales[3 * g + i];
    double RS[9], RSt[9];
    matmul3(Rq, S, RS);
    transpose3(RS, RSt);
    matmul3(RS, RSt, Sig);
}

/* Projection of one Gaussian (mean mu, covariance Sig, opacity op, SH
 * coefficients shc[k*3 + c]) into row r. */
static void project_one(const proj_cam* k, const double mu[3], const double Sig[9], double op, const double* shc,
                        int K, double* r) {
    memset(r, 0, sizeof(double) * OP_STRIDE);
    double d[3] = {mu[0] - k->o[0], mu[1] - k->o[1], mu[2] - k->o[2]};
    /* camera-space mean, each row summed left to right */
    double t[3];
    for (int i = 0; i < 3; i++)
        t[i] = (k->Rv[3 * i] * d[0] + k->Rv[3 * i + 1] * d[1]) + k->Rv[3 * i + 2] * d[2];
    r[OP_Z] = t[2];
    r[OP_ZKEY] = (double)(float)t[2];
    r[OP_TX] = t[0]; r[OP_TY] = t[1];
    r[OP_OPAC] = op;
    if (!(t[2] > k->znear)) return;
    /* Jacobian of the perspective map at the (clamped) mean */
    double tz = t[2];
    double xr = t[0] / tz, yr = t[1] / tz;
    if (xr < k->xlo) xr = k->xlo;
    if (xr > k->xhi) xr = k->xhi;
    if (yr < k->ylo) yr = k->ylo;
    if (yr > k->yhi) yr = k->yhi;
    double xh = xr * tz, yh = yr * tz;
    double J[9] = {k->fx / tz, 0, -k->fx * xh / (tz * tz), 0, k->fy / tz, -k->fy * yh / (tz * tz), 0, 0, 0};
    double JW[9], JWt[9], tmp[9], C2[9];
    matmul3(J, k->Rv, JW);
    transpose3(JW, JWt);
    matmul3(JW, Sig, tmp);
    matmul3(tmp, JWt, C2);
    double s00 = C2[0] + OR_LOWPASS, s01 = C2[1], s11 = C2[4] + OR_LOWPASS;
    double det = s00 * s11 - s01 * s01;
    r[OP_S00] = s00; r[OP_S01] = s01; r[OP_S11] = s11;
    if (!(det > 0.0)) return;
    r[OP_A] = s11 / det; r[OP_B] = -s01 / det; r[OP_C] = s00 / det;
    r[OP_U] = k->fx * t[0] / tz + k->cx;
    r[OP_V] = k->fy * t[1] / tz + k->cy;
    /* colour from spherical harmonics in the world-space view direction */
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dir[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
    double Y[16];
    or_sh_basis(dir, Y);
    for (int c = 0; c < 3; c++) {
        double v = 0.5;
        for (int q = 0; q < K; q++) v += shc[q * 3 + c] * Y[q];
        r[OP_R + c] = v < 0 ? 0 : (v > 1 ? 1 : v);
    }
    r[OP_VALID] = 1.0;
}

/* Project the Gaussians ids[0..m) into the camera; out has OP_STRIDE doubles
 * per entry.  Entries behind the near plane (t_z <= znear) or with a
 * non-positive 2D determinant are marked invalid. */
void or_project(int64_t m, const int32_t* ids, const float* means, const float* scales,
                const float* quats, const float* opacity, const float* sh,
                int32_t sh_degree, const or_camera* cam, double* out) {
    const int K = (sh_degree + 1) * (sh_degree + 1);
    proj_cam k;
    proj_cam_init(&k, cam);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        const int64_t g = ids[e];
        double mu[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
        double Sig[9], shc[48];
        gauss_sigma(scales, quats, g, Sig);
        for (int q = 0; q < 3 * K; q++) shc[q] = (double)sh[g * K * 3 + q];
        project_one(&k, mu, Sig, (double)opacity[g], shc, K, out + OP_STRIDE * e);
    }
}

/* Level-of-detail blending (Sec. III-B: transition regions are smoothly
 * interpolated; the rule is a reading).  A cut node g with parent p is drawn
 * with mean, covariance and SH coefficients p + t (g - p) and opacity
 *   o_p + t (o_g - o_p)  if g is the first of p's children in the cut,
 *   t o_g                otherwise,
 * where, with s_n = 2 f r_n / |c_n - o| the projected size of node n's
 * bounding sphere (f = max(fx, fy)),
 *   t = clamp((s_p - tau) / (s_p - s_g), 0, 1)   (t = 1 when s_g >= s_p).
 * A node's parent is refined only past the threshold (s_p > tau), and a
 * node that is itself refined at s_g > tau gives way to its children, so
 * t runs from 0 when p has just been refined -- the children together are
 * then p itself: the first one carries p, the others are transparent -- to
 * 1 when g is about to be refined in turn, where g is drawn as itself.  The
 * image therefore does not jump when a node is refined.  Roots are not
 * blended.  s_p, s_g and t are evaluated as written, in FP64; cut holds the
 * ascending ids of the whole cut (ids may be a subset of it). */
static double blend_size(const float* bound, int64_t n, const proj_cam* k, double f2) {
    const double dx = (double)bound[4 * n] - k->o[0], dy = (double)bound[4 * n + 1] - k->o[1],
                 dz = (double)bound[4 * n + 2] - k->o[2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    return f2 * (double)bound[4 * n + 3] / sqrt(d2);
}

void or_project_blend(int64_t m, const int32_t* ids, const float* means, const float* scales,
                      const float* quats, const float* opacity, const float* sh, int32_t sh_degree,
                      const int32_t* parent, const int32_t* first_child, const float* bound, int64_t n_cut,
                      const int32_t* cut, float tau, const or_camera* cam, double* out, double* tout) {
    const int K = (sh_degree + 1) * (sh_degree + 1);
    proj_cam k;
    proj_cam_init(&k, cam);
    const double f2 = 2.0 * (cam->fx > cam->fy ? (double)cam->fx : (double)cam->fy);
    const double tauv = tau;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        const int64_t g = ids[e];
        const int64_t p = parent[g];
        double t = 1.0;
        int first = 1;
        if (p >= 0) {
            const double sp = blend_size(bound, p, &k, f2);
            const double sg = blend_size(bound, g, &k, f2);
            if (sg < sp) {
                t = (sp - tauv) / (sp - sg);
                t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            }
            for (int32_t q = first_child[p]; q < g; q++) {
                if (bsearch(&q, cut, (size_t)n_cut, sizeof(int32_t), cmp_i32)) {
                    first = 0;
                    break;
                }
            }
        }
        if (tout) tout[e] = t;
        double mu[3], Sig[9], shc[48], op;
        gauss_sigma(scales, quats, g, Sig);
        for (int i = 0; i < 3; i++) mu[i] = means[3 * g + i];
        op = opacity[g];
        for (int q = 0; q < 3 * K; q++) shc[q] = (double)sh[g * K * 3 + q];
        if (p >= 0) {
            double Sp[9];
            gauss_sigma(scales, quats, p, Sp);
            for (int i = 0; i < 9; i++) Sig[i] = Sp[i] + t * (Sig[i] - Sp[i]);
            for (int i = 0; i < 3; i++) mu[i] = (double)means[3 * p + i] + t * (mu[i] - (double)means[3 * p + i]);
            op = first ? (double)opacity[p] + t * (op - (double)opacity[p]) : t * op;
            for (int q = 0; q < 3 * K; q++) shc[q] = (double)sh[p * K * 3 + q] + t * (shc[q] - (double)sh[p * K * 3 + q]);
        }
        project_one(&k, mu, Sig, op, shc, K, out + OP_STRIDE * e);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing with forks at near-threshold decisions              */
/* ------------------------------------------------------------------------ */

typedef struct { double q, zkey, z, op, col[3]; int64_t idx; } cand;

static int cand_cmp(const void* a, const void* b) {
    const cand* x = (const cand*)a; const cand* y = (const cand*)b;
    if (x->zkey < y->zkey) return -1;
    if (x->zkey > y->zkey) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct {
    const cand* L; int n; double eps_q, eps_a, eps_t; double bg[3];
    int cap; int made; int nalt; double* out; int overflow; int64_t nalg;
} walker;

/* Branch 0 is the path that follows every FP64 decision; the others follow
 * at least one flipped near-threshold decision. */
static void emit_branch(walker* w, int primary, double T, const double C[3], double D) {
    int slot;
    if (primary) slot = 0;
    else { slot = 1 + w->nalt; w->nalt++; }
    if (slot >= w->cap) { w->overflow = 1; return; }
    double* o = w->out + 5 * slot;
    for (int c = 0; c < 3; c++) o[c] = C[c] + T * w->bg[c];
    o[3] = D;
    o[4] = 1.0 - T;
}

enum { OUT_SKIP = 0, OUT_ADD = 1, OUT_STOP = 2 };

/* Composite the sorted list from position i with state (T, C, D).  At each
 * entry the possible outcomes are: skip it (outside q <= 9, or alpha below
 * the minimum), add it, or stop before it (transmittance would fall below
 * the minimum).  The FP64 decisions pick one; any decision within its
 * relative margin also allows the other side, and each extra outcome is
 * walked as a branch of its own while the branch budget lasts. */
static void walk(walker* w, int i, double T, const double Cin[3], double Din, int primary) {
    double C[3] = {Cin[0], Cin[1], Cin[2]}, D = Din;
    for (; i < w->n; i++) {
        const cand* g = &w->L[i];
        int amb_q = fabs(g->q - OR_Q_MAX) <= OR_Q_MAX * w->eps_q;
        int in = g->q <= OR_Q_MAX;
        double a = g->op * exp(-0.5 * g->q);
        if (a > OR_ALPHA_CAP) a = OR_ALPHA_CAP;
        int amb_a = fabs(a - OR_ALPHA_MIN) <= OR_ALPHA_MIN * w->eps_a;
        int use = a >= OR_ALPHA_MIN;
        double Tn = T * (1.0 - a);
        int amb_t = fabs(Tn - OR_T_MIN) <= OR_T_MIN * w->eps_t;
        int stop = Tn < OR_T_MIN;
        int can_in = in || amb_q, can_out = !in || amb_q;
        int can_use = can_in && (use || amb_a), can_skip = can_out || (can_in && (!use || amb_a));
        int can_stop = can_use && (stop || amb_t), can_add = can_use && (!stop || amb_t);
        int prim = !in || !use ? OUT_SKIP : (stop ? OUT_STOP : OUT_ADD);
        if (primary && in) w->nalg++;
        int possible[3] = {can_skip, can_add, can_stop};
        for (int out = 0; out < 3; out++) {
            if (out == prim || !possible[out]) continue;
            if (w->made + 1 > w->cap) { w->overflow = 1; continue; }
            w->made++;
            if (out == OUT_SKIP) {
                walk(w, i + 1, T, C, D, 0);
            } else if (out == OUT_ADD) {
                double Cc[3] = {C[0] + g->col[0] * a * T, C[1] + g->col[1] * a * T,
                                C[2] + g->col[2] * a * T};
                walk(w, i + 1, Tn, Cc, D + g->z * a * T, 0);
            } else {
                emit_branch(w, 0, T, C, D);
            }
        }
        if (prim == OUT_SKIP) continue;
        if (prim == OUT_STOP) { emit_branch(w, primary, T, C, D); return; }
        for (int c = 0; c < 3; c++) C[c] += g->col[c] * a * T;
        D += g->z * a * T;
        T = Tn;
    }
    emit_branch(w, primary, T, C, D);
}

/* Composite the pixels (px[i], py[i]) (pixel centres at +0.5) from the
 * projected entries proj[0..m) (or_project layout).  For each pixel:
 * out[(i*cap + b)*5 + {0,1,2,3,4}] = R, G, B, depth (sum of w z), alpha
 * (1 - T) of branch b; nbranch[i] = number of branches (branch 0 follows
 * every FP64 decision); nalg[i] = entries with q <= 9 evaluated on branch 0
 * up to and including the one that stops it; flags[i] bit 0 = some
 * ambiguous decision could not be forked (branch cap).  eps = relative
 * margins for q vs 9, alpha vs 1/255f, T vs 1e-4f. */
int32_t or_render_pixels(int64_t m, const double* proj, const or_camera* cam, int64_t npix,
                         const int32_t* px, const int32_t* py, const double* eps,
                         int32_t cap, double* out, int32_t* nbranch, int64_t* nalg,
                         int32_t* flags) {
    const int H = cam->height;
    const double eq = eps[0];
    /* Row buckets: the rows whose pixel centres lie within the (slightly
     * enlarged) vertical extent of each ellipse q <= 9(1+eps). */
    int64_t* rc = (int64_t*)calloc((size_t)H + 1, sizeof(int64_t));
    int* need = (int*)calloc((size_t)H, sizeof(int));
    if (!rc || !need) { free(rc); free(need); return -1; }
    for (int64_t i = 0; i < npix; i++) if (py[i] >= 0 && py[i] < H) need[py[i]] = 1;
    int32_t* y0s = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* y1s = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    double* exs = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!y0s || !y1s || !exs) { free(rc); free(need); free(y0s); free(y1s); free(exs); return -1; }
    for (int64_t e = 0; e < m; e++) {
        const double* r = proj + OP_STRIDE * e;
        y0s[e] = 1; y1s[e] = 0; exs[e] = 0;
        if (r[OP_VALID] == 0.0) continue;
        double ey = sqrt(OR_Q_MAX * (1.0 + eq) * r[OP_S11]) + 0.01;
        double ex = sqrt(OR_Q_MAX * (1.0 + eq) * r[OP_S00]) + 0.01;
        double lo = ceil(r[OP_V] - ey - 0.5), hi = floor(r[OP_V] + ey - 0.5);
        if (lo < 0) lo = 0;
        if (hi > H - 1) hi = H - 1;
        if (hi < lo) continue;
        y0s[e] = (int32_t)lo; y1s[e] = (int32_t)hi; exs[e] = ex;
        for (int y = (int)lo; y <= (int)hi; y++) if (need[y]) rc[y + 1]++;
    }
    for (int y = 0; y < H; y++) rc[y + 1] += rc[y];
    int64_t total = rc[H];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)H);
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    if (!fill || !rows) { free(rc); free(need); free(y0s); free(y1s); free(exs); free(fill); free(rows); return -1; }
    memcpy(fill, rc, sizeof(int64_t) * (size_t)H);
    for (int64_t e = 0; e < m; e++)
        for (int y = y0s[e]; y <= y1s[e]; y++) if (need[y]) rows[fill[y]++] = e;
    double bg[3] = {cam->bg[0], cam->bg[1], cam->bg[2]};
    int err = 0;
#pragma omp parallel
    {
        int64_t lcap = 1024;
        cand* L = (cand*)malloc(sizeof(cand) * (size_t)lcap);
        if (!L) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < npix; i++) {
            if (!L) continue;
            double* o = out + (int64_t)5 * cap * i;
            for (int64_t k = 0; k < (int64_t)5 * cap; k++) o[k] = 0;
            nbranch[i] = 0; nalg[i] = 0; flags[i] = 0;
            if (py[i] < 0 || py[i] >= H || px[i] < 0 || px[i] >= cam->width) continue;
            double x = px[i] + 0.5, y = py[i] + 0.5;
            int n = 0;
            for (int64_t k = rc[py[i]]; k < rc[py[i] + 1]; k++) {
                int64_t e = rows[k];
                const double* r = proj + OP_STRIDE * e;
                double dx = x - r[OP_U];
                if (fabs(dx) > exs[e]) continue;
                double dy = y - r[OP_V];
                double q = r[OP_A] * dx * dx + 2.0 * r[OP_B] * dx * dy + r[OP_C] * dy * dy;
                if (q > OR_Q_MAX * (1.0 + eq)) continue;
                if (n == lcap) {
                    lcap *= 2;
                    cand* nl = (cand*)realloc(L, sizeof(cand) * (size_t)lcap);
                    if (!nl) { free(L); L = NULL; break; }
                    L = nl;
                }
                cand* c = &L[n++];
                c->q = q; c->zkey = r[OP_ZKEY]; c->z = r[OP_Z]; c->op = r[OP_OPAC];
                c->col[0] = r[OP_R]; c->col[1] = r[OP_G]; c->col[2] = r[OP_BL]; c->idx = e;
            }
            if (!L) {
#pragma omp atomic write
                err = 1;
                continue;
            }
            qsort(L, (size_t)n, sizeof(cand), cand_cmp);
            walker w = {L, n, eps[0], eps[1], eps[2], {bg[0], bg[1], bg[2]},
                        cap, 1, 0, o, 0, 0};
            double C0[3] = {0, 0, 0};
            walk(&w, 0, 1.0, C0, 0.0, 1);
            nbranch[i] = 1 + w.nalt < cap ? 1 + w.nalt : cap;
            nalg[i] = w.nalg;
            flags[i] = w.overflow;
        }
        free(L);
    }
    free(rc); free(need); free(y0s); free(y1s); free(exs); free(fill); free(rows);
    return err ? -1 : 0;
}

int32_t or_proj_stride(void) { return OP_STRIDE; }

int32_t or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
