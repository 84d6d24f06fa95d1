/*
 * FP64 CPU oracle of shortest-path planning on the navigable grid.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): the test-suite may load it, the
 * planner on the GPU never does, and the two share no code.
 *
 * What it follows (NavGSim, arXiv 2603.15186): the slice map turns the scene
 * into navigable areas for collision checking and path planning (Sec. I,
 * Sec. III), and expert trajectories come from a shortest-path planner from
 * random start positions to annotated goals (Sec. IV, data collection).  The
 * paper names no planner; the reading implemented:
 *   - a cell is navigable when a disc robot centred on it is collision free
 *     (or_navigable: the disc test of or_disc_collision at cell centres);
 *   - moves go to the 8 neighbours, costing 1 (orthogonal) or sqrt 2
 *     (diagonal); a diagonal move needs both cells it passes between to be
 *     navigable (no corner cutting);
 *   - the distance of a cell is the least cost of a path to the goal; it is
 *     reported as the pair (a, b) = (orthogonal, diagonal) moves of such a
 *     path, which is unique because sqrt 2 is irrational;
 *   - a trajectory steps from the start to the first neighbour, in the order
 *     E, W, S, N, SE, SW, NE, NW (x right, y down the rows), that lies on a
 *     shortest path: its pair plus the move's unit equals the current pair.
 *
 * The distance field is Dijkstra's algorithm with a binary heap on FP64
 * keys a + b sqrt 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
static const int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};

static int move_ok(const uint8_t* nav, int nx, int ny, int i, int j, int k) {
    const int u = i + DX[k], v = j + DY[k];
    if (u < 0 || v < 0 || u >= nx || v >= ny) return 0;
    if (!nav[(size_t)v * nx + u]) return 0;
    if (k >= 4 && (!nav[(size_t)j * nx + u] || !nav[(size_t)v * nx + i])) return 0;
    return 1;
}

/* nav[j][i] = 1 when a disc of radius rad centred on cell (i, j)'s centre
 * (x0 + (i + 1/2) cell, y0 + (j + 1/2) cell) meets no occupied cell's closed
 * square, 0 when it meets one, 2 when the nearest occupied square is within
 * a relative margin amb of rad.  Only the cells of the disc's bounding box
 * can meet it; cells outside the grid are free. */
void or_navigable(const uint8_t* map, double x0, double y0, double cell, int32_t nx, int32_t ny, double rad,
                  double amb, int8_t* nav) {
    const int w = (int)ceil(rad * (1.0 + amb) / cell) + 1;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; j++)
        for (int32_t i = 0; i < nx; i++) {
            const double x = x0 + ((double)i + 0.5) * cell, y = y0 + ((double)j + 0.5) * cell;
            double best = INFINITY;
            for (int v = j - w; v <= j + w; v++)
                for (int u = i - w; u <= i + w; u++) {
                    if (u < 0 || v < 0 || u >= nx || v >= ny || !map[(size_t)v * nx + u]) continue;
                    const double ax = x0 + (double)u * cell, ay = y0 + (double)v * cell;
                    const double dx = fmax(fmax(ax - x, 0.0), x - (ax + cell));
                    const double dy = fmax(fmax(ay - y, 0.0), y - (ay + cell));
                    const double d = sqrt(dx * dx + dy * dy);
                    if (d < best) best = d;
                }
            nav[(size_t)j * nx + i] = best <= rad * (1.0 - amb) ? 0 : (best <= rad * (1.0 + amb) ? 2 : 1);
        }
}

typedef struct {
    double key;
    int64_t cell;
} heap_item;

static void heap_push(heap_item* h, int64_t* n, heap_item x) {
    int64_t k = (*n)++;
    while (k > 0) {
        const int64_t p = (k - 1) / 2;
        if (h[p].key <= x.key) break;
        h[k] = h[p];
        k = p;
    }
    h[k] = x;
}

static heap_item heap_pop(heap_item* h, int64_t* n) {
    heap_item top = h[0], last = h[--(*n)];
    int64_t k = 0;
    for (;;) {
        int64_t c = 2 * k + 1;
        if (c >= *n) break;
        if (c + 1 < *n && h[c + 1].key < h[c].key) c++;
        if (h[c].key >= last.key) break;
        h[k] = h[c];
        k = c;
    }
    if (*n > 0) h[k] = last;
    return top;
}

/* dist[g][cell] = (a, b) as two int64 (a = -1: unreachable); goals[g] is a
 * cell index j*nx + i (outside the grid or on a blocked cell: nothing is
 * reachable). */
void or_distance_fields(const uint8_t* nav, int32_t nx, int32_t ny, int32_t n_goals, const int64_t* goals,
                        int64_t* dist) {
    const int64_t N = (int64_t)nx * ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t g = 0; g < n_goals; g++) {
        int64_t* D = dist + (size_t)g * N * 2;
        for (int64_t c = 0; c < N; c++) D[2 * c] = D[2 * c + 1] = -1;
        const int64_t s = goals[g];
        if (s < 0 || s >= N || !nav[s]) continue;
        double* key = (double*)malloc(sizeof(double) * (size_t)N);
        heap_item* h = (heap_item*)malloc(sizeof(heap_item) * (size_t)(8 * N + 1));
        for (int64_t c = 0; c < N; c++) key[c] = INFINITY;
        int64_t hn = 0;
        key[s] = 0.0;
        D[2 * s] = D[2 * s + 1] = 0;
        heap_item it = {0.0, s};
        heap_push(h, &hn, it);
        while (hn > 0) {
            const heap_item top = heap_pop(h, &hn);
            const int64_t c = top.cell;
            if (top.key > key[c]) continue;             /* stale entry */
            const int i = (int)(c % nx), j = (int)(c / nx);
            for (int k = 0; k < 8; k++) {
                if (!move_ok(nav, nx, ny, i, j, k)) continue;
                const int64_t n = (int64_t)(j + DY[k]) * nx + (i + DX[k]);
                const int64_t a = D[2 * c] + (k < 4 ? 1 : 0), b = D[2 * c + 1] + (k < 4 ? 0 : 1);
                const double kk = (double)a + (double)b * sqrt(2.0);
                if (kk < key[n]) {
                    key[n] = kk;
                    D[2 * n] = a;
                    D[2 * n + 1] = b;
                    heap_item e = {kk, n};
                    heap_push(h, &hn, e);
                }
            }
        }
        free(key);
        free(h);
    }
}

/* Trajectory of query q from cell starts[q] down field fields[slot[q]]:
 * len[q] = number of cells from start to goal inclusive (0 when the start
 * is unreachable or off the grid); the first min(len, cap) cells go to
 * path[q*cap ...]. */
void or_trace_paths(const uint8_t* nav, int32_t nx, int32_t ny, const int64_t* dist, int64_t n_q,
                    const int64_t* starts, const int32_t* slot, int32_t cap, int64_t* path, int64_t* len) {
    const int64_t N = (int64_t)nx * ny;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_q; q++) {
        const int64_t* D = dist + (size_t)slot[q] * N * 2;
        int64_t c = starts[q];
        len[q] = 0;
        if (c < 0 || c >= N || D[2 * c] < 0) continue;
        int64_t m = 0;
        for (;;) {
            if (m < cap) path[q * cap + m] = c;
            m++;
            if (D[2 * c] == 0 && D[2 * c + 1] == 0) break;
            const int i = (int)(c % nx), j = (int)(c / nx);
            int64_t next = -1;
            for (int k = 0; k < 8 && next < 0; k++) {
                if (!move_ok(nav, nx, ny, i, j, k)) continue;
                const int64_t n = (int64_t)(j + DY[k]) * nx + (i + DX[k]);
                if (D[2 * n] < 0) continue;
                if (D[2 * n] + (k < 4 ? 1 : 0) == D[2 * c] && D[2 * n + 1] + (k < 4 ? 0 : 1) == D[2 * c + 1]) next = n;
            }
            if (next < 0) { m = -1; break; }            /* not a shortest-path field */
            c = next;
        }
        len[q] = m;
    }
}
