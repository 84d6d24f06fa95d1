// Disc-against-grid test shared by the collision queries and the navigable
// map: cell (i, j) of the map is the closed square [x0 + i cell, x0 + (i+1)
// cell] x [y0 + j cell, y0 + (j+1) cell]; cells outside the grid are free.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hgs {

// True when the closed disc of radius r centred on (x, y) meets an occupied
// (nonzero) cell of map[ny][nx]: the cells of the disc's bounding box, the
// squared distance from the centre to each occupied square against r^2.
__device__ __forceinline__ bool disc_hits(const uint8_t* __restrict__ map, double x0, double y0, double cell, int nx,
                                          int ny, double x, double y, double r) {
    const double r2 = r * r;
    const double fi0 = floor((x - r - x0) / cell), fi1 = floor((x + r - x0) / cell);
    const double fj0 = floor((y - r - y0) / cell), fj1 = floor((y + r - y0) / cell);
    if (!(fi1 >= 0.0 && fi0 <= (double)(nx - 1) && fj1 >= 0.0 && fj0 <= (double)(ny - 1))) return false;
    const int i0 = (int)fmax(fi0, 0.0), i1 = (int)fmin(fi1, (double)(nx - 1));
    const int j0 = (int)fmax(fj0, 0.0), j1 = (int)fmin(fj1, (double)(ny - 1));
    for (int j = j0; j <= j1; ++j) {
        const double ay = y0 + (double)j * cell;
        const double dy = fmax(fmax(ay - y, 0.0), y - (ay + cell));
        for (int i = i0; i <= i1; ++i) {
            if (!map[(size_t)j * nx + i]) continue;
            const double ax = x0 + (double)i * cell;
            const double dx = fmax(fmax(ax - x, 0.0), x - (ax + cell));
            if (dx * dx + dy * dy <= r2) return true;
        }
    }
    return false;
}

}  // namespace hgs
