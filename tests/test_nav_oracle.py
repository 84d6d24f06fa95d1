"""Pins of the planning oracle (CPU): navigable cells against the brute-force
disc test and a closed form, distance fields against closed forms, scipy's
Dijkstra and an exact brute-force relaxation, trajectories against the
shortest-path property."""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra

from oracle import oracle as O

SQ2 = math.sqrt(2.0)
MOVES = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1)]


def _edges(nav):
    """Directed edges (from, to, weight) of the 8-connected grid without
    corner cutting, built with array operations."""
    ny, nx = nav.shape
    jj, ii = np.mgrid[0:ny, 0:nx]
    src, dst, w = [], [], []
    for dx, dy in MOVES:
        u, v = ii + dx, jj + dy
        inside = (u >= 0) & (u < nx) & (v >= 0) & (v < ny)
        uc, vc = np.clip(u, 0, nx - 1), np.clip(v, 0, ny - 1)
        ok = inside & (nav > 0) & (nav[vc, uc] > 0)
        if dx and dy:
            ok &= (nav[jj, uc] > 0) & (nav[vc, ii] > 0)
        src.append((jj * nx + ii)[ok]); dst.append((vc * nx + uc)[ok])
        w.append(np.full(int(ok.sum()), SQ2 if dx and dy else 1.0))
    return np.concatenate(src), np.concatenate(dst), np.concatenate(w)


def _random_nav(rng, ny, nx, p):
    return (rng.uniform(size=(ny, nx)) >= p).astype(np.uint8)


def test_empty_grid_is_the_octile_distance():
    nav = np.ones((23, 31), np.uint8)
    goals = [0, 23 * 31 - 1, 11 * 31 + 17]
    d = O.distance_fields(nav, goals)
    jj, ii = np.mgrid[0:23, 0:31]
    for k, g in enumerate(goals):
        dx, dy = np.abs(ii - g % 31), np.abs(jj - g // 31)
        np.testing.assert_array_equal(d[k, :, :, 0], np.maximum(dx, dy) - np.minimum(dx, dy))
        np.testing.assert_array_equal(d[k, :, :, 1], np.minimum(dx, dy))


@pytest.mark.parametrize("seed,p", [(0, 0.2), (1, 0.35), (2, 0.45)])
def test_distances_equal_scipy_dijkstra(seed, p):
    rng = np.random.default_rng(seed)
    nav = _random_nav(rng, 41, 57, p)
    free = np.flatnonzero(nav)
    goals = rng.choice(free, size=4, replace=False)
    d = O.distance_fields(nav, goals)
    s, t, w = _edges(nav)
    G = coo_matrix((w, (s, t)), shape=(nav.size, nav.size)).tocsr()
    ref = dijkstra(G, directed=True, indices=goals)             # from the goal; the graph is symmetric
    for k in range(len(goals)):
        a, b = d[k, :, :, 0].ravel(), d[k, :, :, 1].ravel()
        reach = a >= 0
        np.testing.assert_array_equal(reach, np.isfinite(ref[k]))
        np.testing.assert_allclose(a[reach] + SQ2 * b[reach], ref[k][reach], rtol=0, atol=1e-9)


def _less(p, q):
    """a1 + b1 sqrt 2 < a2 + b2 sqrt 2, decided in integers."""
    da, db = p[0] - q[0], q[1] - p[1]
    if da < 0 <= db:
        return True
    if da >= 0 >= db:
        return False
    if da < 0:                                   # both negative
        return da * da > 2 * db * db
    return da * da < 2 * db * db                 # both positive


def test_distances_equal_exact_relaxation_on_tiny_grids():
    """Bellman-Ford on (orthogonal, diagonal) pairs with comparisons made in
    integers: the pairs must match exactly."""
    rng = np.random.default_rng(5)
    for trial in range(12):
        ny, nx = rng.integers(3, 8, size=2)
        nav = _random_nav(rng, ny, nx, 0.3)
        free = np.flatnonzero(nav)
        if free.size == 0:
            continue
        g = int(rng.choice(free))
        INF = None
        D = [INF] * nav.size
        D[g] = (0, 0)
        changed = True
        while changed:
            changed = False
            for c in range(nav.size):
                if not nav.flat[c]:
                    continue
                i, j = c % nx, c // nx
                for dx, dy in MOVES:
                    u, v = i + dx, j + dy
                    if not (0 <= u < nx and 0 <= v < ny) or not nav[v, u]:
                        continue
                    if dx and dy and not (nav[j, u] and nav[v, i]):
                        continue
                    n = D[v * nx + u]
                    if n is None:
                        continue
                    cand = (n[0] + (0 if dx and dy else 1), n[1] + (1 if dx and dy else 0))
                    if D[c] is None or _less(cand, D[c]):
                        D[c] = cand
                        changed = True
        d = O.distance_fields(nav, [g])[0].reshape(-1, 2)
        want = np.array([(-1, -1) if x is None else x for x in D])
        np.testing.assert_array_equal(d, want, err_msg=f"trial {trial}")


def test_no_corner_cutting_and_unreachable_regions():
    nav = np.array([[1, 0],
                    [1, 1]], np.uint8)
    d = O.distance_fields(nav, [0])[0]
    assert tuple(d[1, 1]) == (2, 0)              # around the corner, not through it
    assert tuple(d[0, 1]) == (-1, -1)            # blocked cell
    nav2 = np.ones((2, 2), np.uint8)
    assert tuple(O.distance_fields(nav2, [0])[0][1, 1]) == (0, 1)
    # an enclosed pocket is unreachable; a blocked or off-grid goal reaches nothing
    nav3 = np.ones((7, 7), np.uint8)
    nav3[2:5, 2:5] = 0
    nav3[3, 3] = 1
    d3 = O.distance_fields(nav3, [0, 3 * 7 + 3, 2 * 7 + 2, -1, 49])
    assert tuple(d3[0, 3, 3]) == (-1, -1)
    assert (d3[1] >= 0).sum() == 2 and tuple(d3[1, 3, 3]) == (0, 0)
    assert (d3[2:] < 0).all()


def test_wall_with_a_door():
    """A wall across a 9 x 11 room with a one-cell door: the distance from a
    cell behind the wall is the octile distance through the door."""
    nav = np.ones((9, 11), np.uint8)
    nav[:, 5] = 0
    nav[4, 5] = 1
    d = O.distance_fields(nav, [0 * 11 + 0])[0]
    # from (10, 0): to the door (5, 4) then to (0, 0); the door is entered
    # and left orthogonally (its side cells are walls)
    def octile(dx, dy):
        return (max(dx, dy) - min(dx, dy), min(dx, dy))
    a1, b1 = octile(4, 4)                        # (0,0) -> (4,4)
    a2, b2 = octile(4, 4)                        # (6,4) -> (10,0)
    assert tuple(d[0, 10]) == (a1 + 2 + a2, b1 + b2)


@pytest.mark.parametrize("seed", [3, 4])
def test_trajectories_follow_shortest_paths(seed):
    rng = np.random.default_rng(seed)
    nav = _random_nav(rng, 48, 64, 0.3)
    free = np.flatnonzero(nav)
    goals = rng.choice(free, size=3, replace=False)
    d = O.distance_fields(nav, goals)
    starts = rng.choice(free, size=200)
    slots = rng.integers(0, 3, size=200).astype(np.int32)
    cap = 512
    paths, lens = O.trace_paths(nav, d, starts, slots, cap)
    nx = nav.shape[1]
    n_ok = 0
    for q in range(200):
        a, b = d[slots[q]].reshape(-1, 2)[starts[q]]
        if a < 0:
            assert lens[q] == 0
            continue
        n_ok += 1
        assert lens[q] == a + b + 1
        p = paths[q, :lens[q]]
        assert p[0] == starts[q] and p[-1] == goals[slots[q]]
        na = nb = 0
        for c0, c1 in zip(p[:-1], p[1:]):
            dx, dy = c1 % nx - c0 % nx, c1 // nx - c0 // nx
            assert (dx, dy) in MOVES
            assert nav.flat[c1]
            if dx and dy:
                assert nav.flat[c0 // nx * nx + c1 % nx] and nav.flat[c1 // nx * nx + c0 % nx]
                nb += 1
            else:
                na += 1
        assert (na, nb) == (a, b)
    assert n_ok > 100
    # a short cap keeps the head of the path and the full length
    p8, l8 = O.trace_paths(nav, d, starts, slots, 8)
    np.testing.assert_array_equal(l8, lens)
    k = lens >= 8
    np.testing.assert_array_equal(p8[k], paths[k, :8])


def test_navigable_matches_brute_force_disc_test():
    """Cell-centre disc tests against the brute force over every cell, and
    the closed form for one occupied cell."""
    rng = np.random.default_rng(8)
    m = (rng.uniform(size=(37, 45)) < 0.02).astype(np.uint8)
    for r in (0.0, 0.07, 0.25):
        nav = O.navigable(m, -0.3, 0.2, 0.05, r)
        jj, ii = np.mgrid[0:37, 0:45]
        xy = np.stack([-0.3 + (ii.ravel() + 0.5) * 0.05, 0.2 + (jj.ravel() + 0.5) * 0.05], 1)
        coll = O.disc_collision(m, -0.3, 0.2, 0.05, xy, r).reshape(37, 45)
        want = np.where(coll == 2, 2, 1 - coll)
        np.testing.assert_array_equal(nav, want)
    one = np.zeros((21, 21), np.uint8)
    one[10, 10] = 1
    nav = O.navigable(one, 0.0, 0.0, 1.0, 2.2)
    jj, ii = np.mgrid[0:21, 0:21]
    dx = np.maximum(np.abs(ii + 0.5 - 10.5) - 0.5, 0)
    dy = np.maximum(np.abs(jj + 0.5 - 10.5) - 0.5, 0)
    np.testing.assert_array_equal(nav, (np.hypot(dx, dy) > 2.2).astype(np.int8))
