"""Seeded synthetic scenes: the flat random box and the floor-plan buildings.

The paper's scenes are LiDAR-RGB scans of an office floor (NavGSim, Sec. IV-A:
about 700 m^2), which are not available; these generators stand in for them
with the shapes the renderer is exercised on: planar Gaussian sheets for
walls, floors and ceilings (5 mm thin axis) plus box and cylinder clutter,
spherical-harmonic colour up to degree 3 (Sec. III-B describes the scene as
anisotropic 3D Gaussians with Sigma = R S S^T R^T, Supplementary Material).

This module only draws inputs.  It holds none of the renderer's arithmetic
(no projection, no compositing); scenes are plain numpy arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# DC basis value of real spherical harmonics, 1 / (2 sqrt(pi)); used only to
# turn a wanted base colour into a degree-0 coefficient when drawing inputs.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    """A set of 3D Gaussians, optionally organised as a hierarchy.

    means  (n,3) f32 metres; scales (n,3) f32 metres (>0);
    quats  (n,4) f32 (w,x,y,z), not necessarily normalised;
    opacity (n,) f32 in (0,1]; sh (n,K,3) f32, K=(deg+1)^2, coefficient-major.
    Hierarchy (None for a flat scene): node k is Gaussian k, level-major,
    roots first, children of a node contiguous.
    """

    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int
    parent: np.ndarray | None = None
    first_child: np.ndarray | None = None
    child_count: np.ndarray | None = None
    bound: np.ndarray | None = None
    level_offset: np.ndarray | None = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_levels(self) -> int:
        return 0 if self.level_offset is None else len(self.level_offset) - 1

    @property
    def is_hierarchical(self) -> bool:
        return self.parent is not None

    def leaf_ids(self) -> np.ndarray:
        if not self.is_hierarchical:
            return np.arange(self.n, dtype=np.int32)
        return np.nonzero(self.child_count == 0)[0].astype(np.int32)

    def leaves_only(self) -> "Scene":
        """The flat scene made of the hierarchy's leaves."""
        ids = self.leaf_ids()
        return Scene(self.means[ids].copy(), self.scales[ids].copy(),
                     self.quats[ids].copy(), self.opacity[ids].copy(),
                     self.sh[ids].copy(), self.sh_degree, meta=dict(self.meta))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def make_random_box(n: int = 20000, seed: int = 0,
                    box=(4.0, 4.0, 3.0)) -> Scene:
    """Flat random scene: means uniform in a box, log-scales N(-3.5, 0.5),
    uniformly random unit quaternions, opacity sigmoid(N(0,1)), degree-0 SH
    whose colour is uniform in [0,1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box)
    scales = np.exp(rng.normal(-3.5, 0.5, size=(n, 3)))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = _sigmoid(rng.normal(size=n))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = ((rgb - 0.5) / _Y00)[:, None, :]
    return Scene(means.astype(np.float32), scales.astype(np.float32),
                 q.astype(np.float32), opacity.astype(np.float32),
                 sh.astype(np.float32), 0, meta={"kind": "random_box",
                                                  "seed": seed, "box": box})


# ---------------------------------------------------------------------------
# Floor plans
# ---------------------------------------------------------------------------

def _split_rooms(rng, x0, y0, x1, y1, rooms, walls, amin=12.0, amax=40.0):
    w, h = x1 - x0, y1 - y0
    if w * h <= amax:
        rooms.append((x0, y0, x1, y1))
        return
    if w >= h:
        lo, hi = max(0.3 * w, amin / h), min(0.7 * w, w - amin / h)
        s = x0 + rng.uniform(lo, hi) if hi > lo else x0 + 0.5 * w
        walls.append(((s, y0), (s, y1)))
        _split_rooms(rng, x0, y0, s, y1, rooms, walls, amin, amax)
        _split_rooms(rng, s, y0, x1, y1, rooms, walls, amin, amax)
    else:
        lo, hi = max(0.3 * h, amin / w), min(0.7 * h, h - amin / w)
        s = y0 + rng.uniform(lo, hi) if hi > lo else y0 + 0.5 * h
        walls.append(((x0, s), (x1, s)))
        _split_rooms(rng, x0, y0, x1, s, rooms, walls, amin, amax)
        _split_rooms(rng, x0, s, x1, y1, rooms, walls, amin, amax)


class _Surfaces:
    """Rectangles o + u a + v b (u,v in [0,1]) plus cylinder sides and disks."""

    def __init__(self):
        self.rects = []   # (o, a, b, colour, pattern)
        self.cyls = []    # (centre xy, z0, r, h, colour)
        self.disks = []   # (centre xyz, r, colour)

    def add_rect(self, o, a, b, colour, pattern=0):
        self.rects.append((np.asarray(o, float), np.asarray(a, float),
                           np.asarray(b, float), np.asarray(colour, float),
                           pattern))

    def areas(self):
        ar = [np.linalg.norm(a) * np.linalg.norm(b) for _, a, b, _, _ in self.rects]
        ac = [2 * math.pi * r * h for _, _, r, h, _ in self.cyls]
        ad = [math.pi * r * r for _, r, _ in self.disks]
        return np.asarray(ar + ac + ad, float)


def _r2(n, rng):
    """Randomly shifted R2 low-discrepancy points in [0,1)^2."""
    g = 1.32471795724474602596
    a = np.array([1.0 / g, 1.0 / (g * g)])
    i = np.arange(1, n + 1, dtype=float)[:, None]
    return np.mod(rng.uniform(size=2)[None, :] + i * a[None, :], 1.0)


def _rotmat_to_quat(R):
    """Rotation matrices (n,3,3) with det +1 -> quaternions (n,4) (w,x,y,z)."""
    n = R.shape[0]
    q = np.empty((n, 4))
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    # Pick the numerically largest of 4w^2, 4x^2, 4y^2, 4z^2 per matrix.
    cand = np.stack([1 + tr, 1 + 2 * R[:, 0, 0] - tr, 1 + 2 * R[:, 1, 1] - tr,
                     1 + 2 * R[:, 2, 2] - tr], axis=1)
    k = np.argmax(cand, axis=1)
    s = np.sqrt(np.maximum(cand[np.arange(n), k], 1e-300))  # = 2|component|
    for j in range(4):
        m = k == j
        if not m.any():
            continue
        Rm, sm = R[m], s[m]
        if j == 0:
            w = 0.5 * sm
            x = (Rm[:, 2, 1] - Rm[:, 1, 2]) / (2 * sm)
            y = (Rm[:, 0, 2] - Rm[:, 2, 0]) / (2 * sm)
            z = (Rm[:, 1, 0] - Rm[:, 0, 1]) / (2 * sm)
        elif j == 1:
            x = 0.5 * sm
            w = (Rm[:, 2, 1] - Rm[:, 1, 2]) / (2 * sm)
            y = (Rm[:, 0, 1] + Rm[:, 1, 0]) / (2 * sm)
            z = (Rm[:, 0, 2] + Rm[:, 2, 0]) / (2 * sm)
        elif j == 2:
            y = 0.5 * sm
            w = (Rm[:, 0, 2] - Rm[:, 2, 0]) / (2 * sm)
            x = (Rm[:, 0, 1] + Rm[:, 1, 0]) / (2 * sm)
            z = (Rm[:, 1, 2] + Rm[:, 2, 1]) / (2 * sm)
        else:
            z = 0.5 * sm
            w = (Rm[:, 1, 0] - Rm[:, 0, 1]) / (2 * sm)
            x = (Rm[:, 0, 2] + Rm[:, 2, 0]) / (2 * sm)
            y = (Rm[:, 1, 2] + Rm[:, 2, 1]) / (2 * sm)
        q[m] = np.stack([w, x, y, z], axis=1)
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return q


def _pastel(rng):
    return 0.35 + 0.55 * rng.uniform(size=3)


@dataclasses.dataclass
class FloorPlan:
    """Geometry of a generated building (free-space queries, ground truth)."""

    extent: tuple
    n_floors: int
    ceiling: float
    rooms: list          # per floor: list of (x0,y0,x1,y1)
    walls: list          # per floor: list of ((x0,y0),(x1,y1), door_t or None)
    obstacles: list      # per floor: list of ("box", cx, cy, ex, ey, yaw) / ("cyl", cx, cy, r)
    surfaces: np.ndarray | None = None   # SURFACE_DTYPE records the leaves were drawn from


# Record layout of one exact surface (matches the renderer's hgs_surface).
SURFACE_DTYPE = np.dtype([("kind", "<i4"), ("pattern", "<i4"), ("o", "<f4", 3), ("a", "<f4", 3),
                          ("b", "<f4", 3), ("col", "<f4", 3), ("r", "<f4"), ("h", "<f4")])


def surfaces_array(S) -> np.ndarray:
    """The generator's surfaces as SURFACE_DTYPE records."""
    out = np.zeros(len(S.rects) + len(S.cyls) + len(S.disks), SURFACE_DTYPE)
    i = 0
    for (o, a, b, c, pat) in S.rects:
        out[i] = (0, pat, o, a, b, np.clip(c, -10, 10), 0.0, 0.0)
        i += 1
    for (cxy, z0, r, h, c) in S.cyls:
        out[i] = (1, 0, (cxy[0], cxy[1], z0), (0, 0, 0), (0, 0, 0), c, r, h)
        i += 1
    for (cc, r, c) in S.disks:
        out[i] = (2, 0, cc, (0, 0, 0), (0, 0, 0), c, r, 0.0)
        i += 1
    return out


def _make_plan(rng, extent, n_floors, ceiling, n_clutter):
    W, H = extent
    rooms_all, walls_all, obst_all = [], [], []
    for _ in range(n_floors):
        rooms, inner = [], []
        _split_rooms(rng, 0.0, 0.0, W, H, rooms, inner)
        walls = []
        for (p, q) in inner:
            length = math.hypot(q[0] - p[0], q[1] - p[1])
            t = rng.uniform(0.3, max(0.31, length - 1.2))
            walls.append((p, q, t))
        for (p, q) in [((0, 0), (W, 0)), ((W, 0), (W, H)), ((W, H), (0, H)),
                       ((0, H), (0, 0))]:
            walls.append((p, q, None))
        obst = []
        per_floor = n_clutter // n_floors
        doors = []
        for (p, q, t) in walls:
            if t is None:
                continue
            L = math.hypot(q[0] - p[0], q[1] - p[1])
            ux, uy = (q[0] - p[0]) / L, (q[1] - p[1]) / L
            doors.append((p[0] + ux * (t + 0.45), p[1] + uy * (t + 0.45)))
        # furniture-like clutter: along a random wall of a random room, kept
        # away from doorways so that the rooms stay connected
        placed = 0
        while placed < per_floor:
            rx0, ry0, rx1, ry1 = rooms[rng.integers(len(rooms))]
            side = rng.integers(4)
            box = placed % 2 == 0
            if box:
                ex, ey = rng.uniform(0.3, 1.5, size=2)
                yaw = rng.uniform(0, math.pi)
                rad = 0.5 * math.hypot(ex, ey)
            else:
                rad = rng.uniform(0.1, 0.5)
            off = 0.05 + rad + rng.uniform(0.0, 0.6)
            if side == 0:
                cx, cy = rng.uniform(rx0 + rad, rx1 - rad), ry0 + off
            elif side == 1:
                cx, cy = rng.uniform(rx0 + rad, rx1 - rad), ry1 - off
            elif side == 2:
                cx, cy = rx0 + off, rng.uniform(ry0 + rad, ry1 - rad)
            else:
                cx, cy = rx1 - off, rng.uniform(ry0 + rad, ry1 - rad)
            if any(math.hypot(cx - dx, cy - dy) < rad + 1.0 for dx, dy in doors):
                continue
            obst.append(("box", cx, cy, ex, ey, yaw) if box else ("cyl", cx, cy, rad))
            placed += 1
        rooms_all.append(rooms)
        walls_all.append(walls)
        obst_all.append(obst)
    return FloorPlan(tuple(extent), n_floors, ceiling, rooms_all, walls_all, obst_all)


def _plan_surfaces(rng, plan: FloorPlan, heights) -> _Surfaces:
    S = _Surfaces()
    W, H = plan.extent
    C = plan.ceiling
    floor_col = np.array([0.55, 0.42, 0.30])
    for f in range(plan.n_floors):
        z0 = f * C
        S.add_rect((0, 0, z0), (W, 0, 0), (0, H, 0), floor_col * (0.9 + 0.2 * rng.uniform()), 1)
        if f == plan.n_floors - 1:
            S.add_rect((0, 0, z0 + C), (W, 0, 0), (0, H, 0), np.array([0.92, 0.92, 0.90]), 2)
        for (p, q, door) in plan.walls[f]:
            p3 = np.array([p[0], p[1], z0])
            d = np.array([q[0] - p[0], q[1] - p[1], 0.0])
            L = np.linalg.norm(d)
            u = d / L
            col = _pastel(rng)
            if door is None:
                S.add_rect(p3, d, (0, 0, C), col, 3)
            else:
                dw, dh = 0.9, 2.1
                if door > 1e-3:
                    S.add_rect(p3, u * door, (0, 0, C), col, 3)
                S.add_rect(p3 + u * door + np.array([0, 0, dh]), u * dw, (0, 0, C - dh), col, 3)
                rest = L - door - dw
                if rest > 1e-3:
                    S.add_rect(p3 + u * (door + dw), u * rest, (0, 0, C), col, 3)
        for ob in plan.obstacles[f]:
            col = _pastel(rng) * 0.9
            if ob[0] == "box":
                _, cx, cy, ex, ey, yaw = ob
                ez = rng.uniform(0.3, 1.5)
                ux = np.array([math.cos(yaw), math.sin(yaw), 0.0])
                uy = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
                c = np.array([cx, cy, z0])
                corner = c - 0.5 * ex * ux - 0.5 * ey * uy
                zz = np.array([0, 0, ez])
                S.add_rect(corner, ux * ex, zz, col, 0)
                S.add_rect(corner + uy * ey, ux * ex, zz, col, 0)
                S.add_rect(corner, uy * ey, zz, col * 0.95, 0)
                S.add_rect(corner + ux * ex, uy * ey, zz, col * 0.95, 0)
                S.add_rect(corner + zz, ux * ex, uy * ey, col * 1.05, 0)
            else:
                _, cx, cy, r = ob
                h = rng.uniform(0.3, 1.8)
                S.cyls.append((np.array([cx, cy]), z0, r, h, col))
                S.disks.append((np.array([cx, cy, z0 + h]), r, col * 1.05))
    return S


def _pattern(kind, p, col):
    """Procedural low-frequency texture so images carry edges."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    if kind == 1:      # floor boards
        f = 0.85 + 0.15 * np.sign(np.sin(2 * math.pi * x / 0.4))
    elif kind == 2:    # ceiling tiles
        f = 0.9 + 0.1 * ((np.floor(x / 0.6) + np.floor(y / 0.6)) % 2)
    elif kind == 3:    # wall with a skirting band and soft stripes
        f = np.where(np.mod(z, 3.0) < 0.12, 0.55, 0.92 + 0.08 * np.sin(2 * math.pi * (x + y) / 1.3))
    else:
        f = np.ones_like(x)
    return np.clip(col[None, :] * f[:, None], 0.0, 1.0)


def make_floorplan(n_leaves: int, extent=(20.0, 15.0), n_floors: int = 1,
                   ceiling: float = 3.0, n_clutter: int = 300, sh_degree: int = 3,
                   seed: int = 1):
    """Leaves of a synthetic building.

    Returns (Scene of leaves, FloorPlan).  Leaves are allocated to surfaces in
    proportion to area so that the total is exactly ``n_leaves``; each leaf is
    a sheet Gaussian (in-plane scale 0.7x the local spacing, 5 mm thin axis,
    +-2.5 mm normal jitter), opacity sigmoid(N(3,1)), DC colour = surface
    colour + N(0,0.03), SH bands 1..3 ~ N(0,0.02).
    """
    rng = np.random.default_rng(seed)
    plan = _make_plan(rng, extent, n_floors, ceiling, n_clutter)
    S = _plan_surfaces(rng, plan, None)
    plan.surfaces = surfaces_array(S)
    areas = S.areas()
    share = areas / areas.sum() * n_leaves
    counts = np.floor(share).astype(np.int64)
    rem = n_leaves - counts.sum()
    if rem > 0:
        order = np.argsort(-(share - counts), kind="stable")
        counts[order[:rem]] += 1
    pos, t1, t2, nrm, col, spacing = [], [], [], [], [], []
    idx = 0
    for (o, a, b, c, pat) in S.rects:
        k = counts[idx]; idx += 1
        if k == 0:
            continue
        uv = _r2(k, rng)
        p = o[None] + uv[:, :1] * a[None] + uv[:, 1:] * b[None]
        ta = a / np.linalg.norm(a); tb = b / np.linalg.norm(b)
        nn = np.cross(ta, tb)
        pos.append(p); t1.append(np.repeat(ta[None], k, 0)); t2.append(np.repeat(tb[None], k, 0))
        nrm.append(np.repeat(nn[None], k, 0))
        col.append(_pattern(pat, p, c))
        spacing.append(np.full(k, math.sqrt(np.linalg.norm(a) * np.linalg.norm(b) / k)))
    for (cxy, z0, r, h, c) in S.cyls:
        k = counts[idx]; idx += 1
        if k == 0:
            continue
        uv = _r2(k, rng)
        th = 2 * math.pi * uv[:, 0]
        p = np.stack([cxy[0] + r * np.cos(th), cxy[1] + r * np.sin(th), z0 + h * uv[:, 1]], 1)
        nn = np.stack([np.cos(th), np.sin(th), np.zeros(k)], 1)
        ta = np.stack([-np.sin(th), np.cos(th), np.zeros(k)], 1)
        tb = np.repeat(np.array([[0.0, 0.0, 1.0]]), k, 0)
        pos.append(p); t1.append(ta); t2.append(tb); nrm.append(nn)
        col.append(np.repeat(c[None], k, 0))
        spacing.append(np.full(k, math.sqrt(2 * math.pi * r * h / k)))
    for (cc, r, c) in S.disks:
        k = counts[idx]; idx += 1
        if k == 0:
            continue
        uv = _r2(k, rng)
        rr = r * np.sqrt(uv[:, 0]); th = 2 * math.pi * uv[:, 1]
        p = np.stack([cc[0] + rr * np.cos(th), cc[1] + rr * np.sin(th), np.full(k, cc[2])], 1)
        pos.append(p)
        t1.append(np.repeat(np.array([[1.0, 0, 0]]), k, 0))
        t2.append(np.repeat(np.array([[0, 1.0, 0]]), k, 0))
        nrm.append(np.repeat(np.array([[0, 0, 1.0]]), k, 0))
        col.append(np.repeat(c[None], k, 0))
        spacing.append(np.full(k, math.sqrt(math.pi * r * r / k)))
    pos = np.concatenate(pos); t1 = np.concatenate(t1); t2 = np.concatenate(t2)
    nrm = np.concatenate(nrm); col = np.concatenate(col); spacing = np.concatenate(spacing)
    n = pos.shape[0]
    assert n == n_leaves, (n, n_leaves)
    pos = pos + nrm * rng.uniform(-0.0025, 0.0025, size=(n, 1))
    psi = rng.uniform(0, 2 * math.pi, size=(n, 1))
    e1 = np.cos(psi) * t1 + np.sin(psi) * t2
    e2 = -np.sin(psi) * t1 + np.cos(psi) * t2
    Rm = np.stack([e1, e2, nrm], axis=2)          # columns = local axes
    det = np.linalg.det(Rm)
    Rm[det < 0, :, 1] *= -1.0
    quats = _rotmat_to_quat(Rm)
    s_in = 0.7 * spacing[:, None] * np.exp(rng.normal(0.0, 0.15, size=(n, 2)))
    scales = np.concatenate([s_in, np.full((n, 1), 0.005)], axis=1)
    opacity = _sigmoid(rng.normal(3.0, 1.0, size=n))
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = (np.clip(col + rng.normal(0, 0.03, size=(n, 3)), 0, 1) - 0.5) / _Y00
    if K > 1:
        sh[:, 1:, :] = rng.normal(0, 0.02, size=(n, K - 1, 3))
    scene = Scene(pos.astype(np.float32), scales.astype(np.float32),
                  quats.astype(np.float32), opacity.astype(np.float32),
                  sh.astype(np.float32), sh_degree,
                  meta={"kind": "floorplan", "seed": seed, "extent": tuple(extent),
                        "n_floors": n_floors, "n_leaves": n_leaves})
    return scene, plan
