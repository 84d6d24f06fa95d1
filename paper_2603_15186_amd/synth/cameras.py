"""Seeded pinhole cameras and robot poses.

Rendering needs only a camera's intrinsics and extrinsics (NavGSim Sec. III-A).
Conventions: world z is up; the camera frame has x right, y down, z forward;
``R`` maps world to camera coordinates (its rows are the right, down and
forward axes) and ``position`` is the camera centre in world coordinates.
Poses are horizontal (no pitch or roll) at a given height and yaw, as for a
ground robot.
"""
from __future__ import annotations

import collections
import dataclasses
import math

import numpy as np

from .scenes import FloorPlan


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    position: np.ndarray      # (3,) f32
    R: np.ndarray             # (3,3) f32 world->camera, rows right/down/forward
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


def yaw_camera(width, height, fx, position, yaw, fy=None, cx=None, cy=None,
               znear=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Horizontal camera at ``position`` looking along (cos yaw, sin yaw, 0)."""
    fwd = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.array([0.0, 0.0, -1.0])
    R = np.stack([right, down, fwd]).astype(np.float32)
    return Camera(int(width), int(height), float(fx), float(fx if fy is None else fy),
                  float(width / 2 if cx is None else cx), float(height / 2 if cy is None else cy),
                  np.asarray(position, np.float32), R, float(znear), tuple(bg))


def box_camera(center_view: bool = False) -> Camera:
    """256x256, f=256 camera for the random-box scene: outside the 4x4x3 m box
    at (2,-1,1.5) looking +y, or (secondary case) at the box centre."""
    pos = (2.0, 2.0, 1.5) if center_view else (2.0, -1.0, 1.5)
    return yaw_camera(256, 256, 256.0, pos, math.pi / 2)


# ---------------------------------------------------------------------------
# Free space and trajectories on a floor plan
# ---------------------------------------------------------------------------

class FreeSpace:
    """Occupancy of one floor on a 5 cm grid, with a clearance margin."""

    def __init__(self, plan: FloorPlan, floor: int = 0, cell: float = 0.05,
                 clearance: float = 0.3):
        from scipy import ndimage
        W, H = plan.extent
        self.cell = cell
        nx, ny = int(math.ceil(W / cell)), int(math.ceil(H / cell))
        occ = np.zeros((nx, ny), bool)
        xs = (np.arange(nx) + 0.5) * cell
        ys = (np.arange(ny) + 0.5) * cell
        X, Y = np.meshgrid(xs, ys, indexing="ij")
        for (p, q, door) in plan.walls[floor]:
            p = np.asarray(p, float); q = np.asarray(q, float)
            d = q - p; L = np.linalg.norm(d); u = d / L
            t = (X - p[0]) * u[0] + (Y - p[1]) * u[1]
            dist = np.abs((X - p[0]) * u[1] - (Y - p[1]) * u[0])
            on = (dist < 0.03) & (t > -0.03) & (t < L + 0.03)
            if door is not None:
                on &= ~((t > door) & (t < door + 0.9))
            occ |= on
        for ob in plan.obstacles[floor]:
            if ob[0] == "box":
                _, cx, cy, ex, ey, yaw = ob
                lx = (X - cx) * math.cos(yaw) + (Y - cy) * math.sin(yaw)
                ly = -(X - cx) * math.sin(yaw) + (Y - cy) * math.cos(yaw)
                occ |= (np.abs(lx) < ex / 2) & (np.abs(ly) < ey / 2)
            else:
                _, cx, cy, r = ob
                occ |= (X - cx) ** 2 + (Y - cy) ** 2 < r * r
        edt = ndimage.distance_transform_edt(~occ) * cell
        free = edt >= clearance
        # Keep the largest 4-connected free region so every goal is reachable.
        lab, nlab = ndimage.label(free)
        if nlab > 1:
            sizes = np.bincount(lab.ravel())
            sizes[0] = 0
            free = lab == int(np.argmax(sizes))
        self.free = free
        self.shape = (nx, ny)
        self.floor_z = floor * plan.ceiling

    def cells(self):
        return np.argwhere(self.free)

    def to_xy(self, ij):
        return (np.asarray(ij, float) + 0.5) * self.cell

    def bfs_path(self, start, goal):
        nx, ny = self.shape
        prev = -np.ones(nx * ny, np.int64)
        s = start[0] * ny + start[1]; g = goal[0] * ny + goal[1]
        prev[s] = s
        dq = collections.deque([s])
        free = self.free.ravel()
        while dq:
            c = dq.popleft()
            if c == g:
                break
            i, j = divmod(c, ny)
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                a, b = i + di, j + dj
                if 0 <= a < nx and 0 <= b < ny:
                    k = a * ny + b
                    if free[k] and prev[k] < 0:
                        prev[k] = c
                        dq.append(k)
        if prev[g] < 0:
            return None
        path = [g]
        while path[-1] != s:
            path.append(prev[path[-1]])
        path.reverse()
        return np.array([divmod(c, ny) for c in path])


def trajectory(space: FreeSpace, n_poses: int, seed: int, height: float = 1.2,
               step: float = 0.25):
    """Positions and yaws every ``step`` metres along shortest grid paths
    between random free-space goals; yaw follows the heading."""
    rng = np.random.default_rng(seed)
    cells = space.cells()
    cur = cells[rng.integers(len(cells))]
    pts = [space.to_xy(cur)]
    while len(pts) < n_poses + 1:
        goal = cells[rng.integers(len(cells))]
        path = space.bfs_path(tuple(cur), tuple(goal))
        if path is None or len(path) < 2:
            continue
        xy = space.to_xy(path)
        seg = np.linalg.norm(np.diff(xy, axis=0), axis=1)
        s = np.concatenate([[0], np.cumsum(seg)])
        t = np.arange(step, s[-1], step)
        for tt in t:
            pts.append(np.array([np.interp(tt, s, xy[:, 0]), np.interp(tt, s, xy[:, 1])]))
        cur = goal
    pts = np.array(pts[:n_poses + 1])
    d = np.diff(pts, axis=0)
    yaw = np.arctan2(d[:, 1], d[:, 0])
    pos = np.concatenate([pts[:-1], np.full((n_poses, 1), space.floor_z + height)], axis=1)
    return pos, yaw


def random_poses(space: FreeSpace, n: int, seed: int, height=(1.2, 1.2),
                 avoid=None, min_sep: float = 0.0):
    """Random free-space positions with uniform yaw; heights uniform in
    ``height``; positions closer than ``min_sep`` (xy) to any of ``avoid``
    are redrawn."""
    rng = np.random.default_rng(seed)
    cells = space.cells()
    out_p, out_y = [], []
    while len(out_p) < n:
        c = cells[rng.integers(len(cells))]
        xy = space.to_xy(c) + rng.uniform(-0.5, 0.5, size=2) * space.cell
        if avoid is not None and min_sep > 0:
            if np.min(np.linalg.norm(avoid[:, :2] - xy[None], axis=1)) < min_sep:
                continue
        z = space.floor_z + rng.uniform(height[0], height[1])
        out_p.append([xy[0], xy[1], z])
        out_y.append(rng.uniform(0, 2 * math.pi))
    return np.array(out_p), np.array(out_y)
