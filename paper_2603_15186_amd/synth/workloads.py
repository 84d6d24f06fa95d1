"""Named synthetic workloads (scene + cameras) with seeds, and a disk cache.

  box20k    : 20,000-Gaussian flat random box, one 256x256 camera (f=256).
  plan2m    : 2M-leaf 20x15 m floor plan, 8-level hierarchy, SH3;
              200-pose 1280x720 (f=900) trajectory at 1.2 m; tau = 1 px.
  plan8m    : 8M-leaf 40x30 m plan; 256 random views, 128@320x240,
              96@640x480, 32@1280x720 (f = 900 W/1280), height 0.3..1.5 m.
  plan2m-lod: the plan2m scene with 2,000 training and 500 held-out
              1280x720 poses at 1.2 m with uniform yaw; a held-out position
              is at least 0.15 m from every training position (the plan's
              navigable area, about 70 m^2, cannot keep 2,000 poses 0.5 m
              apart from 500 others).
  building30m: two 20x15 m floors, 30M leaves; 64 1920x1080 views (f=1300).

Scenes can be scaled down with ``scale`` (leaf count multiplier) for tests.
"""
from __future__ import annotations

import hashlib
import math
import os

import numpy as np

from .cameras import Camera, FreeSpace, box_camera, random_poses, trajectory, yaw_camera
from .hierarchy import build_hierarchy
from .scenes import Scene, make_floorplan, make_random_box

_SCENE_FIELDS = ("means", "scales", "quats", "opacity", "sh", "parent",
                 "first_child", "child_count", "bound", "level_offset")


def cache_dir():
    d = os.environ.get("HGS_SYNTH_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hgs_synth"))
    os.makedirs(d, exist_ok=True)
    return d


def _save(path, scene: Scene):
    arrs = {k: getattr(scene, k) for k in _SCENE_FIELDS if getattr(scene, k) is not None}
    tmp = path + ".tmp.npz"
    np.savez(tmp, sh_degree=np.int64(scene.sh_degree), **arrs)
    os.replace(tmp, path)


def _load(path) -> Scene:
    z = np.load(path, allow_pickle=False)
    kw = {k: (z[k] if k in z.files else None) for k in _SCENE_FIELDS}
    return Scene(kw.pop("means"), kw.pop("scales"), kw.pop("quats"), kw.pop("opacity"),
                 kw.pop("sh"), int(z["sh_degree"]), **kw)


def floorplan_scene(n_leaves, extent, n_floors, seed, sh_degree=3, n_clutter=300,
                    use_cache=True):
    """Hierarchical floor-plan scene and its plan (cached by parameters)."""
    key = f"plan_{n_leaves}_{extent[0]}x{extent[1]}_{n_floors}_{seed}_{sh_degree}_{n_clutter}_v2"
    path = os.path.join(cache_dir(), hashlib.sha1(key.encode()).hexdigest()[:16] + ".npz")
    leaves = None
    if use_cache and os.path.exists(path):
        scene = _load(path)
        from .scenes import _make_plan, _plan_surfaces, surfaces_array
        rng = np.random.default_rng(seed)    # same draws as make_floorplan
        plan = _make_plan(rng, extent, n_floors, 3.0, n_clutter)
        plan.surfaces = surfaces_array(_plan_surfaces(rng, plan, None))
        return scene, plan
    leaves, plan = make_floorplan(n_leaves, extent, n_floors, 3.0, n_clutter, sh_degree, seed)
    scene = build_hierarchy(leaves)
    if use_cache:
        _save(path, scene)
    return scene, plan


def box20k():
    return make_random_box(20000, seed=0), [box_camera(False)]


def _cams(pos, yaw, W, H, f):
    return [yaw_camera(W, H, f, p, y) for p, y in zip(pos, yaw)]


def plan2m(scale=1.0, n_poses=200, use_cache=True, with_plan=False):
    n = int(round(2_000_000 * scale))
    scene, plan = floorplan_scene(n, (20.0, 15.0), 1, seed=1, use_cache=use_cache)
    fs = FreeSpace(plan, 0)
    pos, yaw = trajectory(fs, n_poses, seed=101, height=1.2)
    out = (scene, _cams(pos, yaw, 1280, 720, 900.0))
    return out + (plan,) if with_plan else out


def plan8m_views(plan, n_views=(128, 96, 32), seed=102):
    fs = FreeSpace(plan, 0)
    total = sum(n_views)
    pos, yaw = random_poses(fs, total, seed, height=(0.3, 1.5))
    res = [(320, 240)] * n_views[0] + [(640, 480)] * n_views[1] + [(1280, 720)] * n_views[2]
    return [yaw_camera(W, H, 900.0 * W / 1280.0, p, y) for (W, H), p, y in zip(res, pos, yaw)]


def plan8m(scale=1.0, n_views=(128, 96, 32), use_cache=True):
    n = int(round(8_000_000 * scale))
    scene, plan = floorplan_scene(n, (40.0, 30.0), 1, seed=2, use_cache=use_cache)
    return scene, plan8m_views(plan, n_views)


def plan2m_lod(scale=1.0, n_train=2000, n_eval=500, use_cache=True, with_plan=False):
    n = int(round(2_000_000 * scale))
    scene, plan = floorplan_scene(n, (20.0, 15.0), 1, seed=1, use_cache=use_cache)
    fs = FreeSpace(plan, 0)
    tp, ty = random_poses(fs, n_train, 103, height=(1.2, 1.2))
    ep, ey = random_poses(fs, n_eval, 104, height=(1.2, 1.2), avoid=tp, min_sep=0.15)
    out = (scene, _cams(tp, ty, 1280, 720, 900.0), _cams(ep, ey, 1280, 720, 900.0))
    return out + (plan,) if with_plan else out


def building30m(scale=1.0, n_views=64, use_cache=True, with_plan=False):
    n = int(round(30_000_000 * scale))
    scene, plan = floorplan_scene(n, (20.0, 15.0), 2, seed=4, use_cache=use_cache)
    cams = []
    per = n_views // 2
    for f in range(2):
        fs = FreeSpace(plan, f)
        pos, yaw = trajectory(fs, per, seed=105 + f, height=1.2)
        cams += _cams(pos, yaw, 1920, 1080, 1300.0)
    return (scene, cams, plan) if with_plan else (scene, cams)


def building30m_training(plan, n_per_floor=300):
    """Training poses of the building's learned cut: random free positions on
    each floor (seeds 301, 302), 1.2 m high, uniform yaw, 1920x1080, f = 1300."""
    cams = []
    for f in range(2):
        pos, yaw = random_poses(FreeSpace(plan, f), n_per_floor, 301 + f, height=(1.2, 1.2))
        cams += _cams(pos, yaw, 1920, 1080, 1300.0)
    return cams


def building30m_calibration(plan, n_per_floor=8):
    """Poses for calibrating the learned cut's p* on the building: other
    trajectories (seeds 205, 206) at the same height and camera."""
    cams = []
    for f in range(2):
        pos, yaw = trajectory(FreeSpace(plan, f), n_per_floor, seed=205 + f, height=1.2)
        cams += _cams(pos, yaw, 1920, 1080, 1300.0)
    return cams


def nav_queries(nav, n_goals=9, per_goal=200, seed=0):
    """Planning queries on a navigable map ([ny, nx], nonzero = navigable):
    the paper's shape of 9 annotated goals with 200 trajectories each.
    Goals and starts are distinct-goal uniform draws from the largest
    4-connected navigable region (every cell of it reaches every other: a
    diagonal move needs both side cells navigable, so 8-connected regions
    without corner cutting are the 4-connected ones).  Returns (goals int32
    [n_goals], starts int32 [n_goals * per_goal], slots int32: the goal
    index of each start), cell indices j * nx + i."""
    from scipy import ndimage
    lab, n = ndimage.label(np.asarray(nav) != 0)
    if n == 0:
        raise ValueError("no navigable cell")
    sizes = np.bincount(lab.ravel())[1:]
    region = np.flatnonzero(lab.ravel() == 1 + int(np.argmax(sizes)))
    rng = np.random.default_rng(seed)
    goals = rng.choice(region, size=n_goals, replace=False).astype(np.int32)
    starts = rng.choice(region, size=n_goals * per_goal).astype(np.int32)
    slots = np.repeat(np.arange(n_goals, dtype=np.int32), per_goal)
    return goals, starts, slots
