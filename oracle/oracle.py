"""Python front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it; the renderer never imports it.  See ``oracle.c`` for
the definition it computes and the passages of NavGSim (arXiv 2603.15186) it
follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")
SOURCES = [SRC_PATH, os.path.join(HERE, "slice.c"), os.path.join(HERE, "nav.c")]

MODE_ALL_LEAVES = 0
MODE_THRESHOLD = 1

# Relative margins within which a compositing decision may go either way:
# q vs 9, alpha vs 1/255f, transmittance vs 1e-4f.  They bound the error of a
# single-precision evaluation of the same quantities (derivation in the
# design notes); decisions inside them are forked.
DEFAULT_EPS = (1e-4, 1e-4, 5e-4)


# The compiler flags that define the oracle's arithmetic.
CFLAGS = ["-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

# HGS_ORACLE_LIB names another build of the same sources to load instead (the
# sanitizer test points it at an address/undefined-behaviour sanitized build).
SAN_ENV = "HGS_ORACLE_LIB"


def build(force: bool = False, out: str = LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP) into
    `out`; `extra` adds flags (e.g. sanitizers) to the optimised build."""
    if os.environ.get(SAN_ENV) and out == LIB_PATH and not force:
        return os.environ[SAN_ENV]
    stale = not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(f) for f in SOURCES)
    if force or stale:
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", *CFLAGS, *extra, *SOURCES, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("position", ctypes.c_float * 3), ("R", ctypes.c_float * 9),
                ("znear", ctypes.c_float), ("bg", ctypes.c_float * 3)]


def _cam(c) -> _Camera:
    k = _Camera()
    k.width, k.height = int(c.width), int(c.height)
    k.fx, k.fy, k.cx, k.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    for i in range(3):
        k.position[i] = float(np.float32(c.position[i]))
        k.bg[i] = float(c.bg[i])
    R = np.asarray(c.R, np.float32).ravel()
    for i in range(9):
        k.R[i] = float(R[i])
    k.znear = float(c.znear)
    return k


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        L.or_cut.restype = ctypes.c_int64
        L.or_cut.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.POINTER(_Camera),
                             ctypes.c_int32, ctypes.c_float, P, ctypes.c_int64]
        L.or_project.restype = None
        L.or_project.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32,
                                 ctypes.POINTER(_Camera), P]
        L.or_project_blend.restype = None
        L.or_project_blend.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32, P, P, P, ctypes.c_int64, P,
                                       ctypes.c_float, ctypes.POINTER(_Camera), P, P]
        L.or_render_pixels.restype = ctypes.c_int32
        L.or_render_pixels.argtypes = [ctypes.c_int64, P, ctypes.POINTER(_Camera), ctypes.c_int64,
                                       P, P, P, ctypes.c_int32, P, P, P, P]
        L.or_sh_basis.restype = None
        L.or_sh_basis.argtypes = [P, P]
        L.or_slice_params.restype = None
        L.or_slice_params.argtypes = [ctypes.c_int64, P, P, P]
        L.or_slice_occupancy.restype = None
        L.or_slice_occupancy.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P,
                                         ctypes.c_double, ctypes.c_double, P]
        L.or_disc_collision.restype = None
        L.or_disc_collision.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int64, P, ctypes.c_double, ctypes.c_double, P]
        L.or_cut_learned.restype = ctypes.c_int64
        L.or_cut_learned.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, ctypes.c_int32, P, P, P,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Camera),
                                     ctypes.c_float, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.or_navigable.restype = None
        L.or_navigable.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_double, ctypes.c_double, P]
        L.or_distance_fields.restype = None
        L.or_distance_fields.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]
        L.or_trace_paths.restype = None
        L.or_trace_paths.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, P, P, ctypes.c_int32,
                                     P, P]
        L.or_proj_stride.restype = ctypes.c_int32
        L.or_num_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# Column layout of ``project``'s output.
PROJ_FIELDS = ("valid", "u", "v", "A", "B", "C", "S00", "S01", "S11", "r", "g", "b",
               "z", "zkey", "opacity", "tx", "ty")
PF = {k: i for i, k in enumerate(PROJ_FIELDS)}


def num_threads() -> int:
    return int(lib().or_num_threads())


def sh_basis(d) -> np.ndarray:
    """Real SH Y_lm(d), index l*l + l + m, l <= 3, for a unit direction."""
    d = _c(d, np.float64)
    out = np.zeros(16)
    lib().or_sh_basis(_p(d), _p(out))
    return out


def cut(scene, cam, mode=MODE_THRESHOLD, tau=1.0) -> np.ndarray:
    """Ascending node ids of the level-of-detail cut."""
    L = lib()
    n = scene.n
    k = _cam(cam)
    if scene.parent is None:
        return np.arange(n, dtype=np.int32)
    bound = _c(scene.bound, np.float32); par = _c(scene.parent, np.int32)
    fc = _c(scene.first_child, np.int32); cc = _c(scene.child_count, np.int32)
    cap = 1 << 16
    while True:
        out = np.empty(cap, np.int32)
        cnt = L.or_cut(n, _p(bound), _p(par), _p(fc), _p(cc), ctypes.byref(k), int(mode),
                       float(tau), _p(out), cap)
        if cnt <= cap:
            return out[:cnt].copy()
        cap = int(cnt)


def cut_learned(scene, cam, params, mean, std, p_star, s_hi, tau=1.0, margin=1e-3, flip=()):
    """Learned level-of-detail cut (see oracle.c): (ascending node ids,
    ascending undecided candidates: logit within `margin` of logit(p*)).
    params: the network's 1377 parameters as used (BF16 values); mean, std:
    feature standardisation; 0 < p* < 1.  Undecided candidates listed in
    `flip` take the other (equally valid) decision; listing a decided one
    raises ValueError."""
    L = lib()
    if not 0.0 < float(p_star) < 1.0:
        raise ValueError("p* must lie in (0, 1)")
    n = scene.n
    lvl = np.zeros(n, np.int32)
    lo = np.asarray(scene.level_offset, np.int64)
    for l in range(lo.size - 1):
        lvl[lo[l]:lo[l + 1]] = l
    arrs = [_c(scene.bound, np.float32), _c(scene.parent, np.int32), _c(scene.first_child, np.int32),
            _c(scene.child_count, np.int32), lvl, _c(scene.quats, np.float32), _c(scene.scales, np.float32),
            _c(scene.opacity, np.float32), _c(scene.sh, np.float32)]
    w = _c(params, np.float64); mu = _c(mean, np.float64); sd = _c(std, np.float64)
    ps = float(np.float32(p_star))
    z_star = math.log(ps) - math.log1p(-ps)
    k = _cam(cam)
    cap = 1 << 16
    while True:
        out = np.empty(cap, np.int32)
        amb = np.empty(cap, np.int32)
        na = ctypes.c_int64()
        bad = ctypes.c_int64()
        fl = np.unique(np.asarray(flip, np.int32))
        cnt = L.or_cut_learned(n, *[_p(a) for a in arrs[:9]], int(scene.sh_degree), _p(w), _p(mu), _p(sd),
                               z_star, float(s_hi), float(margin), ctypes.byref(k), float(tau), _p(fl), fl.size,
                               _p(out), cap, _p(amb), cap, ctypes.byref(na), ctypes.byref(bad))
        if bad.value:
            raise ValueError(f"{bad.value} flipped candidates are decided")
        if cnt <= cap and na.value <= cap:
            return out[:cnt].copy(), amb[:na.value].copy()
        cap = int(max(cnt, na.value))


def project(scene, ids, cam) -> np.ndarray:
    """FP64 projection of the Gaussians ``ids``: (m, len(PROJ_FIELDS))."""
    L = lib()
    ids = _c(ids, np.int32)
    m = ids.size
    stride = int(L.or_proj_stride())
    out = np.zeros((m, stride))
    means = _c(scene.means, np.float32); scales = _c(scene.scales, np.float32)
    quats = _c(scene.quats, np.float32); op = _c(scene.opacity, np.float32)
    sh = _c(scene.sh, np.float32)
    L.or_project(m, _p(ids), _p(means), _p(scales), _p(quats), _p(op), _p(sh),
                 int(scene.sh_degree), ctypes.byref(_cam(cam)), _p(out))
    return out


def project_blend(scene, ids, cam, tau, with_t=False, cut_ids=None):
    """FP64 projection with level-of-detail blending (see oracle.c): each
    cut node is interpolated toward its parent by t = clamp((s_p - tau) /
    (s_p - s_g), 0, 1); the first of a parent's children in the cut carries
    the parent's opacity, the others fade in from 0.  cut_ids: the whole cut
    (ascending; default: ids)."""
    L = lib()
    ids = _c(ids, np.int32)
    cut_ids = ids if cut_ids is None else _c(cut_ids, np.int32)
    if np.any(np.diff(cut_ids) <= 0):
        raise ValueError("the cut's ids must be ascending")
    m = ids.size
    out = np.zeros((m, int(L.or_proj_stride())))
    tout = np.zeros(m)
    means = _c(scene.means, np.float32); scales = _c(scene.scales, np.float32)
    quats = _c(scene.quats, np.float32); op = _c(scene.opacity, np.float32)
    sh = _c(scene.sh, np.float32)
    par = _c(scene.parent, np.int32); fc = _c(scene.first_child, np.int32); bound = _c(scene.bound, np.float32)
    L.or_project_blend(m, _p(ids), _p(means), _p(scales), _p(quats), _p(op), _p(sh), int(scene.sh_degree), _p(par),
                       _p(fc), _p(bound), cut_ids.size, _p(cut_ids), float(tau), ctypes.byref(_cam(cam)), _p(out),
                       _p(tout))
    return (out, tout) if with_t else out


class PixelResult:
    """Oracle output for a set of pixels.

    branches[i, b] = (R, G, B, depth, alpha) of branch b (b < nbranch[i]);
    branch 0 follows every FP64 decision.
    """

    def __init__(self, px, py, branches, nbranch, nalg, flags):
        self.px, self.py = px, py
        self.branches, self.nbranch, self.nalg, self.flags = branches, nbranch, nalg, flags

    @property
    def primary(self):
        return self.branches[:, 0, :]


def render_pixels(proj, cam, px, py, eps=DEFAULT_EPS, cap=8) -> PixelResult:
    L = lib()
    proj = _c(proj, np.float64)
    px = _c(px, np.int32); py = _c(py, np.int32)
    n = px.size
    out = np.zeros((n, cap, 5))
    nb = np.zeros(n, np.int32); nalg = np.zeros(n, np.int64); fl = np.zeros(n, np.int32)
    e = _c(eps, np.float64)
    rc = L.or_render_pixels(proj.shape[0], _p(proj), ctypes.byref(_cam(cam)), n, _p(px), _p(py),
                            _p(e), int(cap), _p(out), _p(nb), _p(nalg), _p(fl))
    if rc != 0:
        raise MemoryError("oracle render_pixels failed")
    return PixelResult(px, py, out, nb, nalg, fl)


def render(scene, cam, mode=MODE_THRESHOLD, tau=1.0, eps=DEFAULT_EPS, cap=8, ids=None, blend=False):
    """Full-image oracle render (with blend: level-of-detail transition
    blending, see project_blend).  Returns (PixelResult over all pixels in
    row-major order, cut ids, projection)."""
    if ids is None:
        ids = cut(scene, cam, mode, tau)
    proj = project_blend(scene, ids, cam, tau) if blend else project(scene, ids, cam)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    res = render_pixels(proj, cam, xx.ravel(), yy.ravel(), eps, cap)
    return res, ids, proj


def image(res: PixelResult, cam):
    """(rgb[3,H,W], depth[H,W], alpha[H,W]) of branch 0 of a full render."""
    p = res.primary
    H, W = cam.height, cam.width
    return (p[:, :3].T.reshape(3, H, W).copy(), p[:, 3].reshape(H, W).copy(),
            p[:, 4].reshape(H, W).copy())


# ------------------------------------------------------------------ GS-slice

def slice_params(scales, quats) -> np.ndarray:
    """Per Gaussian (alpha, beta, lambda, c_xx, c_xy, c_yy) of the horizontal
    slice (see slice.c)."""
    scales = _c(scales, np.float32); quats = _c(quats, np.float32)
    n = scales.shape[0]
    out = np.zeros((n, 6))
    lib().or_slice_params(n, _p(scales), _p(quats), _p(out))
    return out


def slice_occupancy(means, scales, quats, opacity, x0, y0, cell, nx, ny, heights, rho_min=0.5, amb=1e-9):
    """(n_planes, ny, nx) int8 map: 0 free, 1 occupied, 2 undecided."""
    means = _c(means, np.float32); scales = _c(scales, np.float32)
    quats = _c(quats, np.float32); opacity = _c(opacity, np.float32)
    heights = _c(heights, np.float32)
    occ = np.zeros((heights.size, ny, nx), np.int8)
    lib().or_slice_occupancy(means.shape[0], _p(means), _p(scales), _p(quats), _p(opacity), float(x0), float(y0),
                             float(cell), int(nx), int(ny), heights.size, _p(heights), float(rho_min), float(amb),
                             _p(occ))
    return occ


def disc_collision(occ_map, x0, y0, cell, xy, radius, amb=1e-9):
    """Per query (x, y): 1 if a disc of `radius` meets an occupied cell of
    occ_map ([ny, nx] bytes), 0 if not, 2 if undecided (see slice.c)."""
    m = _c(occ_map, np.uint8)
    ny, nx = m.shape
    xy = _c(xy, np.float64).reshape(-1, 2)
    out = np.zeros(xy.shape[0], np.int8)
    lib().or_disc_collision(_p(m), float(x0), float(y0), float(cell), int(nx), int(ny), xy.shape[0], _p(xy),
                            float(radius), float(amb), _p(out))
    return out


# ------------------------------------------------------------------ planning


def navigable(occ_map, x0, y0, cell, radius, amb=1e-9):
    """[ny, nx] int8: 1 where a disc robot of `radius` centred on the cell is
    collision free, 0 where it collides, 2 undecided (see nav.c)."""
    m = _c(occ_map, np.uint8)
    ny, nx = m.shape
    out = np.zeros((ny, nx), np.int8)
    lib().or_navigable(_p(m), float(x0), float(y0), float(cell), int(nx), int(ny), float(radius), float(amb),
                       _p(out))
    return out


def distance_fields(nav, goals):
    """Shortest-path distances to each goal cell (index j*nx + i) over the
    8-connected navigable grid: int64 array [n_goals, ny, nx, 2] of (a, b) =
    (orthogonal, diagonal) moves, cost a + b sqrt 2; (-1, -1) unreachable."""
    m = _c(nav, np.uint8)
    ny, nx = m.shape
    goals = _c(goals, np.int64).ravel()
    out = np.zeros((goals.size, ny, nx, 2), np.int64)
    lib().or_distance_fields(_p(m), int(nx), int(ny), goals.size, _p(goals), _p(out))
    return out


def trace_paths(nav, dist, starts, slots, cap):
    """Trajectories from cells `starts` down fields dist[slots]: (paths
    [n, cap] int64 cell indices, lengths [n]); see nav.c for the rule."""
    m = _c(nav, np.uint8)
    ny, nx = m.shape
    dist = _c(dist, np.int64)
    starts = _c(starts, np.int64).ravel()
    slots = _c(slots, np.int32).ravel()
    n = starts.size
    paths = np.full((n, max(int(cap), 1)), -1, np.int64)
    lens = np.zeros(n, np.int64)
    lib().or_trace_paths(_p(m), int(nx), int(ny), _p(dist), n, _p(starts), _p(slots), int(cap), _p(paths),
                         _p(lens))
    return paths[:, :cap], lens
