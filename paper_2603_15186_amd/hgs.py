"""ctypes binding of libhgs.so (the C ABI in include/hgs.h).

The functions keep the C names and only marshal arguments: every step of a
render runs in the library's HIP kernels.  PyTorch provides device memory and
streams.  There is no fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgs.so")

HGS_OK = 0
HGS_E_INVALID = -1
HGS_E_STATE = -2
HGS_E_OOM = -3
HGS_E_HIP = -4
HGS_E_CAPACITY = -5
HGS_E_BAD_HIERARCHY = -6
HGS_E_UNSUPPORTED = -7

HGS_LOD_ALL_LEAVES = 0
HGS_LOD_THRESHOLD = 1
HGS_LOD_LEARNED = 2

HGS_OPT_SYNC_CHECK = 1
HGS_OPT_AUTO_REGROW = 2
HGS_OPT_COUNT_NALG = 3
HGS_OPT_BATCH_DEPTH = 4
HGS_OPT_USE_GRAPH = 5
HGS_OPT_PERSISTENT = 6
HGS_OPT_EXACT_TILES = 7
HGS_OPT_INITIAL_CAPACITY = 8
HGS_OPT_STAGE_TIMING = 9

PROJECTED_FIELDS = ("u", "v", "A", "B", "C", "r", "g", "b", "depth", "opacity", "ntiles", "valid")


class hgs_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class hgs_hierarchy(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("parent", ctypes.c_void_p), ("first_child", ctypes.c_void_p),
                ("child_count", ctypes.c_void_p), ("bound", ctypes.c_void_p), ("n_levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("level_offset", ctypes.c_void_p)]


class hgs_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("position", ctypes.c_float * 3), ("R", ctypes.c_float * 9), ("znear", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class hgs_output(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


class hgs_stats(ctypes.Structure):
    _fields_ = [("cut_size", ctypes.c_int64), ("visible", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("n_alg", ctypes.c_int64), ("tiles", ctypes.c_int64), ("regrows", ctypes.c_int64),
                ("timed_renders", ctypes.c_int64), ("ms_cut", ctypes.c_double), ("ms_project", ctypes.c_double), ("ms_sort", ctypes.c_double),
                ("ms_composite", ctypes.c_double), ("ms_total", ctypes.c_double)]


# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
EXPORTS = [
    ("hgs_create", ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(_P)]),
    ("hgs_destroy", None, [_P]),
    ("hgs_last_error", ctypes.c_char_p, [_P]),
    ("hgs_validate_scene", ctypes.c_int32, [ctypes.POINTER(hgs_gaussians), ctypes.POINTER(hgs_hierarchy),
                                            ctypes.c_char_p, ctypes.c_int64]),
    ("hgs_load_scene", ctypes.c_int32, [_P, ctypes.POINTER(hgs_gaussians), ctypes.POINTER(hgs_hierarchy)]),
    ("hgs_set_cameras", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(hgs_camera)]),
    ("hgs_set_lod", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_float]),
    ("hgs_set_option", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64]),
    ("hgs_render", ctypes.c_int32, [_P, _P, ctypes.POINTER(hgs_output)]),
    ("hgs_check", ctypes.c_int32, [_P]),
    ("hgs_get_cut", ctypes.c_int32, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("hgs_get_projected", ctypes.c_int32, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("hgs_get_stats", ctypes.c_int32, [_P, ctypes.POINTER(hgs_stats)]),
    ("hgs_sort_pairs", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhgs.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libhgs.so not found at {path}; build it with paper_2603_15186_amd/build.py")
    import torch  # noqa: F401  -- load torch's HIP runtime first
    lib = ctypes.CDLL(path)
    for name, res, args in EXPORTS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hgs status {status}: {msg}")
        self.status = status


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_gaussians(scene, keep):
    """hgs_gaussians view of a scene's arrays; `keep` collects the owners."""
    arrs = [_np(scene.means, np.float32), _np(scene.scales, np.float32), _np(scene.quats, np.float32),
            _np(scene.opacity, np.float32), _np(scene.sh, np.float32)]
    keep.extend(arrs)
    g = hgs_gaussians(scene.n, int(scene.sh_degree), 0, *[_ptr(a) for a in arrs])
    return g


def make_hierarchy(scene, keep):
    if scene.parent is None:
        return None
    arrs = [_np(scene.parent, np.int32), _np(scene.first_child, np.int32), _np(scene.child_count, np.int32),
            _np(scene.bound, np.float32), _np(scene.level_offset, np.int64)]
    keep.extend(arrs)
    return hgs_hierarchy(scene.n, _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), _ptr(arrs[3]),
                         len(scene.level_offset) - 1, 0, _ptr(arrs[4]))


def make_camera(cam) -> hgs_camera:
    k = hgs_camera()
    k.width, k.height = int(cam.width), int(cam.height)
    k.fx, k.fy, k.cx, k.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float32).ravel()
    for i in range(9):
        k.R[i] = float(R[i])
    for i in range(3):
        k.position[i] = float(np.float32(cam.position[i]))
        k.bg[i] = float(cam.bg[i])
    k.znear = float(cam.znear)
    return k


def validate_scene(scene):
    """Host-only validation: (status, message)."""
    lib = load_library()
    keep = []
    g = make_gaussians(scene, keep)
    h = make_hierarchy(scene, keep)
    buf = ctypes.create_string_buffer(512)
    st = lib.hgs_validate_scene(ctypes.byref(g), ctypes.byref(h) if h is not None else None, buf, 512)
    return st, buf.value.decode()


class Renderer:
    """A context on one GPU: load a scene, set cameras and LOD, render into
    torch tensors (planar rgb[3,H,W], depth[H,W], alpha[H,W])."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.hgs_create(int(device), ctypes.byref(h))
        if st != HGS_OK:
            raise HgsError(st, "hgs_create failed")
        self.ctx = h
        self.device = device
        self.cams = []

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != HGS_OK:
            raise HgsError(st, self.lib.hgs_last_error(self.ctx).decode())
        return st

    def load_scene(self, scene):
        keep = []
        g = make_gaussians(scene, keep)
        h = make_hierarchy(scene, keep)
        self._check(self.lib.hgs_load_scene(self.ctx, ctypes.byref(g), ctypes.byref(h) if h is not None else None))

    def set_cameras(self, cams):
        arr = (hgs_camera * len(cams))(*[make_camera(c) for c in cams])
        self._check(self.lib.hgs_set_cameras(self.ctx, len(cams), arr))
        self.cams = list(cams)

    def set_lod(self, mode, tau=1.0):
        self._check(self.lib.hgs_set_lod(self.ctx, int(mode), float(tau)))

    def set_option(self, opt, value):
        self._check(self.lib.hgs_set_option(self.ctx, int(opt), int(value)))

    def alloc_outputs(self):
        import torch
        dev = torch.device("cuda", self.device)
        outs = []
        for c in self.cams:
            outs.append((torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev),
                         torch.empty((c.height, c.width), dtype=torch.float32, device=dev),
                         torch.empty((c.height, c.width), dtype=torch.float32, device=dev)))
        return outs

    def render(self, outs=None, stream=None):
        """Render every view; returns the list of (rgb, depth, alpha)."""
        import torch
        if outs is None:
            outs = self.alloc_outputs()
        arr = (hgs_output * len(outs))()
        for i, (rgb, dep, alp) in enumerate(outs):
            for t in (rgb, dep, alp):
                if t is not None and (not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()):
                    raise ValueError("outputs must be contiguous float32 CUDA tensors")
            c = self.cams[i]
            if tuple(rgb.shape) != (3, c.height, c.width):
                raise ValueError(f"view {i}: rgb must have shape (3, {c.height}, {c.width})")
            arr[i].rgb = rgb.data_ptr()
            arr[i].depth = dep.data_ptr() if dep is not None else None
            arr[i].alpha = alp.data_ptr() if alp is not None else None
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hgs_render(self.ctx, ctypes.c_void_p(stream.cuda_stream), arr))
        return outs

    def check(self):
        return self.lib.hgs_check(self.ctx)

    def get_cut(self, view=0):
        n = ctypes.c_int64()
        self._check(self.lib.hgs_get_cut(self.ctx, view, None, 0, ctypes.byref(n)))
        out = np.empty(max(n.value, 1), np.int32)
        self._check(self.lib.hgs_get_cut(self.ctx, view, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def get_projected(self, view=0):
        n = ctypes.c_int64()
        self._check(self.lib.hgs_get_projected(self.ctx, view, None, 0, ctypes.byref(n)))
        out = np.empty((max(n.value, 1), 12), np.float32)
        self._check(self.lib.hgs_get_projected(self.ctx, view, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def stats(self) -> dict:
        s = hgs_stats()
        self._check(self.lib.hgs_get_stats(self.ctx, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in hgs_stats._fields_}

    def sort_pairs(self, keys, vals, key_bits, stream=None):
        """Sort device uint32 tensors (as int32 storage) in place."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hgs_sort_pairs(self.ctx, ctypes.c_void_p(stream.cuda_stream), keys.data_ptr(),
                                            vals.data_ptr(), keys.numel(), int(key_bits)))
