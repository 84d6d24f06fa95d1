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
LIB_PATH = os.environ.get("HGS_LIBRARY") or os.path.join(HERE, "libhgs.so")

HGS_OK = 0
HGS_E_INVALID = -1
HGS_E_STATE = -2
HGS_E_OOM = -3
HGS_E_HIP = -4
HGS_E_CAPACITY = -5
HGS_E_BAD_HIERARCHY = -6
HGS_E_UNSUPPORTED = -7
HGS_SORT_NOALLOC_MAX = 4194304

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
HGS_OPT_SORT_DIGIT_BITS = 10
HGS_OPT_PASS_VIEWS = 11
HGS_OPT_LOD_BLEND = 12
HGS_OPT_LANES = 13
HGS_OPT_KEEP_STATE = 14
HGS_OPT_TILE_SHAPE = 15
HGS_OPT_PIXELS_PER_THREAD = 16

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


class hgs_region(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("ref", ctypes.c_void_p), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("ref_w", ctypes.c_int32), ("ref_h", ctypes.c_int32), ("x0", ctypes.c_int32), ("y0", ctypes.c_int32)]


class hgs_stats(ctypes.Structure):
    _fields_ = [("cut_size", ctypes.c_int64), ("visible", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("n_alg", ctypes.c_int64), ("tiles", ctypes.c_int64), ("regrows", ctypes.c_int64),
                ("timed_renders", ctypes.c_int64), ("graph_launches", ctypes.c_int64), ("ms_cut", ctypes.c_double), ("ms_project", ctypes.c_double), ("ms_sort", ctypes.c_double),
                ("ms_composite", ctypes.c_double), ("ms_total", ctypes.c_double), ("passes", ctypes.c_int64),
                ("n_eval", ctypes.c_int64), ("timed_backwards", ctypes.c_int64), ("ms_bwd_composite", ctypes.c_double),
                ("ms_bwd_total", ctypes.c_double), ("visited", ctypes.c_int64)]


class hgs_slice_grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("cell", ctypes.c_double), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("n_planes", ctypes.c_int32), ("rho_min", ctypes.c_float),
                ("heights", ctypes.c_void_p)]


class hgs_image_grad(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


class hgs_scene_grad(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class hgs_plan(ctypes.Structure):
    _fields_ = [("batch_depth", ctypes.c_int32), ("persistent", ctypes.c_int32), ("sort_digit_bits", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("ms", ctypes.c_double), ("ms_default", ctypes.c_double),
                ("lanes", ctypes.c_int32), ("reserved", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("pixels_per_thread", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


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
    ("hgs_autotune", ctypes.c_int32, [_P, _P, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(hgs_plan)]),
    ("hgs_sort_pairs", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32]),
    ("hgs_sort_pairs_noalloc", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32]),
    ("hgs_set_keep_nodes", ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    ("hgs_lod_candidates", ctypes.c_int32, [_P, _P, ctypes.c_float, _P, _P, _P, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64)]),
    ("hgs_load_lod_mlp", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_float, ctypes.c_float]),
    ("hgs_mlp_forward", ctypes.c_int32, [_P, _P, _P, ctypes.c_int64, _P, _P, _P, _P]),
    ("hgs_mlp_train_step", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P,
                                            ctypes.c_int32, ctypes.c_float, _P, _P]),
    ("hgs_mlp_backward", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    ("hgs_mlp_adam", ctypes.c_int32, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_float]),
    ("hgs_mlp_bf16_from_master", ctypes.c_int32, [_P, _P, _P, _P]),
    ("hgs_feature_stats", ctypes.c_int32, [_P, _P, _P, ctypes.c_int64, _P]),
    ("hgs_downsample2x", ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    ("hgs_stream_copy", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64]),
    ("hgs_region_mse", ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.POINTER(hgs_region), _P]),
    ("hgs_lod_labels", ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.POINTER(hgs_region), ctypes.c_float, _P, _P]),
    ("hgs_set_surfaces", ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    ("hgs_render_surfaces", ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    ("hgs_slice_occupancy", ctypes.c_int32, [_P, _P, ctypes.POINTER(hgs_slice_grid), _P, _P]),
    ("hgs_disc_collision", ctypes.c_int32, [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_double, _P]),
    ("hgs_render_backward", ctypes.c_int32, [_P, _P, _P, _P]),
    ("hgs_navigable_map", ctypes.c_int32, [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P]),
    ("hgs_distance_fields", ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                             ctypes.POINTER(ctypes.c_int64)]),
    ("hgs_trace_paths", ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                         ctypes.c_int64, _P, _P, ctypes.c_int32, _P, _P]),
]

N_MLP_PARAMS = 1377

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
        self.scene_n = int(scene.n)
        self.scene_sh_degree = int(scene.sh_degree)
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

    def set_tile_shape(self, width, height, pixels_per_thread=1):
        """Tile shape (HGS_OPT_TILE_SHAPE) and pixels per compositing thread
        (HGS_OPT_PIXELS_PER_THREAD); images do not depend on them."""
        self.set_option(HGS_OPT_PIXELS_PER_THREAD, 1)
        self.set_option(HGS_OPT_TILE_SHAPE, (int(width) << 16) | int(height))
        self.set_option(HGS_OPT_PIXELS_PER_THREAD, int(pixels_per_thread))

    def autotune(self, cache_path=None, reps=3, stream=None) -> dict:
        """Pick the fastest image-preserving launch plan for the current
        scene, views and LOD (see hgs_autotune) and keep it."""
        p = hgs_plan()
        path = None if cache_path is None else os.fspath(cache_path).encode()
        self._check(self.lib.hgs_autotune(self.ctx, self._stream(stream), path, int(reps), ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in hgs_plan._fields_}

    # ------------------------------------------------------------ learned LOD
    def _stream(self, stream):
        import torch
        return ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)

    def set_keep_nodes(self, nodes):
        a = _np(nodes, np.int32)
        self._check(self.lib.hgs_set_keep_nodes(self.ctx, a.size, _ptr(a)))

    def lod_candidates(self, s_hi, cap=1 << 20, stream=None):
        """(entries int32[n,2] (node, view), features f32[n,8], rects int32[n,4]) as
        device tensors for the current cameras (threshold cut)."""
        import torch
        dev = torch.device("cuda", self.device)
        while True:
            ent = torch.empty((cap, 2), dtype=torch.int32, device=dev)
            feat = torch.empty((cap, 8), dtype=torch.float32, device=dev)
            rect = torch.empty((cap, 4), dtype=torch.int32, device=dev)
            n = ctypes.c_int64()
            st = self.lib.hgs_lod_candidates(self.ctx, self._stream(stream), float(s_hi), ent.data_ptr(),
                                             feat.data_ptr(), rect.data_ptr(), cap, ctypes.byref(n))
            if st == HGS_E_CAPACITY and n.value > cap:
                cap = int(n.value * 1.1) + 1024
                continue
            self._check(st)
            return ent[:n.value], feat[:n.value], rect[:n.value]

    def load_lod_mlp(self, bf16_params, mean, std, p_star, s_hi):
        w = _np(bf16_params, np.uint16); m = _np(mean, np.float32); sd = _np(std, np.float32)
        assert w.size == N_MLP_PARAMS and m.size == 8 and sd.size == 8
        self._check(self.lib.hgs_load_lod_mlp(self.ctx, _ptr(w), _ptr(m), _ptr(sd), float(p_star), float(s_hi)))

    def mlp_forward(self, feats, w, mean, std, stream=None):
        import torch
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        m = _np(mean, np.float32); sd = _np(std, np.float32)
        self._check(self.lib.hgs_mlp_forward(self.ctx, self._stream(stream), feats.data_ptr(), feats.shape[0],
                                             w.data_ptr(), _ptr(m), _ptr(sd), out.data_ptr()))
        return out

    def mlp_train_step(self, feats, labels, mean, std, master, w, m, v, step, lr, grad_out=None, loss_out=None,
                       stream=None):
        mm = _np(mean, np.float32); sd = _np(std, np.float32)
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        self._check(self.lib.hgs_mlp_train_step(self.ctx, self._stream(stream), feats.data_ptr(), labels.data_ptr(),
                                                feats.shape[0], _ptr(mm), _ptr(sd), ptr(master), w.data_ptr(),
                                                ptr(m), ptr(v), int(step), float(lr), ptr(grad_out), ptr(loss_out)))

    def mlp_backward(self, feats, labels, mean, std, w, grad_out, loss_out=None, stream=None):
        mm = _np(mean, np.float32); sd = _np(std, np.float32)
        self._check(self.lib.hgs_mlp_backward(self.ctx, self._stream(stream), feats.data_ptr(), labels.data_ptr(),
                                              feats.shape[0], _ptr(mm), _ptr(sd), w.data_ptr(), grad_out.data_ptr(),
                                              loss_out.data_ptr() if loss_out is not None else None))

    def mlp_adam(self, grad, master, w, m, v, step, lr, stream=None):
        self._check(self.lib.hgs_mlp_adam(self.ctx, self._stream(stream), grad.data_ptr(), master.data_ptr(),
                                          w.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr)))

    def mlp_bf16_from_master(self, master, w, stream=None):
        self._check(self.lib.hgs_mlp_bf16_from_master(self.ctx, self._stream(stream), master.data_ptr(), w.data_ptr()))

    def feature_stats(self, feats, stream=None):
        import torch
        out = torch.empty(16, dtype=torch.float32, device=feats.device)
        self._check(self.lib.hgs_feature_stats(self.ctx, self._stream(stream), feats.data_ptr(), feats.shape[0],
                                               out.data_ptr()))
        return out

    def stream_copy(self, src, dst, stream=None):
        """dst <- src (device tensors of the same byte size, a multiple of
        16), asynchronous: the HBM bandwidth probe."""
        n = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != n:
            raise ValueError("src and dst differ in size")
        self._check(self.lib.hgs_stream_copy(self.ctx, self._stream(stream), src.data_ptr(), dst.data_ptr(), n))

    def downsample2x(self, src, stream=None):
        import torch
        _, H2, W2 = src.shape
        dst = torch.empty((3, H2 // 2, W2 // 2), dtype=torch.float32, device=src.device)
        self._check(self.lib.hgs_downsample2x(self.ctx, self._stream(stream), src.data_ptr(), W2 // 2, H2 // 2,
                                              dst.data_ptr()))
        return dst

    def region_mse(self, regions, out, stream=None):
        """regions: list of (img tensor [3,h,w], ref tensor [3,H,W], x0, y0)."""
        arr = (hgs_region * len(regions))()
        for i, (img, ref, x0, y0) in enumerate(regions):
            arr[i] = hgs_region(img.data_ptr(), ref.data_ptr(), img.shape[2], img.shape[1], ref.shape[2],
                                ref.shape[1], int(x0), int(y0))
        self._check(self.lib.hgs_region_mse(self.ctx, self._stream(stream), len(regions), arr, out.data_ptr()))
        return out

    def lod_labels(self, pairs, label_db, stream=None):
        """pairs: list of (refined img, kept img, ref, x0, y0) windows of
        candidates; returns device float tensors (labels, drop_db)."""
        import torch
        n = len(pairs)
        arr = (hgs_region * (2 * n))()
        for i, (a, b, ref, x0, y0) in enumerate(pairs):
            for k, img in enumerate((a, b)):
                arr[2 * i + k] = hgs_region(img.data_ptr(), ref.data_ptr(), img.shape[2], img.shape[1], ref.shape[2],
                                            ref.shape[1], int(x0), int(y0))
        dev = pairs[0][2].device if n else torch.device("cuda", self.device)
        labels = torch.empty(n, dtype=torch.float32, device=dev)
        drop = torch.empty(n, dtype=torch.float32, device=dev)
        self._check(self.lib.hgs_lod_labels(self.ctx, self._stream(stream), n, arr, float(label_db), labels.data_ptr(),
                                            drop.data_ptr()))
        return labels, drop

    # ------------------------------------------------------------ ground truth
    def set_surfaces(self, surfaces):
        """surfaces: numpy records of synth.SURFACE_DTYPE."""
        a = np.ascontiguousarray(surfaces)
        assert a.dtype.itemsize == 64
        self._check(self.lib.hgs_set_surfaces(self.ctx, a.size, a.ctypes.data_as(ctypes.c_void_p)))

    def render_surfaces(self, view, ss=3, out=None, stream=None):
        import torch
        c = self.cams[view]
        if out is None:
            out = torch.empty((3, c.height, c.width), dtype=torch.float32, device=torch.device("cuda", self.device))
        self._check(self.lib.hgs_render_surfaces(self.ctx, self._stream(stream), int(view), int(ss), out.data_ptr()))
        return out

    def slice_occupancy(self, x0, y0, cell, nx, ny, heights, rho_min=0.5, occ=True, stream=None):
        """GS-slice occupancy of the scene's leaves on planes at `heights`:
        (occ uint8 [n_planes, ny, nx] or None, map uint8 [ny, nx])."""
        import torch
        h = np.ascontiguousarray(np.asarray(heights, np.float32).ravel())
        dev = torch.device("cuda", self.device)
        o = torch.empty((h.size, ny, nx), dtype=torch.uint8, device=dev) if occ else None
        m = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
        g = hgs_slice_grid(float(x0), float(y0), float(cell), int(nx), int(ny), h.size, float(rho_min),
                           h.ctypes.data_as(ctypes.c_void_p))
        self._check(self.lib.hgs_slice_occupancy(self.ctx, self._stream(stream), ctypes.byref(g),
                                                 o.data_ptr() if o is not None else None, m.data_ptr()))
        return o, m

    def disc_collision(self, occ_map, x0, y0, cell, xy, radius, stream=None):
        """Flags (uint8 [n]) of discs of `radius` at xy (device float64 [n, 2])
        that meet an occupied cell of occ_map (device uint8 [ny, nx])."""
        import torch
        ny, nx = occ_map.shape
        n = xy.shape[0]
        out = torch.empty(n, dtype=torch.uint8, device=xy.device)
        self._check(self.lib.hgs_disc_collision(self.ctx, self._stream(stream), occ_map.data_ptr(), float(x0), float(y0),
                                                float(cell), int(nx), int(ny), int(n), xy.data_ptr(), float(radius),
                                                out.data_ptr()))
        return out

    def backward(self, grads, out=None, stream=None):
        """Backward pass of the last render.  grads: per view (d_rgb [3,H,W],
        d_depth [H,W], d_alpha [H,W]) float32 CUDA tensors or None.  Returns
        the dict of parameter gradients (means, scales, quats, opacity, sh
        [n, K, 3]), added to `out` when given, else to zeros."""
        import torch
        dev = torch.device("cuda", self.device)
        n, K = self.scene_n, (self.scene_sh_degree + 1) ** 2
        if out is None:
            out = {"means": torch.zeros((n, 3), dtype=torch.float32, device=dev),
                   "scales": torch.zeros((n, 3), dtype=torch.float32, device=dev),
                   "quats": torch.zeros((n, 4), dtype=torch.float32, device=dev),
                   "opacity": torch.zeros(n, dtype=torch.float32, device=dev),
                   "sh": torch.zeros((n, K, 3), dtype=torch.float32, device=dev)}
        if len(grads) != len(self.cams):
            raise ValueError("one gradient triple per view")
        arr = (hgs_image_grad * len(grads))()
        for i, g in enumerate(grads):
            c = self.cams[i]
            shapes = ((3, c.height, c.width), (c.height, c.width), (c.height, c.width))
            ptrs = []
            for t, shp in zip(g, shapes):
                if t is None:
                    ptrs.append(None)
                    continue
                if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shp):
                    raise ValueError(f"image gradients of view {i} must be contiguous float32 CUDA tensors {shp}")
                ptrs.append(t.data_ptr())
            arr[i] = hgs_image_grad(*ptrs)
        for k, t in out.items():
            self._dev(t, torch.float32, k)
        sg = hgs_scene_grad(out["means"].data_ptr(), out["scales"].data_ptr(), out["quats"].data_ptr(),
                            out["opacity"].data_ptr(), out["sh"].data_ptr())
        self._check(self.lib.hgs_render_backward(self.ctx, self._stream(stream), arr, ctypes.byref(sg)))
        return out

    # ------------------------------------------------------------ planning
    @staticmethod
    def _dev(t, dtype, name):
        import torch
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
        return t

    def navigable_map(self, occ_map, x0, y0, cell, radius, stream=None):
        """uint8 [ny, nx]: 1 where a disc robot of `radius` centred on the
        cell meets no occupied cell of occ_map (device uint8 [ny, nx])."""
        import torch
        self._dev(occ_map, torch.uint8, "occ_map")
        ny, nx = occ_map.shape
        nav = torch.empty_like(occ_map)
        self._check(self.lib.hgs_navigable_map(self.ctx, self._stream(stream), occ_map.data_ptr(), float(x0),
                                               float(y0), float(cell), int(nx), int(ny), float(radius),
                                               nav.data_ptr()))
        return nav

    def distance_fields(self, nav, goals, dist=None, stream=None):
        """Distance fields to the goal cells (indices j*nx + i): (int64
        tensor [n_goals, ny, nx] holding the uint64 pairs a | b << 32, -1
        unreachable; relaxation rounds).  Blocks until complete."""
        import torch
        self._dev(nav, torch.uint8, "nav")
        ny, nx = nav.shape
        g = np.ascontiguousarray(np.asarray(goals, np.int32).ravel())
        if dist is None:
            dist = torch.empty((g.size, ny, nx), dtype=torch.int64, device=nav.device)
        self._dev(dist, torch.int64, "dist")
        if dist.numel() < g.size * ny * nx:
            raise ValueError("dist is too small")
        rounds = ctypes.c_int64()
        self._check(self.lib.hgs_distance_fields(self.ctx, self._stream(stream), nav.data_ptr(), int(nx), int(ny),
                                                 g.size, g.ctypes.data_as(ctypes.c_void_p), dist.data_ptr(),
                                                 ctypes.byref(rounds)))
        return dist, rounds.value

    def trace_paths(self, nav, dist, starts, slots, cap, stream=None):
        """Trajectories (int32 [n, cap] cell indices, int32 [n] lengths) from
        device int32 start cells down fields dist[slots]."""
        import torch
        self._dev(nav, torch.uint8, "nav")
        self._dev(dist, torch.int64, "dist")
        self._dev(starts, torch.int32, "starts")
        self._dev(slots, torch.int32, "slots")
        ny, nx = nav.shape
        n = starts.numel()
        if slots.numel() != n:
            raise ValueError("starts and slots differ in length")
        paths = torch.empty((n, max(int(cap), 1)), dtype=torch.int32, device=nav.device)
        lens = torch.empty(n, dtype=torch.int32, device=nav.device)
        self._check(self.lib.hgs_trace_paths(self.ctx, self._stream(stream), nav.data_ptr(), int(nx), int(ny),
                                             dist.data_ptr(), int(dist.shape[0]), int(n), starts.data_ptr(),
                                             slots.data_ptr(), int(cap), paths.data_ptr(), lens.data_ptr()))
        return paths[:, :cap], lens

    def sort_pairs_noalloc(self, keys, vals, key_bits, stream=None):
        """Sort device uint32 tensors (as int32 storage) in place in the
        library's static scratch area (no allocation; asynchronous)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hgs_sort_pairs_noalloc(self.ctx, ctypes.c_void_p(stream.cuda_stream), keys.data_ptr(),
                                                    vals.data_ptr(), keys.numel(), int(key_bits)))

    def sort_pairs(self, keys, vals, key_bits, stream=None):
        """Sort device uint32 tensors (as int32 storage) in place."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hgs_sort_pairs(self.ctx, ctypes.c_void_p(stream.cuda_stream), keys.data_ptr(),
                                            vals.data_ptr(), keys.numel(), int(key_bits)))
