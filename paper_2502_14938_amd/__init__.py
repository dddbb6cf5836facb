"""Python binding of libgscache.so (include/gscache.h): argument marshalling
only.  Every step of the hot path runs in the library's HIP kernels; PyTorch
supplies device memory and the stream.  There is no CPU fallback: if the
library is missing the import of this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgscache.so")

GSC_OK = 0
GSC_E_INVALID_ARG, GSC_E_NOT_LOADED, GSC_E_OOM, GSC_E_CAPACITY, GSC_E_BUDGET, GSC_E_HIP = -1, -2, -3, -4, -5, -6
GSC_E_UNCHANGED, GSC_E_TIMEOUT, GSC_E_EXPIRED = -7, -8, -9
ERRORS = {-1: "GSC_E_INVALID_ARG", -2: "GSC_E_NOT_LOADED", -3: "GSC_E_OOM", -4: "GSC_E_CAPACITY",
          -5: "GSC_E_BUDGET", -6: "GSC_E_HIP", -7: "GSC_E_UNCHANGED", -8: "GSC_E_TIMEOUT", -9: "GSC_E_EXPIRED"}
PREC = {"f32": 0, "bf16": 1, "fp8": 2}
FLAG_DEREDUNDANCY, FLAG_REUSE, FLAG_PREDICTOR, FLAG_FULL_KEY_SORT, FLAG_LOD_FADE = 1, 2, 4, 8, 16
GUIDE = {"linear": 0, "fixed": 1, "exp": 2, "staged": 3}
DBG = {"visible": 0, "misses": 1, "gauss": 2, "derived": 3, "pairs": 4, "ranges": 5, "preproc": 6, "depth": 7,
       "sort_keys": 8, "raw_ranges": 9, "sort_vals": 10}
PRED_NPARAMS = 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1  # 4673


class GscError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Config(C.Structure):
    _fields_ = [("k", C.c_int32), ("feat_dim", C.c_int32), ("hidden", C.c_int32), ("d_max", C.c_int32),
                ("guide", C.c_int32), ("precision", C.c_int32), ("flags", C.c_uint32),
                ("predictor_threshold", C.c_float), ("cache_capacity", C.c_int64), ("max_width", C.c_int32),
                ("max_height", C.c_int32), ("max_pairs", C.c_int64)]


class Camera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("pos", C.c_double * 3), ("fovx", C.c_double), ("fovy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_double)]


class Anchors(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("level", C.c_void_p), ("radius", C.c_void_p),
                ("feat", C.c_void_p), ("scale", C.c_void_p), ("offsets", C.c_void_p), ("d_ref", C.c_double),
                ("is_device", C.c_int32), ("dist_unit", C.c_double)]


class Mlp(C.Structure):
    _fields_ = [("W1", C.c_void_p * 3), ("b1", C.c_void_p * 3), ("W2", C.c_void_p * 3), ("b2", C.c_void_p * 3)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("mu", C.c_void_p), ("cov", C.c_void_p), ("rgb", C.c_void_p),
                ("alpha", C.c_void_p)]


class FrameStats(C.Structure):
    _fields_ = [("frame", C.c_int64), ("n_visible", C.c_int64), ("n_miss", C.c_int64), ("n_gauss", C.c_int64),
                ("n_pairs", C.c_int64 * 2), ("n_evicted", C.c_int64), ("depth_used", C.c_int32),
                ("depth_next", C.c_int32), ("overflow", C.c_int32), ("pad", C.c_int32),
                ("device_bytes", C.c_int64), ("n_eval", C.c_int64 * 2),
                ("n_contrib", C.c_int64 * 2), ("n_tall", C.c_int64)]

    def as_dict(self):
        return {"frame": self.frame, "n_visible": self.n_visible, "n_miss": self.n_miss, "n_gauss": self.n_gauss,
                "n_pairs": [self.n_pairs[0], self.n_pairs[1]], "n_evicted": self.n_evicted,
                "depth_used": self.depth_used, "depth_next": self.depth_next, "overflow": self.overflow,
                "device_bytes": self.device_bytes, "n_eval": [self.n_eval[0], self.n_eval[1]],
                "n_contrib": [self.n_contrib[0], self.n_contrib[1]], "n_tall": self.n_tall}


_lib = None

SYMBOLS = {
    "gsc_create": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "gsc_destroy": ([C.c_void_p], None),
    "gsc_last_error": ([C.c_void_p], C.c_char_p),
    "gsc_set_stream": ([C.c_void_p, C.c_void_p], C.c_int),
    "gsc_load_anchors": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "gsc_set_camera_pair": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_double], C.c_int),
    "gsc_derive": ([C.c_void_p], C.c_int),
    "gsc_render_stereo": ([C.c_void_p] * 5, C.c_int),
    "gsc_render_gaussians": ([C.c_void_p] * 6, C.c_int),
    "gsc_render_gaussians_noalloc": ([C.c_void_p] * 6, C.c_int),
    "gsc_sync": ([C.c_void_p], C.c_int),
    "gsc_get_stats": ([C.c_void_p, C.c_void_p], C.c_int),
    "gsc_reset_cache": ([C.c_void_p], C.c_int),
    "gsc_debug_copy": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "gsc_predictor_load": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "gsc_predictor_get": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "gsc_predictor_train": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_float,
                             C.c_float, C.c_uint64, C.c_void_p], C.c_int),
    "gsc_predictor_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p],
                           C.c_int),
    "gsc_predictor_infer": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "gsc_predictor_collect": ([C.c_void_p, C.c_int], C.c_int),
    "gsc_predictor_labels": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "gsc_server_create": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "gsc_server_destroy": ([C.c_void_p], None),
    "gsc_server_admit": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int),
    "gsc_server_viewer_bytes": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int64),
    "gsc_server_submit": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p],
                          C.c_int64),
    "gsc_server_step": ([C.c_void_p], C.c_int),
    "gsc_server_poll": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "gsc_server_pending": ([C.c_void_p], C.c_int),
    "gsc_server_policy": ([C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int], C.c_int),
    "gsc_server_overlap": ([C.c_void_p, C.c_int], C.c_int),
    "gsc_timing": ([C.c_void_p, C.c_int], C.c_int),
    "gsc_timing_stages": ([C.c_void_p, C.c_uint32], C.c_int),
    "gsc_count_work": ([C.c_void_p, C.c_int], C.c_int),
    "gsc_pipeline": ([C.c_void_p, C.c_int], C.c_int),
    "gsc_ssim": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p], C.c_int),
    "gsc_timing_read": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "gsc_server_last_error": ([C.c_void_p], C.c_char_p),
    "gsc_server_leave": ([C.c_void_p, C.c_int32], C.c_int),
}


def lib():
    """Load libgscache.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgscache.so not built: run python -c 'import __graft_entry__ as g; g.build()' "
                              "or python paper_2502_14938_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


NOALLOC_MAX_GAUSSIANS, NOALLOC_MAX_PAIRS, NOALLOC_MAX_SIDE = 65536, 1 << 21, 2048


def render_gaussians_noalloc(mu, cov, rgb, alpha, cam: dict, out, T=None, status=None, stream=None):
    """gsc_render_gaussians_noalloc: the raster-only render of explicit
    Gaussians on the library's static device buffer (no allocation, no
    context); `status` (int32 device tensor, optional) receives the overflow
    bits.  Asynchronous on `stream` (default: torch's current stream)."""
    g = Gaussians()
    g.n = int(alpha.shape[0])
    for t in (mu, cov, rgb, alpha):
        assert t.is_cuda and t.is_contiguous() and t.dtype.itemsize == 4
    g.mu, g.cov, g.rgb, g.alpha = mu.data_ptr(), cov.data_ptr(), rgb.data_ptr(), alpha.data_ptr()
    c = camera(cam)
    st = stream if stream is not None else _current_stream()
    L = lib()
    rc = L.gsc_render_gaussians_noalloc(C.byref(g), C.byref(c), _ptr(out), _ptr(T), _ptr(status), st)
    if rc != GSC_OK:
        raise GscError(rc, (L.gsc_last_error(None) or b"").decode())


def camera(cam: dict) -> Camera:
    c = Camera()
    R = np.asarray(cam["R"], np.float64).reshape(9)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.pos[i] = float(cam["pos"][i])
    c.fovx, c.fovy = float(cam["fovx"]), float(cam["fovy"])
    c.width, c.height, c.znear = int(cam["width"]), int(cam["height"]), float(cam["znear"])
    return c


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


STAGES = ("schedule", "derive", "compose", "preprocess", "tall_spans", "depth_sort", "pair_scan", "dup_rows",
          "tall_list", "dup_big", "tile_sort", "ranges", "blend")


class Renderer:
    """One viewer's renderer: a gsc_ctx with its own cache on the current device."""

    def __init__(self, k=10, d_max=10, guide="linear", precision="f32", reuse=False, deredundancy=True,
                 predictor=False, full_key_sort=False, max_width=2048, max_height=1080, cache_capacity=0,
                 max_pairs=0, predictor_threshold=0.5, lod_fade=False, stream=None):
        L = lib()
        cfg = Config()
        cfg.k, cfg.feat_dim, cfg.hidden, cfg.d_max = k, 32, 32, d_max
        cfg.guide, cfg.precision = GUIDE[guide], PREC[precision]
        cfg.flags = ((FLAG_DEREDUNDANCY if deredundancy else 0) | (FLAG_REUSE if reuse else 0) |
                     (FLAG_PREDICTOR if predictor else 0) | (FLAG_FULL_KEY_SORT if full_key_sort else 0) |
                     (FLAG_LOD_FADE if lod_fade else 0))
        cfg.predictor_threshold = predictor_threshold
        cfg.cache_capacity, cfg.max_width, cfg.max_height, cfg.max_pairs = cache_capacity, max_width, max_height, max_pairs
        self.cfg = cfg
        h = C.c_void_p()
        st = stream if stream is not None else _current_stream()
        self._check(L.gsc_create(C.byref(cfg), st, C.byref(h)), None)
        self.h = h
        self._keep = []

    def _check(self, rc, h=-1):
        if rc != GSC_OK and rc is not None and rc < 0:
            L = lib()
            msg = L.gsc_last_error(self.h if h == -1 else h)
            raise GscError(rc, (msg or b"").decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().gsc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        self._check(lib().gsc_set_stream(self.h, stream if stream is not None else _current_stream()))

    def load(self, scene):
        """Copy a synth.Scene (host arrays) into the library."""
        arrs = [np.ascontiguousarray(scene.pos, np.float32), np.ascontiguousarray(scene.level, np.uint8),
                np.ascontiguousarray(scene.radius, np.float32), np.ascontiguousarray(scene.feat, np.float32),
                np.ascontiguousarray(scene.scale, np.float32), np.ascontiguousarray(scene.offsets, np.float32)]
        a = Anchors()
        a.n = scene.n
        a.pos, a.level, a.radius, a.feat, a.scale, a.offsets = [x.ctypes.data for x in arrs]
        a.d_ref = float(min(scene.d_ref, 1e30))
        a.is_device = 0
        # a distance input: layer 1 has F + 4 columns and the scene its unit
        n_in = np.asarray(scene.mlp["alpha"][0]).shape[1]
        a.dist_unit = float(getattr(scene, "dist_unit", 0.0)) if n_in == scene.F + 4 else 0.0
        m = Mlp()
        keep = []
        for h, name in enumerate(("alpha", "color", "cov")):
            W1, b1, W2, b2 = [np.ascontiguousarray(x, np.float32) for x in scene.mlp[name]]
            keep += [W1, b1, W2, b2]
            m.W1[h], m.b1[h], m.W2[h], m.b2[h] = W1.ctypes.data, b1.ctypes.data, W2.ctypes.data, b2.ctypes.data
        self._check(lib().gsc_load_anchors(self.h, C.byref(a), C.byref(m)))

    def set_camera_pair(self, left: dict, right: dict, t_arrival: float = 0.0):
        l, r = camera(left), camera(right)
        self._check(lib().gsc_set_camera_pair(self.h, C.byref(l), C.byref(r), float(t_arrival)))

    def derive(self):
        self._check(lib().gsc_derive(self.h))

    def render_stereo(self, out_left, out_right, T_left=None, T_right=None):
        for t in (out_left, out_right, T_left, T_right):
            if t is not None:
                assert t.is_cuda and t.is_contiguous() and t.dtype.itemsize == 4
        self._check(lib().gsc_render_stereo(self.h, _ptr(out_left), _ptr(out_right), _ptr(T_left), _ptr(T_right)))

    def frame(self, left, right, out_left, out_right, T_left=None, T_right=None, t_arrival=0.0):
        self.set_camera_pair(left, right, t_arrival)
        self.derive()
        self.render_stereo(out_left, out_right, T_left, T_right)

    def render_gaussians(self, mu, cov, rgb, alpha, cam: dict, out, T=None, n_contrib=None):
        g = Gaussians()
        g.n = int(alpha.shape[0])
        for t in (mu, cov, rgb, alpha):
            assert t.is_cuda and t.is_contiguous() and t.dtype.itemsize == 4
        g.mu, g.cov, g.rgb, g.alpha = mu.data_ptr(), cov.data_ptr(), rgb.data_ptr(), alpha.data_ptr()
        c = camera(cam)
        self._check(lib().gsc_render_gaussians(self.h, C.byref(g), C.byref(c), _ptr(out), _ptr(T), _ptr(n_contrib)))

    def sync(self):
        return self._check(lib().gsc_sync(self.h))

    def stats(self) -> dict:
        s = FrameStats()
        self._check(lib().gsc_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def reset_cache(self):
        self._check(lib().gsc_reset_cache(self.h))

    def debug(self, what: str, eye: int = 0):
        """Synchronous copy of an internal list for parity tests."""
        L = lib()
        code = DBG[what]
        n = C.c_int64()
        self._check(L.gsc_debug_copy(self.h, code, eye, None, 0, C.byref(n)))
        cnt = n.value
        shape, dt = {"visible": ((cnt,), np.int32), "misses": ((cnt,), np.int32), "gauss": ((cnt,), np.int32),
                     "derived": ((cnt, 13), np.float32), "pairs": ((cnt, 2), np.int32),
                     "ranges": ((cnt, 2), np.int32), "preproc": ((cnt, 8), np.float32),
                     "depth": ((cnt,), np.int32), "sort_keys": ((cnt,), np.uint32),
                     "raw_ranges": ((cnt, 2), np.int32), "sort_vals": ((cnt,), np.uint32)}[what]
        out = np.zeros(shape, dt)
        if cnt:
            self._check(L.gsc_debug_copy(self.h, code, eye, out.ctypes.data, cnt, C.byref(n)))
        return out

    # ---------------------------------------------------------- predictor
    def count_work(self, enable=True):
        """Let the blend count its visits and contributions (stats n_eval, n_contrib)."""
        self._check(lib().gsc_count_work(self.h, 1 if enable else 0))

    def pipeline(self, enable=True):
        """Two frames in flight: each frame's blend overlaps the next frame's
        stages up to its tile ranges.  A frame's images are complete only
        after sync() (or a later call that waits, such as stats())."""
        self._check(lib().gsc_pipeline(self.h, 1 if enable else 0))

    def ssim(self, a, b) -> float:
        """Mean SSIM of two device float32 [C, H, W] images (H, W >= 11)."""
        assert a.is_cuda and b.is_cuda and a.shape == b.shape and a.dim() == 3
        assert a.dtype == b.dtype and a.dtype.itemsize == 4 and a.is_contiguous() and b.is_contiguous()
        out = C.c_double()
        self._check(lib().gsc_ssim(self.h, _ptr(a), _ptr(b), int(a.shape[0]), int(a.shape[1]), int(a.shape[2]),
                                   C.byref(out)))
        return out.value

    def timing(self, enable=True, stages=None):
        """Record device time of every frame from now on (or stop): the frame
        and each stage in `stages` (names from STAGES; None: all)."""
        mask = 0xFFFFFFFF if stages is None else sum(1 << STAGES.index(x) for x in stages)
        self._check(lib().gsc_timing_stages(self.h, mask))
        self._check(lib().gsc_timing(self.h, 1 if enable else 0))

    def timing_read(self, max_frames=4096):
        """(summed device ms per stage, per-frame device ms, frames recorded)
        since timing was switched on or last read."""
        ms = np.zeros(len(STAGES), np.float64)
        fr = np.zeros(max_frames, np.float64)
        n = C.c_int64()
        self._check(lib().gsc_timing_read(self.h, ms.ctypes.data, len(STAGES), fr.ctypes.data, max_frames,
                                          C.byref(n)))
        return dict(zip(STAGES, ms.tolist())), fr[:min(n.value, max_frames)], n.value

    def predictor_load(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == PRED_NPARAMS
        self._check(lib().gsc_predictor_load(self.h, p.ctypes.data, p.size))

    def predictor_get(self) -> np.ndarray:
        p = np.zeros(PRED_NPARAMS, np.float32)
        self._check(lib().gsc_predictor_get(self.h, p.ctypes.data, p.size))
        return p

    def predictor_train(self, X, y, batch=1024, epochs=20, lr=1e-3, pos_weight=1.0, seed=0):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.uint8)
        losses = np.zeros(epochs, np.float32)
        self._check(lib().gsc_predictor_train(self.h, X.ctypes.data, y.ctypes.data, len(y), batch, epochs, lr,
                                              pos_weight, seed, losses.ctypes.data))
        return losses

    def predictor_grad(self, X_dev, y_dev, pos_weight=1.0):
        g = np.zeros(PRED_NPARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        self._check(lib().gsc_predictor_grad(self.h, _ptr(X_dev), _ptr(y_dev), int(X_dev.shape[0]), pos_weight,
                                             g.ctypes.data, loss.ctypes.data))
        return float(loss[0]), g

    def predictor_infer(self, X_dev, p_dev):
        self._check(lib().gsc_predictor_infer(self.h, _ptr(X_dev), int(X_dev.shape[0]), _ptr(p_dev)))

    def predictor_collect(self, enable=True):
        self._check(lib().gsc_predictor_collect(self.h, 1 if enable else 0))

    def predictor_labels(self, with_ids=False):
        """Features and labels of the last frame's reuse candidates (numpy)."""
        n = C.c_int64()
        self._check(lib().gsc_predictor_labels(self.h, None, None, None, 0, C.byref(n)))
        X = np.zeros((n.value, 6), np.float32)
        y = np.zeros(n.value, np.uint8)
        ids = np.zeros(n.value, np.int32)
        if n.value:
            self._check(lib().gsc_predictor_labels(self.h, X.ctypes.data, y.ctypes.data, ids.ctypes.data, n.value,
                                                   C.byref(n)))
        return (X, y, ids) if with_ids else (X, y)


def pack_params(params) -> np.ndarray:
    """Flatten [W1, b1, W2, b2, W3, b3] (numpy) in the library's order."""
    return np.concatenate([np.asarray(p, np.float32).reshape(-1) for p in params])


def unpack_params(flat) -> list:
    flat = np.asarray(flat)
    shapes = [(64, 6), (64,), (64, 64), (64,), (1, 64), (1,)]
    out, o = [], 0
    for s in shapes:
        m = int(np.prod(s))
        out.append(flat[o:o + m].reshape(s))
        o += m
    return out


class Server:
    """Continuous-batching server over the scene of a loaded Renderer
    (gsc_server_*): viewers with their own device caches, admitted against a
    device-memory budget; frame requests batched across viewers."""

    def __init__(self, renderer: Renderer, budget_bytes: int, stream=None):
        h = C.c_void_p()
        st = stream if stream is not None else _current_stream()
        rc = lib().gsc_server_create(renderer.h, int(budget_bytes), st, C.byref(h))
        if rc != GSC_OK:
            raise GscError(rc, "gsc_server_create failed (scene loaded with de-redundancy? predictor loaded?)")
        self.h = h
        self.renderer = renderer  # keeps the scene alive
        self._outs = {}

    def _check(self, rc):
        if rc is not None and rc < 0:
            raise GscError(rc, (lib().gsc_server_last_error(self.h) or b"").decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().gsc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def viewer_bytes(self, width, height) -> int:
        return self._check(lib().gsc_server_viewer_bytes(self.h, width, height))

    def admit(self, width, height):
        """Viewer id, or None when the budget does not allow it now."""
        rc = lib().gsc_server_admit(self.h, width, height)
        if rc == GSC_E_BUDGET:
            return None
        return self._check(rc)

    def submit(self, viewer, left: dict, right: dict, t_arrival, out_left, out_right):
        """Request id, or None when the queue policy's pose gate did not queue it."""
        l, r = camera(left), camera(right)
        rc = lib().gsc_server_submit(self.h, viewer, C.byref(l), C.byref(r), float(t_arrival),
                                     _ptr(out_left), _ptr(out_right))
        if rc == GSC_E_UNCHANGED:
            return None
        rid = self._check(rc)
        self._outs[rid] = (out_left, out_right)  # keep the buffers alive until completion
        return rid

    def policy(self, pose_m=0.0, pose_rad=0.0, timeout_s=0.0, ordered=False):
        """Queue policy (each part off at <= 0): pose gate, timeout on the
        host monotonic clock (time.monotonic()), display order."""
        self._check(lib().gsc_server_policy(self.h, float(pose_m), float(pose_rad), float(timeout_s),
                                            1 if ordered else 0))

    def overlap(self, enable=True):
        """Two batches in flight: each batch's blend overlaps the next batch's
        earlier stages (call before admitting viewers)."""
        self._check(lib().gsc_server_overlap(self.h, 1 if enable else 0))

    def step(self) -> int:
        return self._check(lib().gsc_server_step(self.h))

    def poll(self, cap=256):
        """[(request id, completion time, status)] finished since the last poll."""
        ids = np.zeros(cap, np.int64)
        t = np.zeros(cap, np.float64)
        stt = np.zeros(cap, np.int32)
        n = self._check(lib().gsc_server_poll(self.h, ids.ctypes.data, t.ctypes.data, stt.ctypes.data, cap))
        out = []
        for i in range(n):
            self._outs.pop(int(ids[i]), None)
            out.append((int(ids[i]), float(t[i]), int(stt[i])))
        return out

    def pending(self) -> int:
        return self._check(lib().gsc_server_pending(self.h))

    def leave(self, viewer):
        self._check(lib().gsc_server_leave(self.h, viewer))
