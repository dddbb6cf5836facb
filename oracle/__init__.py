"""FP64 CPU oracle for the GS-Cache per-frame hot path (arXiv 2502.14938).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the GPU path.  The float math lives in gsc_oracle.c
(plain C, double precision); this module marshals arrays and adds the parts
that are integer bookkeeping (compose, the derived-Gaussian cache, depth
scheduling) or tiny dense maths (the reuse predictor), in NumPy float64.

Section references are to the paper: Section 3.1 (eqs. 1-3, structured
derivation), Section 4 (cache design, Alg. 1 dynamic cache depth, eq. 4
guiding function, eqs. 5-6 binocular de-redundancy), Section 6
(AnchorDecoder / RasterizeGaussians optimisations).

Parity status: every function here is pinned by tests in
tests/test_oracle_*.py against closed forms, brute force, library routines
the oracle does not itself use, or invariants; see the header of each test.
"""
from __future__ import annotations

import ctypes as C
import math
import os

from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TILE = 16
MIN_ALPHA = 1.0 / 255.0
T_STOP = 1e-4


class OrcCamera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("pos", C.c_double * 3), ("fovx", C.c_double),
                ("fovy", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
                os.path.join(_HERE, "gsc_oracle.c")):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        lib.orc_threads.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_unified_camera.argtypes = [P, P, P]
        lib.orc_select.argtypes = [C.c_int64, P, P, P, P, C.c_double, C.c_int, P, P, P]
        lib.orc_select.restype = C.c_int64
        lib.orc_derive.argtypes = [C.c_int64, P, P, P, P, P, C.c_int, C.c_int, C.c_int, P, P, C.c_int,
                                   C.c_double, P, P, P, P, P]
        lib.orc_preprocess.argtypes = [C.c_int64, P, P, P, P, P, P, P, P, P, P]
        lib.orc_rect_min_q.argtypes = [C.c_double] * 9
        lib.orc_rect_min_q.restype = C.c_double
        lib.orc_tile_pairs.argtypes = [C.c_int64, P, P, P, P, P, C.c_int, C.c_int, C.c_int64, P, P, P]
        lib.orc_tile_pairs.restype = C.c_int64
        lib.orc_sort_pairs.argtypes = [C.c_int64, P, P, P, P]
        lib.orc_blend.argtypes = [C.c_int, C.c_int] + [P] * 13 + [C.c_double, P, P, P]
        lib.orc_round_bf16.argtypes = [C.c_double]
        lib.orc_round_bf16.restype = C.c_double
        lib.orc_round_e4m3.argtypes = [C.c_double]
        lib.orc_round_e4m3.restype = C.c_double
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def to_orc(cam: dict) -> OrcCamera:
    c = OrcCamera()
    R = np.asarray(cam["R"], np.float64).reshape(9)
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.pos[i] = float(cam["pos"][i])
    c.fovx, c.fovy = float(cam["fovx"]), float(cam["fovy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.znear = float(cam["znear"])
    return c


def from_orc(c: OrcCamera) -> dict:
    return {"R": np.array(c.R[:], np.float64).reshape(3, 3), "pos": np.array(c.pos[:], np.float64),
            "fovx": c.fovx, "fovy": c.fovy, "width": c.width, "height": c.height, "znear": c.znear}


def threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n host threads from now on."""
    _load().orc_set_threads(int(n))


def round_bf16(x: float) -> float:
    return _load().orc_round_bf16(float(x))


def round_e4m3(x: float) -> float:
    return _load().orc_round_e4m3(float(x))


# ---------------------------------------------------------------- stages

def unified_camera(left: dict, right: dict) -> dict:
    """Section 4, eqs. 5-6 (binocular de-redundancy)."""
    lib = _load()
    l, r, u = to_orc(left), to_orc(right), OrcCamera()
    lib.orc_unified_camera(C.byref(l), C.byref(r), C.byref(u))
    return from_orc(u)


def select(scene, ucam: dict, fade: bool = False, weights: bool = False):
    """Anchor filtering (LOD + frustum).  Returns (ids ascending int32, band
    uint8[n]), and with weights=True also the per-anchor opacity weight
    float64[n] of the fractional level transition (fade=True; all 1 without
    it)."""
    lib = _load()
    pos = _c(scene.pos, np.float32); lev = _c(scene.level, np.uint8); rad = _c(scene.radius, np.float32)
    out = np.empty(scene.n, np.int32); band = np.empty(scene.n, np.uint8)
    w = np.empty(scene.n, np.float64)
    u = to_orc(ucam)
    m = lib.orc_select(scene.n, _p(pos), _p(lev), _p(rad), C.byref(u), float(scene.d_ref), int(bool(fade)),
                       _p(out), _p(band), _p(w))
    return (out[:m].copy(), band, w) if weights else (out[:m].copy(), band)


def _mlp_ptrs(scene):
    keep = []
    arr = (C.c_void_p * 12)()
    for h, name in enumerate(("alpha", "color", "cov")):
        for i, w in enumerate(scene.mlp[name]):
            a = _c(w, np.float32)
            keep.append(a)
            arr[4 * h + i] = a.ctypes.data
    return arr, keep


def derive(scene, ids, pu, prec: int = 0) -> dict:
    """Section 3.1 eq. 3 (AnchorDecoder) for the anchors `ids` seen from p_u.
    prec: 0 exact FP64, 1 bf16 emulation, 2 e4m3fn-weight emulation.  A scene
    whose layer-1 weights have F + 4 columns takes the anchor-to-p_u distance
    over scene.dist_unit as its last input.
    Returns arrays of m*k rows: mu, cov (xx xy xz yy yz zz), rgb, alpha, alpha_pre."""
    lib = _load()
    ids = _c(ids, np.int32)
    m, k = len(ids), scene.k
    out = {"mu": np.empty((m * k, 3)), "cov": np.empty((m * k, 6)), "rgb": np.empty((m * k, 3)),
           "alpha": np.empty(m * k), "alpha_pre": np.empty(m * k)}
    arr, keep = _mlp_ptrs(scene)
    pu = _c(pu, np.float64)
    pos = _c(scene.pos, np.float32); feat = _c(scene.feat, np.float32)
    scl = _c(scene.scale, np.float32); off = _c(scene.offsets, np.float32)
    ni = scene.mlp["alpha"][0].shape[1]
    assert ni in (scene.F + 3, scene.F + 4)
    dist_unit = float(getattr(scene, "dist_unit", 0.0)) if ni == scene.F + 4 else 0.0
    assert ni == scene.F + 3 or dist_unit > 0.0, "a distance input needs scene.dist_unit > 0"
    lib.orc_derive(m, _p(ids), _p(pos), _p(feat), _p(scl), _p(off), scene.F, scene.H, k, arr, _p(pu),
                   int(prec), dist_unit, _p(out["mu"]), _p(out["cov"]), _p(out["rgb"]), _p(out["alpha"]),
                   _p(out["alpha_pre"]))
    return out


def compose(n_visible: int, k: int, alpha: np.ndarray) -> np.ndarray:
    """Alg. 1 'compose' / render buffer with the opacity mask (Section 6):
    G_t lists (visible position i, j) for i ascending, j ascending, alpha > 0.
    Returns flat row indices i*k + j into the derived arrays."""
    a = np.asarray(alpha).reshape(n_visible, k)
    ii, jj = np.nonzero(a > 0.0)
    return (ii * k + jj).astype(np.int64)


def preprocess(mu, cov, alpha, cam: dict) -> dict:
    """EWA projection (Section 3.1) per Gaussian for one eye."""
    lib = _load()
    n = len(alpha)
    mu = _c(mu, np.float64); cov = _c(cov, np.float64); alpha = _c(alpha, np.float64)
    out = {"mean2d": np.zeros((n, 2)), "conic": np.zeros((n, 3)), "sigma2d": np.zeros((n, 3)),
           "depth": np.zeros(n), "keep": np.zeros(n, np.uint8), "band": np.zeros(n, np.uint8)}
    e = to_orc(cam)
    lib.orc_preprocess(n, _p(mu), _p(cov), _p(alpha), C.byref(e), _p(out["mean2d"]), _p(out["conic"]),
                       _p(out["sigma2d"]), _p(out["depth"]), _p(out["keep"]), _p(out["band"]))
    return out


def rect_min_q(mx, my, a, b, c, x0, x1, y0, y1) -> float:
    return _load().orc_rect_min_q(mx, my, a, b, c, x0, x1, y0, y1)


def tile_pairs(pre: dict, alpha, W: int, H: int):
    """Opacity-aware exact tile lists (Section 6).  Returns (tile, g, flags) in
    emission order (g ascending, tiles row-major); flags bit0 = listed,
    bit1 = marginal.  Marginal unlisted pairs are included with bit0 = 0."""
    lib = _load()
    n = len(alpha)
    alpha = _c(alpha, np.float64)
    args = [_p(pre["mean2d"]), _p(pre["conic"]), _p(pre["sigma2d"]), _p(alpha), _p(pre["keep"])]
    need = lib.orc_tile_pairs(n, *args, W, H, 0, None, None, None)
    total = -need if need < 0 else need
    tile = np.empty(total, np.int32); g = np.empty(total, np.int32); fl = np.empty(total, np.uint8)
    got = lib.orc_tile_pairs(n, *args, W, H, total, _p(tile), _p(g), _p(fl))
    assert got == total
    return tile, g, fl


def sort_pairs(tile, g, depth) -> np.ndarray:
    """Stable order by (tile, float32(depth)) (Section 6 key-value pairs)."""
    lib = _load()
    tile = _c(tile, np.int32); g = _c(g, np.int32); depth = _c(depth, np.float64)
    order = np.empty(len(tile), np.int64)
    lib.orc_sort_pairs(len(tile), _p(tile), _p(g), _p(depth), _p(order))
    return order


def tile_ranges(sorted_tile, n_tiles: int):
    st = np.searchsorted(sorted_tile, np.arange(n_tiles), side="left").astype(np.int64)
    en = np.searchsorted(sorted_tile, np.arange(n_tiles), side="right").astype(np.int64)
    return st, en


def blend(W, H, starts, ends, sorted_g, pre, alpha, rgb, alpha_band: float = 1e-7, ghosts=None):
    """Front-to-back alpha compositing per pixel (Section 3.1).  Returns the
    image, final transmittance, contributors, ambiguity band and the number
    of Gaussians each pixel visited (up to and including the one ending it).
    ghosts: (starts, ends, g) per tile of the marginal pairs the tile test
    left out; they are never composited, only flag the pixels where they
    reach the alpha threshold."""
    lib = _load()
    npx = W * H
    img = np.zeros((3, H, W)); T = np.zeros((H, W)); nc = np.zeros((H, W), np.int32)
    band = np.zeros((H, W), np.uint8)
    ne = np.zeros((H, W), np.int32)
    sg = _c(sorted_g, np.int32); alpha = _c(alpha, np.float64); rgb = _c(rgb, np.float64)
    if ghosts is not None:
        gk = [_c(ghosts[0], np.int64), _c(ghosts[1], np.int64), _c(ghosts[2], np.int32)]
        gp = [_p(x) for x in gk]
    else:
        gp = [None, None, None]
    lib.orc_blend(W, H, _p(_c(starts, np.int64)), _p(_c(ends, np.int64)), _p(sg), _p(pre["mean2d"]),
                  _p(pre["conic"]), _p(alpha), _p(rgb), _p(pre["depth"]), _p(img), _p(T), _p(nc), _p(band), _p(ne),
                  float(alpha_band), *gp)
    return img, T, nc, band, ne


def render_gaussians(mu, cov, rgb, alpha, cam: dict, debug: bool = False, alpha_band: float = 1e-7):
    """Rasterise explicit Gaussians for one camera: preprocess -> tile lists ->
    sort -> ranges -> blend.  Returns a dict with image [3,H,W], T, n_contrib,
    pixel band, and (if debug) the intermediate lists."""
    W, H = int(cam["width"]), int(cam["height"])
    alpha = np.asarray(alpha, np.float64)
    pre = preprocess(mu, cov, alpha, cam)
    tile, g, fl = tile_pairs(pre, alpha, W, H)
    listed = (fl & 1) == 1
    lt, lg = tile[listed], g[listed]
    order = sort_pairs(lt, lg, pre["depth"])
    st_tile, st_g = lt[order], lg[order]
    ntiles = ((W + TILE - 1) // TILE) * ((H + TILE - 1) // TILE)
    s, e = tile_ranges(st_tile, ntiles)
    ghost = fl == 2                                   # marginal, left out
    go = np.argsort(tile[ghost], kind="stable")
    gt, gg = tile[ghost][go], g[ghost][go]
    gs_, ge_ = tile_ranges(gt, ntiles)
    img, T, nc, band, ne = blend(W, H, s, e, st_g, pre, alpha, np.asarray(rgb, np.float64), alpha_band,
                                 ghosts=(gs_, ge_, gg))
    out = {"image": img, "T": T, "n_contrib": nc, "band": band, "n_pairs": int(listed.sum()), "n_eval": ne}
    if debug:
        out.update(pre=pre, pairs_tile=tile, pairs_g=g, pairs_flags=fl, sorted_tile=st_tile,
                   sorted_g=st_g, starts=s, ends=e)
    return out


# ------------------------------------------------------- derived-Gaussian cache

def guide_depth(guide: str, d_max: int, nx: int, nm: int) -> int:
    """Next reuse depth from eq. 4, depth = H(|X'|/|X|), for nx > 0 visible
    anchors of which nm were decoded this frame (the update rate r = nm/nx),
    in exact rational arithmetic."""
    r = Fraction(nm, nx)
    if guide == "linear":
        d = math.floor(d_max * (1 - r) + Fraction(1, 2))  # round half up
    elif guide == "exp":
        d = d_max // 2 ** math.floor(8 * r)
    elif guide == "staged":
        d = d_max if r < Fraction(1, 8) else (d_max // 2 if r < Fraction(3, 8) else 1)
    else:
        raise ValueError(guide)
    return int(min(max(d, 1), d_max))


class CacheSim:
    """Exact integer model of the computation cache with dynamic reuse depth
    (Section 4, Alg. 1, eq. 4), per viewer.

    Readings: a line holds one anchor's k derived Gaussians and the frame tau
    at which they were derived.  At frame t with depth d_t:
      1. invalidate every line with t - tau > d_t (Alg. 1: a line older than
         the current reuse depth is no longer valid);
      2. a visible anchor hits iff it still holds a line (then 1 <= t - tau
         <= d_t) and reuse is on and the predictor does not mark it stale;
      3. misses (ascending anchor id) are re-derived with frame t's camera:
         an anchor that holds a line keeps its slot; the others take free
         slots in ascending slot order; if free slots are short, lines of
         anchors not visible now are evicted in ascending (last_used, anchor)
         order (Section 4: the scheduler picks stale lines to evict); if
         still short -> capacity error;
      4. last_used <- t for every visible anchor's line, tau <- t for misses;
      5. linear guiding function (eq. 4, update rate r = |M|/|X|):
         d_{t+1} = clamp(round_half_up(D_max (1 - r)), 1, D_max), computed
         exactly as floor((2 D_max (|X|-|M|) + |X|) / (2 |X|)); unchanged
         when |X| = 0.  d_0 = D_max.
    Other guiding functions H of eq. 4 (guide=): "fixed" keeps D_max;
    "exp" and "staged" are readings of the exponential and staged responses
    the quality evaluation (Section 7) names for accelerating and staged
    motion, without formulas: exp halves D_max once per eighth of update
    rate, d = D_max // 2**floor(8 r); staged steps from D_max (r < 1/8) to
    D_max // 2 (r < 3/8) to 1; both clamped to [1, D_max].
    """

    def __init__(self, n_anchors: int, capacity: int, d_max: int = 10, reuse: bool = True, guide: str = "linear"):
        if guide not in ("linear", "fixed", "exp", "staged"):
            raise ValueError(guide)
        self.n, self.C, self.D, self.reuse, self.guide = n_anchors, capacity, d_max, reuse, guide
        self.slot_of = np.full(n_anchors, -1, np.int64)
        self.line_anchor = np.full(capacity, -1, np.int64)
        self.tau = np.zeros(capacity, np.int64)
        self.last_used = np.zeros(capacity, np.int64)
        self.d = d_max
        self.t = 0

    def frame(self, visible: np.ndarray, stale: np.ndarray | None = None) -> dict:
        t, d = self.t, self.d
        vis = np.asarray(visible, np.int64)
        # 1. invalidate lines past the current depth
        used = self.line_anchor >= 0
        dead = used & (t - self.tau > d)
        self.slot_of[self.line_anchor[dead]] = -1
        self.line_anchor[dead] = -1
        # 2. hits
        s = self.slot_of[vis]
        has = s >= 0
        hit = has & self.reuse
        if stale is not None:
            hit &= ~np.asarray(stale, bool)
        miss_ids = vis[~hit]
        # 3. slots for misses without a line
        need = miss_ids[self.slot_of[miss_ids] < 0]
        free = np.nonzero(self.line_anchor < 0)[0]
        evicted = np.zeros(0, np.int64)
        if len(need) > len(free):
            short = len(need) - len(free)
            in_vis = np.zeros(self.n, bool)
            in_vis[vis] = True
            cand = np.nonzero((self.line_anchor >= 0) & ~in_vis[np.maximum(self.line_anchor, 0)])[0]
            if len(cand) < short:
                raise RuntimeError("cache capacity exceeded")
            order = np.lexsort((self.line_anchor[cand], self.last_used[cand]))
            ev = cand[order[:short]]
            evicted = self.line_anchor[ev].copy()
            self.slot_of[self.line_anchor[ev]] = -1
            self.line_anchor[ev] = -1
            free = np.nonzero(self.line_anchor < 0)[0]
        slots = free[:len(need)]
        self.slot_of[need] = slots
        self.line_anchor[slots] = need
        # 4. bookkeeping
        ms = self.slot_of[miss_ids]
        self.tau[ms] = t
        self.last_used[self.slot_of[vis]] = t
        # 5. depth
        nx, nm = len(vis), len(miss_ids)
        if self.guide == "fixed":
            self.d = self.D
        elif nx > 0:
            self.d = guide_depth(self.guide, self.D, nx, nm)
        self.t += 1
        return {"t": t, "d_used": d, "d_next": self.d, "hit": hit, "misses": miss_ids,
                "n_visible": nx, "n_miss": nm, "evicted": evicted, "slot": self.slot_of[vis].copy()}


# ----------------------------------------------------------- whole frame

# Pixel alpha band when opacities carry the fractional-LOD weight: the other
# side computes the weight in float32 (absolute error ~2.4e-7 over the
# octave), so a pixel alpha within 1e-6 of 1/255 is marginal.
FADE_ALPHA_BAND = 1e-6


def render_frame(scene, left: dict, right: dict, cache: CacheSim | None = None, cache_lines: dict | None = None,
                 prec: int = 0, deredundancy: bool = True, stale=None, debug: bool = False, lod_fade: bool = False):
    """One stereo frame of the cache-centric pipeline (Alg. 1 with eqs. 5-6):
    unified camera -> selection -> cache schedule -> derive misses -> compose
    -> per-eye rasterisation.  `cache_lines` maps anchor id -> derived rows
    (k rows each) and persists across frames together with `cache`.
    With deredundancy=False each eye selects and derives with its own camera
    (no cache).  lod_fade: the fractional level transition (select); each
    kept anchor's Gaussians are rasterised with opacity alpha * w_a, while
    the render buffer's mask and the cache keep the derived alpha."""
    out = {}
    if not deredundancy:
        imgs = []
        for eye in (left, right):
            ids, _ = select(scene, eye)
            der = derive(scene, ids, eye["pos"], prec)
            G = compose(len(ids), scene.k, der["alpha"])
            imgs.append(render_gaussians(der["mu"][G], der["cov"][G], der["rgb"][G], der["alpha"][G], eye))
        return {"left": imgs[0], "right": imgs[1]}
    U = unified_camera(left, right)
    ids, sel_band, lod_w = select(scene, U, fade=lod_fade, weights=True)
    k = scene.k
    if cache is None:
        der = derive(scene, ids, U["pos"], prec)
        info = None
    else:
        info = cache.frame(ids, stale)
        miss = info["misses"]
        fresh = derive(scene, miss, U["pos"], prec)
        for i, a in enumerate(miss):
            cache_lines[int(a)] = {key: v[i * k:(i + 1) * k].copy() for key, v in fresh.items()}
        der = {key: np.concatenate([cache_lines[int(a)][key] for a in ids]) if len(ids) else
               np.zeros((0,) + fresh[key].shape[1:]) for key in fresh}
    G = compose(len(ids), k, der["alpha"])
    mu, cov, rgb, al = der["mu"][G], der["cov"][G], der["rgb"][G], der["alpha"][G]
    ab = 1e-7
    if lod_fade:
        al = al * lod_w[np.asarray(ids, np.int64)[G // k]]
        ab = FADE_ALPHA_BAND
    out["left"] = render_gaussians(mu, cov, rgb, al, left, debug, alpha_band=ab)
    out["right"] = render_gaussians(mu, cov, rgb, al, right, debug, alpha_band=ab)
    out.update(unified=U, visible=ids, select_band=sel_band, G=G, cache=info,
               mask_band=np.abs(der["alpha_pre"]) < 1e-6, lod_w=lod_w)
    if debug:
        out["derived"] = der
    return out


# ------------------------------------------------------------------ metrics

def psnr(img, ref) -> float:
    """10 log10(1 / MSE) over all 3*H*W values (values in [0,1])."""
    mse = float(np.mean((np.asarray(img, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


# SSIM (Table 4's third quality metric), as defined by Wang et al. (2004):
# per channel, local means, variances and covariance under an 11 x 11
# Gaussian window (sigma 1.5, weights normalised to sum 1), constants
# C1 = (0.01 L)^2 and C2 = (0.03 L)^2 for dynamic range L = 1, the SSIM map
# ((2 mu_x mu_y + C1)(2 s_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
# over every window position inside the image ("valid"), averaged over
# positions and channels.  FP64.

def ssim_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def _blur_valid(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Separable correlation of [H, W] with w (x) w over the valid region."""
    n = len(w)
    H, W = img.shape
    rows = sum(w[i] * img[i:H - n + 1 + i, :] for i in range(n))
    return sum(w[j] * rows[:, j:W - n + 1 + j] for j in range(n))


def ssim(img, ref) -> float:
    """Mean SSIM of two [C, H, W] images in [0, 1] (H, W >= 11)."""
    a = np.asarray(img, np.float64)
    b = np.asarray(ref, np.float64)
    w = ssim_window()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    vals = []
    for ch in range(a.shape[0]):
        x, y = a[ch], b[ch]
        mx, my = _blur_valid(x, w), _blur_valid(y, w)
        sxx = _blur_valid(x * x, w) - mx * mx
        syy = _blur_valid(y * y, w) - my * my
        sxy = _blur_valid(x * y, w) - mx * my
        m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        vals.append(m)
    return float(np.mean(vals))


def max_abs(img, ref) -> float:
    return float(np.max(np.abs(np.asarray(img, np.float64) - np.asarray(ref, np.float64))))


# -------------------------------------------------------- reuse predictor

PRED_FEATURES = 6


def reuse_features(scene, anchors, pu_now, pu_then, age, d_max, fx):
    """Six per-candidate features for the learned reuse decision:
    1 - cos(angle between view directions then and now); log(dist_now /
    dist_then); age / D_max; level / L_max; |p_u(now) - p_u(then)| / dist_now;
    log2(s_level * fx / dist_now) with s_level the anchor's largest offset
    scale (its voxel size)."""
    a = np.asarray(anchors, np.int64)
    x = scene.pos[a].astype(np.float64)
    vn = x - np.asarray(pu_now, np.float64)
    vt = x - np.asarray(pu_then, np.float64).reshape(-1, 3)
    dn = np.linalg.norm(vn, axis=1); dt = np.linalg.norm(vt, axis=1)
    cosang = np.sum(vn * vt, axis=1) / (dn * dt)
    lmax = max(int(scene.l_max), 1)
    f = np.empty((len(a), PRED_FEATURES))
    f[:, 0] = 1.0 - cosang
    f[:, 1] = np.log(dn / dt)
    f[:, 2] = np.asarray(age, np.float64) / d_max
    f[:, 3] = scene.level[a].astype(np.float64) / lmax
    f[:, 4] = np.linalg.norm(np.asarray(pu_now) - np.asarray(pu_then).reshape(-1, 3), axis=1) / dn
    f[:, 5] = np.log2(scene.scale[a, 0:3].astype(np.float64).max(1) * fx / dn)
    return f


def reuse_label(cached: dict, fresh: dict, k: int, size_px) -> np.ndarray:
    """1 (re-derive) iff reusing the anchor would change the image visibly.

    Reading (the reuse decision of Section 4 only says lines are reused while
    the view changes little): a Gaussian's drift is the largest of its
    opacity change, its opacity times its largest colour-channel change, and
    its opacity times half the relative change of its covariance (max |dSigma|
    over max |Sigma| of the fresh one; half because the footprint radius goes
    as the square root of Sigma).  The anchor's drift is the largest over its
    k Gaussians; weighted by its projected footprint area in pixels,
    max(1, size_px^2) with size_px = s_level f_x / distance (the last
    feature), it must exceed 16/255, the change of a 4x4-pixel patch by one
    8-bit level."""
    a_c = np.asarray(cached["alpha"], np.float64).reshape(-1, k)
    a_f = np.asarray(fresh["alpha"], np.float64).reshape(-1, k)
    am = np.maximum(np.abs(a_c), np.abs(a_f))
    dc = np.abs(np.asarray(cached["rgb"]) - np.asarray(fresh["rgb"])).reshape(-1, k, 3).max(2)
    ds = np.abs(np.asarray(cached["cov"]) - np.asarray(fresh["cov"])).reshape(-1, k, 6).max(2)
    sm = np.abs(np.asarray(fresh["cov"])).reshape(-1, k, 6).max(2)
    with np.errstate(divide="ignore", invalid="ignore"):
        geo = np.where(sm > 0, ds / np.where(sm > 0, sm, 1.0), np.where(ds > 0, np.inf, 0.0))
    drift = np.maximum(np.abs(a_c - a_f), am * np.maximum(dc, 0.5 * geo)).max(1)
    area = np.maximum(1.0, np.asarray(size_px, np.float64) ** 2)
    return (drift * area > 16.0 / 255.0).astype(np.uint8)


def pred_forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    logit = (h2 @ W3.T + b3)[:, 0]
    return logit, (X, z1, h1, z2, h2)


def pred_loss_grad(params, X, y, pos_weight: float):
    """Mean weighted binary cross-entropy on sigmoid(logit) and its analytic
    gradient: loss_i = -(w y log p + (1-y) log(1-p)), w = pos_weight."""
    W1, b1, W2, b2, W3, b3 = params
    logit, (X, z1, h1, z2, h2) = pred_forward(params, X)
    y = np.asarray(y, np.float64)
    n = len(y)
    # log p = -softplus(-l), log(1-p) = -softplus(l)
    sp_neg = np.logaddexp(0.0, -logit)
    sp_pos = np.logaddexp(0.0, logit)
    loss = float(np.mean(pos_weight * y * sp_neg + (1.0 - y) * sp_pos))
    p = 1.0 / (1.0 + np.exp(-logit))
    dlogit = (pos_weight * y * (p - 1.0) + (1.0 - y) * p) / n
    gW3 = dlogit[None, :] @ h2
    gb3 = np.array([dlogit.sum()])
    dh2 = dlogit[:, None] @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; step counts from 1."""
    for i in range(len(params)):
        m[i] = b1 * m[i] + (1 - b1) * grads[i]
        v[i] = b2 * v[i] + (1 - b2) * grads[i] ** 2
        mh = m[i] / (1 - b1 ** step)
        vh = v[i] / (1 - b2 ** step)
        params[i] = params[i] - lr * mh / (np.sqrt(vh) + eps)
    return params
