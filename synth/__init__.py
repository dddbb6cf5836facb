"""Seeded synthetic inputs: anchor scenes, MLP weights, stereo camera paths.

This module only *makes inputs*.  It holds none of the renderer's arithmetic
(no unified camera, no selection, no derivation, no projection, no blending):
both the CPU oracle and the GPU library receive the arrays it returns.

Scenes follow the structured-3DGS layout of the paper's Section 3.1 (anchors
carrying a feature vector f, per-anchor offsets and scales, MLP weights theta
that derive k neural Gaussians per anchor, eq. 3).  The paper's trained
MatrixCity models are not available; these seeded scenes stand in for them.

Array conventions (all little-endian, C-contiguous):
  pos      float32 [n, 3]     anchor position (world, metres, z up for city)
  level    uint8   [n]        octree level of detail (0 = coarsest)
  radius   float32 [n]        bounding-sphere radius of everything the anchor
                              can derive (data, precomputed here)
  feat     float32 [n, F]     anchor feature f
  scale    float32 [n, 6]     [0:3] offset scale, [3:6] base Gaussian scale
  offsets  float32 [n, k, 3]  learnable offsets O_j
  mlp      dict head -> (W1 [H, F+3], b1 [H], W2 [c*k, H], b2 [c*k]) float32,
           heads 'alpha' (c=1), 'color' (c=3), 'cov' (c=7), rows = outputs
           like torch.nn.Linear.

Cameras are dicts: R float64 [3,3] world->camera with rows (right, down,
forward); pos float64 [3]; fovx, fovy radians; width, height pixels; znear m.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HEADS = (("alpha", 1), ("color", 3), ("cov", 7))


@dataclass
class Scene:
    pos: np.ndarray
    level: np.ndarray
    radius: np.ndarray
    feat: np.ndarray
    scale: np.ndarray
    offsets: np.ndarray
    mlp: dict
    d_ref: float = 1.0e30
    l_max: int = 0
    meta: dict = field(default_factory=dict)
    dist_unit: float = 0.0   # metres per unit of the MLP's distance input (layer 1 with F + 4 columns)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def k(self) -> int:
        return int(self.offsets.shape[1])

    @property
    def F(self) -> int:
        return int(self.feat.shape[1])

    @property
    def H(self) -> int:
        return int(self.mlp["alpha"][0].shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.pos[idx].copy(), self.level[idx].copy(), self.radius[idx].copy(),
                     self.feat[idx].copy(), self.scale[idx].copy(), self.offsets[idx].copy(),
                     self.mlp, self.d_ref, self.l_max, dict(self.meta), self.dist_unit)


def glorot_mlp(F: int, H: int, k: int, seed: int = 0, quat_w_bias: float = 0.0, dist_input: bool = False) -> dict:
    """Two-layer MLPs (F+3 -> H -> c*k) per head, Glorot-uniform weights, zero
    biases, drawn from PCG64(seed) in the order alpha.W1, alpha.W2, color.W1,
    color.W2, cov.W1, cov.W2.  quat_w_bias sets the bias of every quaternion-w
    output of the cov head (output 7j+3).  dist_input: layer 1 takes one more
    input (F+4 columns, the camera-distance feature)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mlp = {}
    ni = F + 4 if dist_input else F + 3
    for name, c in HEADS:
        fan1 = (ni, H)
        lim1 = math.sqrt(6.0 / (fan1[0] + fan1[1]))
        W1 = rng.uniform(-lim1, lim1, size=(H, ni)).astype(np.float32)
        lim2 = math.sqrt(6.0 / (H + c * k))
        W2 = rng.uniform(-lim2, lim2, size=(c * k, H)).astype(np.float32)
        b1 = np.zeros(H, np.float32)
        b2 = np.zeros(c * k, np.float32)
        if name == "cov" and quat_w_bias:
            b2[3::7] = quat_w_bias
        mlp[name] = (W1, b1, W2, b2)
    return mlp


def _radius(scale: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    # Data attribute: reach of the farthest offset plus 3.5 base-scale sigmas.
    reach = np.sqrt(((scale[:, None, 0:3].astype(np.float64) * offsets) ** 2).sum(-1)).max(1)
    return (reach + 3.5 * scale[:, 3:6].max(1)).astype(np.float32)


def tiny_scene(n: int = 2000, F: int = 32, H: int = 32, k: int = 10, seed: int = 0) -> Scene:
    """Tiny plain scene: anchors uniform in a 10 m cube, N(0,1) features,
    U(-1,1) offsets, fixed scales, level 0 everywhere (Scaffold-like)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-5.0, 5.0, size=(n, 3)).astype(np.float32)
    feat = rng.standard_normal(size=(n, F)).astype(np.float32)
    offsets = rng.uniform(-1.0, 1.0, size=(n, k, 3)).astype(np.float32)
    scale = np.tile(np.array([0.5, 0.5, 0.5, 0.25, 0.25, 0.25], np.float32), (n, 1))
    level = np.zeros(n, np.uint8)
    mlp = glorot_mlp(F, H, k, seed=seed)
    return Scene(pos, level, _radius(scale, offsets), feat, scale, offsets, mlp,
                 d_ref=1.0e30, l_max=0, meta={"name": "tiny", "seed": seed})


def tiny_lod_scene(n: int = 2000, F: int = 32, H: int = 32, k: int = 10, seed: int = 0, l_max: int = 3,
                   d_ref: float = 40.0, dist_input: bool = False, dist_unit: float = 10.0) -> Scene:
    """The tiny scene with octree levels 0..l_max (N_l proportional to 2^l,
    drawn at random) and a LOD reference distance at the tiny camera's range
    (anchors 10-20 m from the tiny pair; level l is kept within d_ref 2^-l:
    40, 20, 10, 5 m), offset and base scales halving per level; optionally
    the MLPs' distance input (distance / dist_unit)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-5.0, 5.0, size=(n, 3)).astype(np.float32)
    feat = rng.standard_normal(size=(n, F)).astype(np.float32)
    offsets = rng.uniform(-1.0, 1.0, size=(n, k, 3)).astype(np.float32)
    w = 2.0 ** np.arange(l_max + 1)
    level = rng.choice(l_max + 1, size=n, p=w / w.sum()).astype(np.uint8)
    base = np.array([0.5, 0.5, 0.5, 0.25, 0.25, 0.25], np.float32)
    scale = (base[None, :] * (0.5 ** level.astype(np.float32))[:, None]).astype(np.float32)
    mlp = glorot_mlp(F, H, k, seed=seed, dist_input=dist_input)
    return Scene(pos, level, _radius(scale, offsets), feat, scale, offsets, mlp, d_ref=d_ref, l_max=l_max,
                 meta={"name": "tiny_lod", "seed": seed}, dist_unit=dist_unit if dist_input else 0.0)


def city_scene(n: int = 1_000_000, F: int = 32, H: int = 32, k: int = 10, seed: int = 0,
               n_buildings: int = 3000, half_extent: float = 1000.0, l_max: int = 10,
               d_ref: float = 2.0 ** 19, dist_input: bool = False) -> Scene:
    """Synthetic city: z-up ground plane over [-E, E]^2 plus random box
    buildings; anchors area-weighted over ground, roofs and walls, split into
    octree levels 0..l_max with N_l proportional to 2^l.  dist_input: the
    MLPs take the camera distance in units of the half extent E."""
    rng = np.random.Generator(np.random.PCG64(seed))
    E = half_extent
    cx = rng.uniform(-E, E, n_buildings)
    cy = rng.uniform(-E, E, n_buildings)
    hx = rng.uniform(5.0, 20.0, n_buildings)
    hy = rng.uniform(5.0, 20.0, n_buildings)
    ht = np.clip(rng.lognormal(math.log(20.0), 0.6, n_buildings), 4.0, 250.0)

    # Surfaces: kind 0 ground, 1 roof, 2 wall facing +-x, 3 wall facing +-y.
    kinds, areas, params = [0], [(2 * E) ** 2], [(0.0, 0.0, E, E, 0.0, 0.0)]
    for b in range(n_buildings):
        kinds.append(1); areas.append(4 * hx[b] * hy[b]); params.append((cx[b], cy[b], hx[b], hy[b], ht[b], 0.0))
        for sgn in (-1.0, 1.0):
            kinds.append(2); areas.append(2 * hy[b] * ht[b]); params.append((cx[b] + sgn * hx[b], cy[b], 0.0, hy[b], ht[b], sgn))
            kinds.append(3); areas.append(2 * hx[b] * ht[b]); params.append((cx[b], cy[b] + sgn * hy[b], hx[b], 0.0, ht[b], sgn))
    kinds = np.array(kinds, np.int64)
    areas = np.array(areas, np.float64)
    params = np.array(params, np.float64)
    a_total = float(areas.sum())

    weights = 2.0 ** np.arange(l_max + 1)
    counts = np.round(n * weights / weights.sum()).astype(np.int64)
    counts[-1] += n - counts.sum()

    pos = np.empty((n, 3), np.float64)
    level = np.empty(n, np.uint8)
    scale = np.empty((n, 6), np.float64)
    start = 0
    for l in range(l_max + 1):
        m = int(counts[l])
        sl = math.sqrt(a_total / m)
        surf = rng.choice(len(areas), size=m, p=areas / a_total)
        u = rng.uniform(-1.0, 1.0, size=(m, 2))
        kd = kinds[surf]
        pr = params[surf]
        p = np.empty((m, 3))
        sc = np.empty((m, 6))
        tt = np.array([1.0, 1.0, 0.1]); bt = np.array([0.5, 0.5, 0.05])
        # ground / roof: tangent x, y; normal z
        g = kd <= 1
        p[g, 0] = pr[g, 0] + u[g, 0] * pr[g, 2]
        p[g, 1] = pr[g, 1] + u[g, 1] * pr[g, 3]
        p[g, 2] = pr[g, 4]
        sc[g, 0:3] = sl * tt
        sc[g, 3:6] = sl * bt
        # wall facing x: tangent y, z; normal x
        w = kd == 2
        p[w, 0] = pr[w, 0]
        p[w, 1] = pr[w, 1] + u[w, 0] * pr[w, 3]
        p[w, 2] = (u[w, 1] * 0.5 + 0.5) * pr[w, 4]
        sc[w, 0:3] = sl * tt[[2, 0, 1]]
        sc[w, 3:6] = sl * bt[[2, 0, 1]]
        # wall facing y: tangent x, z; normal y
        w = kd == 3
        p[w, 0] = pr[w, 0] + u[w, 0] * pr[w, 2]
        p[w, 1] = pr[w, 1]
        p[w, 2] = (u[w, 1] * 0.5 + 0.5) * pr[w, 4]
        sc[w, 0:3] = sl * tt[[0, 2, 1]]
        sc[w, 3:6] = sl * bt[[0, 2, 1]]
        pos[start:start + m] = p
        level[start:start + m] = l
        scale[start:start + m] = sc
        start += m

    feat = rng.standard_normal(size=(n, F), dtype=np.float32)
    offsets = rng.uniform(-1.0, 1.0, size=(n, k, 3)).astype(np.float32)
    scale = scale.astype(np.float32)
    mlp = glorot_mlp(F, H, k, seed=seed, quat_w_bias=1.0, dist_input=dist_input)
    return Scene(pos.astype(np.float32), level, _radius(scale, offsets), feat, scale, offsets, mlp,
                 d_ref=d_ref, l_max=l_max,
                 meta={"name": "city", "seed": seed, "n_buildings": n_buildings,
                       "surface_area_m2": a_total, "level_counts": counts.tolist()},
                 dist_unit=half_extent if dist_input else 0.0)


# ----------------------------------------------------------------------------------------
# cameras and trajectories

def look_camera(pos, forward, up, width, height, fovx, fovy=None, znear=0.2) -> dict:
    """Camera at pos looking along forward; rows of R are right, down, forward."""
    f = np.asarray(forward, np.float64); f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64)); r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    if fovy is None:
        fovy = 2.0 * math.atan(math.tan(fovx / 2.0) * height / width)
    return {"R": np.stack([r, d, f]), "pos": np.asarray(pos, np.float64).copy(),
            "fovx": float(fovx), "fovy": float(fovy), "width": int(width),
            "height": int(height), "znear": float(znear)}


def stereo_pair(head, forward, up, width, height, fovx, fovy=None, ipd=0.064, znear=0.2):
    """Parallel eyes at head -+ ipd/2 along the right axis."""
    c = look_camera(head, forward, up, width, height, fovx, fovy, znear)
    right = c["R"][0]
    left = dict(c, pos=np.asarray(head, np.float64) - 0.5 * ipd * right)
    rght = dict(c, pos=np.asarray(head, np.float64) + 0.5 * ipd * right)
    left["R"] = c["R"].copy(); rght["R"] = c["R"].copy()
    return left, rght


def tiny_pair(width=256, height=256, fov_deg=60.0, ipd=0.064):
    """Camera at (0,0,-15) looking +z with y down; eyes +-ipd/2 along x."""
    return stereo_pair((0.0, 0.0, -15.0), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0), width, height,
                       math.radians(fov_deg), math.radians(fov_deg), ipd)


CITY_W, CITY_H = 2048, 1080
CITY_FOVX = math.radians(90.0)
CITY_FOVY = 2.0 * math.atan(540.0 / 1024.0)


def city_flythrough(frames: int = 300, width=CITY_W, height=CITY_H):
    """Rise from 2 m to 300 m toward the origin: head(s) = (-800+517s,
    -800+517s, 2+298s), s = i/(frames-1), looking at the origin, z up."""
    out = []
    for i in range(frames):
        s = i / max(frames - 1, 1)
        head = np.array([-800.0 + 517.0 * s, -800.0 + 517.0 * s, 2.0 + 298.0 * s])
        fovx = CITY_FOVX
        fovy = 2.0 * math.atan(math.tan(fovx / 2.0) * height / width)
        out.append(stereo_pair(head, -head, (0.0, 0.0, 1.0), width, height, fovx, fovy))
    return out


def city_walk(frames: int = 600, seed: int = 1, start=(-500.0, -500.0, 10.0), yaw0=None,
              pitch0=-10.0, width=CITY_W, height=CITY_H):
    """Small-step walk: each frame a U(0.05,0.5) m step along the horizontal
    heading, then a U(0.1,2) degree turn about yaw (p=0.8) or pitch (p=0.2);
    each turn sign persists and flips with p=0.1; pitch in [-30, 0] degrees;
    altitude in [2, 100] m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.array(start, np.float64)
    yaw = math.degrees(math.atan2(-p[1], -p[0])) if yaw0 is None else float(yaw0)
    pitch = float(pitch0)
    sy, sp = 1.0, -1.0
    fovx = CITY_FOVX
    fovy = 2.0 * math.atan(math.tan(fovx / 2.0) * height / width)
    out = []
    for _ in range(frames):
        fwd = np.array([math.cos(math.radians(pitch)) * math.cos(math.radians(yaw)),
                        math.cos(math.radians(pitch)) * math.sin(math.radians(yaw)),
                        math.sin(math.radians(pitch))])
        out.append(stereo_pair(p.copy(), fwd, (0.0, 0.0, 1.0), width, height, fovx, fovy))
        step = rng.uniform(0.05, 0.5)
        p[0] += step * math.cos(math.radians(yaw))
        p[1] += step * math.sin(math.radians(yaw))
        p[2] = min(max(p[2], 2.0), 100.0)
        ang = rng.uniform(0.1, 2.0)
        if rng.uniform() < 0.8:
            if rng.uniform() < 0.1:
                sy = -sy
            yaw += sy * ang
        else:
            if rng.uniform() < 0.1:
                sp = -sp
            pitch = min(max(pitch + sp * ang, -30.0), 0.0)
    return out


def city_staged_walk(frames: int = 300, start=(-500.0, -500.0, 30.0), yaw0: float = 45.0, pitch: float = -15.0,
                     stages=((0.2, 0.3), (1.0, 3.0), (3.0, 10.0)), width=CITY_W, height=CITY_H):
    """Walk in equal stages of constant speed, each (step m, yaw turn deg)
    per frame: slow, medium, fast (staged speed changes).  The update rate of
    the cache rises from stage to stage."""
    p = np.array(start, np.float64)
    yaw = float(yaw0)
    fovx = CITY_FOVX
    fovy = 2.0 * math.atan(math.tan(fovx / 2.0) * height / width)
    out = []
    for i in range(frames):
        step, turn = stages[min(len(stages) - 1, i * len(stages) // frames)]
        fwd = np.array([math.cos(math.radians(pitch)) * math.cos(math.radians(yaw)),
                        math.cos(math.radians(pitch)) * math.sin(math.radians(yaw)),
                        math.sin(math.radians(pitch))])
        out.append(stereo_pair(p.copy(), fwd, (0.0, 0.0, 1.0), width, height, fovx, fovy))
        p[0] += step * math.cos(math.radians(yaw))
        p[1] += step * math.sin(math.radians(yaw))
        yaw += turn
    return out


SERVING_RESOLUTIONS = ((1280, 720), (2048, 1080), (2560, 1440))


def serving_workload(viewers: int = 8, frames: int = 600, rate_hz: float = 72.0,
                     session_gap_s: float = 0.25, seed: int = 7):
    """Viewer v: a walk seeded 100+v from a random start, a per-eye resolution
    drawn (seed 200+v) from SERVING_RESOLUTIONS, a session start from a
    Poisson process with the given mean gap (seed), and Poisson frame
    requests at rate_hz.  Returns a list of dicts with 'res', 'start',
    'arrivals' (seconds, absolute) and 'cams' (list of stereo pairs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(session_gap_s, viewers)
    starts = np.cumsum(gaps) - gaps[0]
    out = []
    for v in range(viewers):
        rr = np.random.Generator(np.random.PCG64(200 + v))
        w, h = SERVING_RESOLUTIONS[int(rr.integers(0, len(SERVING_RESOLUTIONS)))]
        rs = np.random.Generator(np.random.PCG64(100 + v))
        st = (rs.uniform(-600, 600), rs.uniform(-600, 600), rs.uniform(5, 50))
        cams = city_walk(frames, seed=100 + v, start=st, yaw0=rs.uniform(-180, 180),
                         width=w, height=h)
        inter = rs.exponential(1.0 / rate_hz, frames)
        arrivals = starts[v] + np.cumsum(inter)
        out.append({"res": (w, h), "start": float(starts[v]), "arrivals": arrivals, "cams": cams})
    return out


def predictor_init(seed: int = 3, width: int = 64, n_in: int = 6):
    """Initial reuse-predictor weights Linear(n_in,64)-ReLU-Linear(64,64)-
    ReLU-Linear(64,1) (rows = outputs): Glorot-uniform weights, zero biases,
    drawn from PCG64(seed) in layer order (W1, W2, W3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for o, i in ((width, n_in), (width, width), (1, width)):
        lim = math.sqrt(6.0 / (o + i))
        params.append(rng.uniform(-lim, lim, size=(o, i)))
        params.append(np.zeros(o))
    return params


def random_gaussians(n: int, seed: int = 0, box: float = 4.0, zc: float = 0.0, s_lo=0.05, s_hi=0.6):
    """Explicit anisotropic Gaussians (raster-only inputs): means in a box,
    a random symmetric positive-definite covariance, rgb in (0,1), opacity in
    (0,1).  Returns float32 arrays mu [n,3], cov [n,6] (xx,xy,xz,yy,yz,zz),
    rgb [n,3], alpha [n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-box, box, size=(n, 3))
    mu[:, 2] += zc
    # A random symmetric positive-definite matrix A A^T with A's entries
    # scaled so that sqrt(eigenvalues) fall roughly in [s_lo, s_hi].
    A = rng.standard_normal(size=(n, 3, 3)) * rng.uniform(s_lo, s_hi, size=(n, 1, 1)) / math.sqrt(3.0)
    C = A @ np.transpose(A, (0, 2, 1)) + (s_lo * s_lo) * np.eye(3)
    cov = np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], 1)
    rgb = rng.uniform(0.05, 0.95, size=(n, 3))
    alpha = rng.uniform(0.02, 0.98, size=n)
    return (mu.astype(np.float32), cov.astype(np.float32), rgb.astype(np.float32),
            alpha.astype(np.float32))
