"""Pins of three oracle parts that its other tests leave open.

  * The EWA Jacobian's off-axis clamp (Section 3.1 splatting; the slope
    t_x/t_z, t_y/t_z held to +-1.3 tan(fov/2) per axis): three Gaussians
    outside the clamp cone whose 2D covariance, mean and conic were worked
    out by hand (the numbers are written below with their derivation), on an
    identity camera and on an axis-permuting one with unequal fields of view,
    so a wrong factor, a clamp taken on the wrong axis or quantity, a
    transposed rotation or a clamped mean gives other numbers.
  * Where the BF16 / FP8 emulation of the derivation rounds (Section 6,
    AnchorDecoder; the precision forms): an independent float64 torch
    recomputation that takes every rounding from torch's own bfloat16 and
    float8_e4m3fn conversions and every product from F.linear must match
    oracle.derive element by element; alternative placements (no rounding of
    the input or of the hidden layer, rounding before the bias, rounded
    biases, per-column or per-tensor FP8 scales, FP8 activations) must not.
  * compose (Alg. 1's render buffer with the opacity mask of Section 6): a
    hand-built opacity table with zeros, signed zeros, negatives and values
    at the edge of the double range against the id list written out by hand.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth


# ---------------------------------------------------------------- EWA clamp

def _cam(R, pos, W, H, tan_x, tan_y):
    return {"R": np.asarray(R, np.float64), "pos": np.asarray(pos, np.float64), "fovx": 2 * math.atan(tan_x),
            "fovy": 2 * math.atan(tan_y), "width": W, "height": H, "znear": 0.2}


def _project_one(mu, cov, cam):
    pre = oracle.preprocess(np.asarray([mu], np.float64), np.asarray([cov], np.float64), np.array([0.5]), cam)
    assert pre["keep"][0] == 1
    return pre


# Camera for all three cases: W = 200, H = 100, tan(fovx/2) = 1, tan(fovy/2)
# = 0.5, so fx = 200 / 2 = 100, fy = 100 / (2 * 0.5) = 100, principal point
# (100, 50); the clamp limits are 1.3 (x) and 0.65 (y).
CLAMP_CASES = [
    # identity camera at the origin, isotropic unit covariance at (10, 0, 2):
    # t = (10, 0, 2), slope x = 5 -> 1.3; J = [[100/2, 0, -100*1.3/2], [0, 100/2, 0]]
    # = [[50, 0, -65], [0, 50, 0]]; J J^T + 0.3 I = [[2500 + 4225 + 0.3, 0],
    # [0, 2500.3]]; mean (100*5 + 100, 0 + 50) = (600, 50), unclamped
    dict(R=np.eye(3), pos=(0, 0, 0), mu=(10, 0, 2), cov=(1, 0, 0, 1, 0, 1),
         sigma=(6725.3, 0.0, 2500.3), mean=(600.0, 50.0)),
    # same camera, (0, 3, 2): slope y = 1.5 -> 0.65 (the y limit, not x's 1.3);
    # J = [[50, 0, 0], [0, 50, -100*0.65/2 = -32.5]]; Sigma2D = [[2500.3, 0],
    # [0, 2500 + 1056.25 + 0.3]]; mean (100, 100*1.5 + 50 = 200)
    dict(R=np.eye(3), pos=(0, 0, 0), mu=(0, 3, 2), cov=(1, 0, 0, 1, 0, 1),
         sigma=(2500.3, 0.0, 3556.55), mean=(100.0, 200.0)),
    # camera at (1, 2, 3) whose right, down, forward axes are world y, z, x;
    # mu = p + R^T t for t = (-8, -2, 4) = (1 + 4, 2 - 8, 3 - 2) = (5, -6, 1);
    # world covariance [[4, .5, 0], [.5, 1, 0], [0, 0, 9]] is, in camera axes,
    # Sc = [[1, 0, .5], [0, 9, 0], [.5, 0, 4]]; slopes -2 -> -1.3 (clamped),
    # -0.5 (inside 0.65); J = [[25, 0, -100*(-1.3)/4 = 32.5], [0, 25,
    # -100*(-0.5)/4 = 12.5]]; J Sc = [[41.25, 0, 142.5], [6.25, 225, 50]];
    # J Sc J^T = [[1031.25 + 4631.25, 1781.25], [1781.25, 5625 + 625]];
    # mean (100*(-2) + 100, 100*(-0.5) + 50) = (-100, 0)
    dict(R=[[0, 1, 0], [0, 0, 1], [1, 0, 0]], pos=(1, 2, 3), mu=(5, -6, 1), cov=(4, 0.5, 0, 1, 0, 9),
         sigma=(5662.8, 1781.25, 6250.3), mean=(-100.0, 0.0)),
]


@pytest.mark.parametrize("case", CLAMP_CASES, ids=["x-slope", "y-slope", "permuted-anisotropic"])
def test_ewa_jacobian_clamp_hand_worked(case):
    cam = _cam(case["R"], case["pos"], 200, 100, 1.0, 0.5)
    pre = _project_one(case["mu"], case["cov"], cam)
    a, b, c = case["sigma"]
    assert np.allclose(pre["sigma2d"][0], [a, b, c], rtol=1e-13, atol=1e-10), pre["sigma2d"][0]
    assert np.allclose(pre["mean2d"][0], case["mean"], rtol=0, atol=1e-10), pre["mean2d"][0]
    det = a * c - b * b
    assert np.allclose(pre["conic"][0], [c / det, -b / det, a / det], rtol=1e-12, atol=0)
    # the projected mean leaves the image, and it is the covariance alone
    # that the clamp changes: the unclamped Jacobian would give a different
    # Sigma2D (here the x row of case 1 would be 2500 + 62500 + 0.3)
    assert case["sigma"] != (65000.3, 0.0, 2500.3)


def test_ewa_clamp_is_continuous_at_the_limit():
    # just inside and just outside the clamp cone the covariance agrees to the
    # size of the step (the clamp replaces the slope, it does not jump)
    cam = _cam(np.eye(3), (0, 0, 0), 200, 100, 1.0, 0.5)
    out = []
    for slope in (1.3 - 1e-9, 1.3 + 1e-9):
        pre = _project_one((2.0 * slope, 0.0, 2.0), (1, 0.2, 0.1, 1, 0, 1), cam)
        out.append(pre["sigma2d"][0])
    assert np.allclose(out[0], out[1], rtol=1e-7)


# ------------------------------------------------ precision emulation

def _q_bf16(x):
    return torch.as_tensor(x, dtype=torch.float64).to(torch.bfloat16).to(torch.float64)


def _q_weights(W, prec, scale="row"):
    W = torch.as_tensor(np.asarray(W, np.float32), dtype=torch.float64)
    if prec == 1:
        return _q_bf16(W)
    if scale == "row":
        s = W.abs().amax(dim=1, keepdim=True) / 448.0
    elif scale == "col":
        s = W.abs().amax(dim=0, keepdim=True) / 448.0
    else:
        s = W.abs().amax() / 448.0
    s = torch.where(s > 0, s, torch.ones_like(s))
    return (W / s).to(torch.float8_e4m3fn).to(torch.float64) * s


def emulated_heads(scene, ids, pu, prec, round_z=True, round_h=True, round_before_bias=False, round_bias=False,
                   scale="row", fp8_act=False):
    """The three heads' pre-activations, recomputed in float64 with torch:
    the reading is z = [f; d] rounded to bf16, weights rounded (bf16, or
    e4m3fn with one scale per output row = max |row| / 448), biases exact,
    h = ReLU(W1 z + b1) rounded to bf16, o = W2 h + b2.  The keyword
    arguments switch to alternative placements of the rounding."""
    x = torch.as_tensor(scene.pos[ids].astype(np.float64))
    v = x - torch.as_tensor(np.asarray(pu, np.float64))
    d = v / v.norm(dim=1, keepdim=True)
    z = torch.cat([torch.as_tensor(scene.feat[ids].astype(np.float64)), d], 1)
    act = (lambda t: t.to(torch.float8_e4m3fn).to(torch.float64)) if fp8_act else _q_bf16
    if round_z:
        z = act(z)
    outs = {}
    for name in ("alpha", "color", "cov"):
        W1, b1, W2, b2 = scene.mlp[name]
        W1q, W2q = _q_weights(W1, prec, scale), _q_weights(W2, prec, scale)
        b1d = torch.as_tensor(b1.astype(np.float64))
        b2d = torch.as_tensor(b2.astype(np.float64))
        if round_bias:
            b1d, b2d = _q_bf16(b1d), _q_bf16(b2d)
        if round_before_bias:
            h = torch.relu(act(F.linear(z, W1q)) + b1d)
        else:
            h = torch.relu(F.linear(z, W1q, b1d))
            if round_h:
                h = act(h)
        outs[name] = F.linear(h, W2q, b2d).numpy()
    return outs


@pytest.fixture(scope="module")
def biased_scene():
    # nonzero first-layer biases (the generator's are zero), so that the
    # placement of the bias relative to the rounding matters
    s = synth.tiny_scene(n=300)
    rng = np.random.default_rng(4)
    mlp = {}
    for name, _ in synth.HEADS:
        W1, b1, W2, b2 = s.mlp[name]
        mlp[name] = (W1, rng.uniform(-0.3, 0.3, b1.shape).astype(np.float32), W2,
                     rng.uniform(-0.3, 0.3, b2.shape).astype(np.float32))
    s.mlp = mlp
    return s


@pytest.mark.parametrize("prec", [1, 2])
def test_emulation_matches_independent_torch_recomputation(biased_scene, prec):
    s = biased_scene
    ids = np.arange(0, s.n, 3, dtype=np.int32)
    pu = np.array([0.4, -0.3, -14.0])
    der = oracle.derive(s, ids, pu, prec)
    ref = emulated_heads(s, ids, pu, prec)
    m, k = len(ids), s.k
    assert np.allclose(der["alpha_pre"].reshape(m, k), ref["alpha"], rtol=0, atol=1e-12)
    assert np.allclose(der["rgb"].reshape(m, k, 3), 1 / (1 + np.exp(-ref["color"].reshape(m, k, 3))), atol=1e-12)
    o = ref["cov"].reshape(m, k, 7)
    sc = s.scale[ids, 3:6].astype(np.float64)[:, None, :] / (1 + np.exp(-o[..., 0:3]))
    cov = der["cov"].reshape(m, k, 6)
    q = o[..., 3:7] / np.linalg.norm(o[..., 3:7], axis=-1, keepdims=True)
    # the rotation's first column times scale: Sigma_xx = sum_l R_0l^2 s_l^2
    w, xq, yq, zq = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r00, r01, r02 = 1 - 2 * (yq * yq + zq * zq), 2 * (xq * yq - w * zq), 2 * (xq * zq + w * yq)
    sxx = r00 ** 2 * sc[..., 0] ** 2 + r01 ** 2 * sc[..., 1] ** 2 + r02 ** 2 * sc[..., 2] ** 2
    assert np.allclose(cov[..., 0], sxx, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("prec,alt", [
    (1, dict(round_z=False)), (1, dict(round_h=False)), (1, dict(round_before_bias=True)),
    (1, dict(round_bias=True)),
    (2, dict(round_z=False)), (2, dict(round_h=False)), (2, dict(round_before_bias=True)),
    (2, dict(scale="col")), (2, dict(scale="tensor")), (2, dict(fp8_act=True)),
], ids=lambda v: str(v))
def test_emulation_rejects_other_rounding_placements(biased_scene, prec, alt):
    s = biased_scene
    ids = np.arange(0, s.n, 3, dtype=np.int32)
    pu = np.array([0.4, -0.3, -14.0])
    der = oracle.derive(s, ids, pu, prec)
    other = emulated_heads(s, ids, pu, prec, **alt)
    d = np.abs(der["alpha_pre"] - other["alpha"].reshape(-1)).max()
    assert d > 1e-6, (alt, d)


# -------------------------------------------------------------- compose

def test_compose_hand_built_table():
    # 4 visible anchors, k = 3; kept iff opacity > 0 (tanh of the head's output)
    alpha = np.array([[0.5, 0.0, -0.2],
                      [0.0, -0.0, -1.0],
                      [-0.0, 1e-300, 0.3],
                      [0.9, 0.1, -1e-300]])
    G = oracle.compose(4, 3, alpha.reshape(-1))
    # (0,0) -> 0; row 1 empty; (2,1) -> 7, (2,2) -> 8; (3,0) -> 9, (3,1) -> 10
    assert G.tolist() == [0, 7, 8, 9, 10]
    assert oracle.compose(0, 3, np.zeros(0)).tolist() == []
    assert oracle.compose(2, 1, np.array([-1.0, -2.0])).tolist() == []


# ---------------------------------------------------------------- float32 position bands
# A decision of the tile test or of the pixel alpha threshold is marginal
# when its margin in q is within what a float32 screen position allows: two
# float32 ulps of |mx| + |my| + W + H times |grad q| (bounded by
# 2 sqrt(q (a + c))), on top of the 1e-5 relative band of the tile test and
# the 1e-7 alpha band of the pixel test.  Pinned by the same geometry placed
# near the image origin and near x = 2000 px: the same margin is decided in
# the first case and marginal in the second.

def _one_gaussian(mx, my, alpha, W, H):
    pre = {"mean2d": np.array([[mx, my]], np.float64), "conic": np.array([[1.0, 0.0, 1.0]]),
           "sigma2d": np.array([[1.0, 0.0, 1.0]]), "keep": np.ones(1, np.uint8)}
    return pre, np.array([alpha])


@pytest.mark.parametrize("x_tile,W,marginal", [(1, 64, False), (125, 2048, True)])
def test_tile_band_grows_with_the_screen_coordinate(x_tile, W, marginal):
    alpha = 0.5
    tau = 2.0 * math.log(255.0 * alpha)
    margin = 2e-3                      # q at tile (x_tile, 0) is tau - margin: listed
    x0 = 16 * x_tile + 0.5             # left pixel-centre column of the tile
    mx = x0 - math.sqrt(tau - margin)
    pre, al = _one_gaussian(mx, 8.0, alpha, W, 64)
    tile, g, fl = oracle.tile_pairs(pre, al, W, 64)
    row0 = {int(t): int(f) for t, f in zip(tile, fl) if t < W // 16}
    assert row0[x_tile] & 1 == 1                         # listed
    assert bool(row0[x_tile] & 2) == marginal
    delta = 2.0 ** -23 * (abs(mx) + 8.0 + W + 64)
    band = 1e-5 * (tau + 1.0) + 2.0 * math.sqrt(tau * 2.0) * delta
    assert (margin <= band) == marginal


@pytest.mark.parametrize("px,W,marginal", [(20, 64, False), (2000, 2048, True)])
def test_pixel_alpha_band_grows_with_the_screen_coordinate(px, W, marginal):
    # one Gaussian whose alpha at the pixel centre (px + 0.5, 8.5) is 1/255
    # times (1 + 1e-3): composited by the exact arithmetic
    alpha = 0.5
    a_px = (1.0 / 255.0) * (1.0 + 1e-3)
    q = 2.0 * math.log(alpha / a_px)
    mx = px + 0.5 - math.sqrt(q)
    pre, al = _one_gaussian(mx, 8.5, alpha, W, 16)
    pre["depth"] = np.array([5.0])
    ntiles = (W // 16) * 1
    t = px // 16
    starts = np.zeros(ntiles, np.int64); ends = np.zeros(ntiles, np.int64)
    ends[t] = 1
    starts[t + 1:] = 1; ends[t + 1:] = 1
    img, T, nc, band, ne = oracle.blend(W, 16, starts, ends, np.array([0], np.int32), pre, al,
                                        np.array([[1.0, 1.0, 1.0]]))
    assert nc[8, px] == 1 and abs(img[0, 8, px] - a_px) < 1e-15
    assert bool(band[8, px]) == marginal
    da = a_px * math.sqrt(q * 2.0) * 2.0 ** -23 * (abs(mx) + 8.5 + W + 16)
    assert (a_px - 1.0 / 255.0 < 1e-7 + da) == marginal


def test_marginal_pair_left_out_flags_the_pixels_it_reaches():
    """A Gaussian whose minimum q over a tile exceeds its threshold by less
    than the tile test's band is left out of that tile, but the other side
    may list it and composite it where its alpha reaches 1/255: the pixel at
    the minimum is flagged, a pixel where q is well above the threshold is
    not, and neither image value changes."""
    alpha = 0.5
    tau = 2.0 * math.log(255.0 * alpha)
    W, H = 64, 16
    x0 = 16 * 1 + 0.5                           # tile (1, 0): pixel centres from x = 16.5
    mx = x0 - math.sqrt(tau + 1e-6)             # min q over the tile = tau + 1e-6 (in band, unlisted)
    pre, al = _one_gaussian(mx, 8.5, alpha, W, H)
    pre["depth"] = np.array([5.0])
    tile, g, fl = oracle.tile_pairs(pre, al, W, H)
    fl_t = {int(t): int(f) for t, f in zip(tile, fl)}
    assert fl_t[1] == 2                          # marginal, not listed
    listed = (fl & 1) == 1
    ntiles = W // 16
    s, e = oracle.tile_ranges(tile[listed], ntiles)
    order = np.argsort(tile[listed], kind="stable")
    sg = g[listed][order]
    gs_, ge_ = oracle.tile_ranges(tile[fl == 2], ntiles)
    img0, _, _, band0, _ = oracle.blend(W, H, s, e, sg, pre, al, np.array([[1.0, 1.0, 1.0]]))
    img1, _, _, band1, _ = oracle.blend(W, H, s, e, sg, pre, al, np.array([[1.0, 1.0, 1.0]]),
                                        ghosts=(gs_, ge_, g[fl == 2].astype(np.int32)))
    assert np.array_equal(img0, img1)
    assert band1[8, 16] == 1 and band0[8, 16] == 0    # the pixel at the minimum
    assert band1[8, 31] == 0                          # q far above the threshold
    assert band1[0, 16] == 0                          # q above by (8 px)^2 * c
