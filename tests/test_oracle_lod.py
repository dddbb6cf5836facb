"""Pins of the oracle's Octree-GS-fidelity parts (CPU only).

Fractional level transition (a reading of the distance-driven level of
detail of Section 3.1's Octree-GS): a level-l anchor, l > 0, is kept while
its distance to the unified camera centre is below 2 d_l (d_l = d_ref 2^-l)
and its Gaussians' opacities carry w = clamp(2 - dist / d_l, 0, 1).
Pinned by values the definition fixes at chosen distances, by the reduction
to the integer rule, and by the property the fade exists for: no popping,
i.e. the image changes continuously as an anchor crosses a level distance.

Distance input (the cited methods' optional camera-distance MLP feature):
layer 1 takes [f; d_view; dist / dist_unit].  Pinned by the reduction to the
plain input when that column is zero and by a hand-evaluated one-unit net.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def axis_scene(dists, levels, d_ref=40.0, k=1, F=4, H=2, dist_input=False, dist_unit=10.0, seed=0):
    """Anchors on the +z axis at the given distances from the origin."""
    n = len(dists)
    pos = np.zeros((n, 3), np.float32)
    pos[:, 2] = np.asarray(dists, np.float32)
    rng = np.random.Generator(np.random.PCG64(seed))
    feat = rng.standard_normal((n, F)).astype(np.float32)
    offsets = np.zeros((n, k, 3), np.float32)
    scale = np.tile(np.array([0.1, 0.1, 0.1, 0.05, 0.05, 0.05], np.float32), (n, 1))
    mlp = synth.glorot_mlp(F, H, k, seed=seed, dist_input=dist_input)
    return synth.Scene(pos, np.asarray(levels, np.uint8), np.full(n, 0.2, np.float32), feat, scale, offsets, mlp,
                       d_ref=d_ref, l_max=int(max(levels)), dist_unit=dist_unit if dist_input else 0.0)


CAM = synth.look_camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0), 64, 64, math.radians(60))


def test_fade_weights_at_chosen_distances():
    # level 2 with d_ref 40: d_l = 10 m
    dists = [5.0, 10.0, 15.0, 17.5, 19.0, 20.5, 25.0]
    sc = axis_scene(dists, [2] * len(dists))
    ids, band, w = oracle.select(sc, CAM, fade=True, weights=True)
    assert ids.tolist() == [0, 1, 2, 3, 4]           # dist < 2 d_l = 20 m
    assert w[:5] == pytest.approx([1.0, 1.0, 0.5, 0.25, 0.1], abs=1e-6)
    ids0, _ = oracle.select(sc, CAM)                  # the integer rule: dist <= d_l
    assert ids0.tolist() == [0, 1]
    # level 0 is kept at any distance with weight 1
    sc0 = axis_scene([5.0, 300.0], [0, 0])
    ids, _, w = oracle.select(sc0, CAM, fade=True, weights=True)
    assert ids.tolist() == [0, 1] and w.tolist() == [1.0, 1.0]
    # without fade every weight is 1
    _, _, w = oracle.select(sc, CAM, fade=False, weights=True)
    assert np.all(w == 1.0)


def test_fade_selection_band_at_the_outer_distance():
    sc = axis_scene([20.0 * (1 - 1e-9), 20.0 * (1 + 1e-9), 17.0], [2, 2, 2])
    ids, band, w = oracle.select(sc, CAM, fade=True, weights=True)
    assert band[0] == 1 and band[1] == 1 and band[2] == 0
    assert w[0] == pytest.approx(0.0, abs=1e-6)


def test_fade_keeps_a_superset_of_the_integer_rule():
    sc = synth.tiny_lod_scene(n=3000)
    L, R = synth.tiny_pair(96, 80)
    U = oracle.unified_camera(L, R)
    a, _ = oracle.select(sc, U)
    b, _, w = oracle.select(sc, U, fade=True, weights=True)
    assert set(a.tolist()) <= set(b.tolist())
    assert len(b) > len(a)                            # the fading octave adds anchors here
    assert np.all(w[a] == 1.0)                        # fully present where the integer rule keeps them
    extra = np.setdiff1d(b, a)
    assert np.all((w[extra] > 0.0) & (w[extra] < 1.0))


def test_fade_removes_popping():
    """Move the camera straight toward a level-l anchor that sits just beyond
    d_l.  Under the integer rule the anchor (all its Gaussians) appears at
    once as it crosses d_l: a jump in the image.  With the fade it is already
    present with weight ~1 there, so the image changes by an amount that
    shrinks with the step."""
    sc = synth.tiny_lod_scene(n=1500, seed=4)
    fov = math.radians(60)
    base = np.array([0.0, 0.0, -15.0])
    U = oracle.unified_camera(*synth.stereo_pair(base, (0, 0, 1), (0, -1, 0), 80, 64, fov))
    a_int, _ = oracle.select(sc, U)
    a_fade, _, w = oracle.select(sc, U, fade=True, weights=True)
    extra = np.setdiff1d(a_fade, a_int)
    a = int(extra[np.argmax(w[extra])])              # the faded anchor nearest its d_l
    v = sc.pos[a].astype(np.float64) - U["pos"]
    dist = float(np.linalg.norm(v))
    dl = sc.d_ref * 2.0 ** -int(sc.level[a])
    u = v / dist
    start = base + u * (dist - dl - 5e-4)            # the anchor at d_l + 0.5 mm
    imgs = {}
    for fade in (False, True):
        for step in (0.0, 1e-3, 2e-3):
            L, R = synth.stereo_pair(start + u * step, (0, 0, 1), (0, -1, 0), 80, 64, fov)
            imgs[fade, step] = oracle.render_frame(sc, L, R, lod_fade=fade)["left"]["image"]
    jump = np.abs(imgs[False, 1e-3] - imgs[False, 0.0]).max()
    d1 = np.abs(imgs[True, 1e-3] - imgs[True, 0.0]).max()
    d2 = np.abs(imgs[True, 2e-3] - imgs[True, 0.0]).max()
    assert jump > 1e-3
    assert d1 < 0.05 * jump
    assert d1 <= 0.75 * d2 + 1e-9                     # roughly linear in the step


def test_fade_scales_each_anchors_gaussians():
    """render_frame with the fade equals rasterising the derived Gaussians
    with each one's opacity scaled by its own anchor's weight (looked up per
    Gaussian here, anchor by anchor)."""
    sc = synth.tiny_lod_scene(n=800, seed=2)
    L, R = synth.tiny_pair(64, 48)
    ref = oracle.render_frame(sc, L, R, lod_fade=True, debug=True)
    U = oracle.unified_camera(L, R)
    ids, _, w = oracle.select(sc, U, fade=True, weights=True)
    der = oracle.derive(sc, ids, U["pos"])
    rows = []
    alpha = []
    for i, a in enumerate(ids):
        for j in range(sc.k):
            r = i * sc.k + j
            if der["alpha"][r] > 0.0:
                rows.append(r)
                alpha.append(der["alpha"][r] * w[a])
    rows = np.array(rows)
    img = oracle.render_gaussians(der["mu"][rows], der["cov"][rows], der["rgb"][rows], np.array(alpha), L)
    assert np.abs(img["image"] - ref["left"]["image"]).max() == 0.0


def test_distance_input_zero_column_reduces_to_plain():
    sc = axis_scene([5.0, 7.0, 12.0], [0, 0, 0], k=3, F=4, H=6, dist_input=True)
    plain = axis_scene([5.0, 7.0, 12.0], [0, 0, 0], k=3, F=4, H=6, dist_input=False)
    mlp = {}
    for name in sc.mlp:
        W1, b1, W2, b2 = sc.mlp[name]
        W1 = W1.copy()
        W1[:, -1] = 0.0
        mlp[name] = (W1, b1, W2, b2)
        plain.mlp[name] = (np.ascontiguousarray(W1[:, :-1]), b1, W2, b2)
    sc.mlp = mlp
    pu = np.array([0.3, -0.2, 0.1])
    a = oracle.derive(sc, np.arange(3, dtype=np.int32), pu)
    b = oracle.derive(plain, np.arange(3, dtype=np.int32), pu)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_distance_input_one_unit_closed_form():
    """Only the distance column of layer 1 nonzero (weight 1 into hidden unit
    0), layer 2 reading unit 0 with weight 2 for opacity and 1 for red:
    alpha = tanh(2 dist/u), red = sigmoid(dist/u)."""
    sc = axis_scene([5.0, 30.0], [0, 0], k=1, F=4, H=2, dist_input=True, dist_unit=10.0)
    z = lambda a: np.zeros_like(a)  # noqa: E731
    mlp = {}
    for name in sc.mlp:
        W1, b1, W2, b2 = sc.mlp[name]
        W1 = z(W1); W1[0, -1] = 1.0
        W2 = z(W2)
        if name == "alpha":
            W2[0, 0] = 2.0
        if name == "color":
            W2[0, 0] = 1.0
        mlp[name] = (W1, z(b1), W2, z(b2))
    sc.mlp = mlp
    pu = np.array([3.0, 4.0, 0.0])   # anchor 0 at (0,0,5): dist sqrt(9+16+25) = sqrt(50)
    out = oracle.derive(sc, np.array([0, 1], np.int32), pu)
    d0 = math.sqrt(50.0) / 10.0
    d1 = math.sqrt(9 + 16 + 900) / 10.0
    assert out["alpha"][0] == pytest.approx(math.tanh(2 * d0), rel=1e-14)
    assert out["alpha"][1] == pytest.approx(math.tanh(2 * d1), rel=1e-14)
    assert out["rgb"][0, 0] == pytest.approx(1.0 / (1.0 + math.exp(-d0)), rel=1e-14)
    assert out["rgb"][0, 1] == pytest.approx(0.5, rel=1e-14)
