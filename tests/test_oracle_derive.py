"""Pins of the oracle's unified camera, anchor selection and derivation.

  * unified camera (eqs. 5-6): coincident eyes give the eye itself; for a
    parallel pair the unified frustum's side planes pass through the eyes'
    outer side planes (the setback makes its half-width b/2 at the eye
    plane), and points sampled in either eye frustum lie in it;
  * selection: the LOD rule against its log2 form; the frustum test against
    planes built independently from the frustum's corner rays;
  * derivation (eq. 3, eq. 2): an independent float64 torch MLP; zero-weight
    and fixed-quaternion closed forms; rotation against scipy's quaternion
    convention; j-major output layout; bf16 / e4m3fn rounding against
    torch's own conversions.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle
import synth


def test_unified_camera_coincident_eyes():
    c = synth.look_camera((1.0, 2.0, 3.0), (0.3, -0.2, 1.0), (0, -1, 0), 64, 48, math.radians(70))
    u = oracle.unified_camera(c, c)
    assert np.allclose(u["pos"], c["pos"], atol=1e-14)
    assert np.allclose(u["R"], c["R"], atol=1e-14)


@pytest.mark.parametrize("fov,ipd", [(90.0, 0.064), (60.0, 0.5), (100.0, 1.0)])
def test_unified_camera_covers_both_eyes(fov, ipd):
    L, R = synth.stereo_pair((3, -1, 2), (0.4, 0.9, -0.1), (0, 0, 1), 200, 120, math.radians(fov), ipd=ipd)
    U = oracle.unified_camera(L, R)
    tx = math.tan(math.radians(fov) / 2)
    ty = math.tan(U["fovy"] / 2)

    def cam_coords(c, x):
        return (np.asarray(c["R"]) @ (np.asarray(x) - np.asarray(c["pos"])).T).T

    # outer boundary rays of each eye lie on the unified side planes
    for eye, sgn in ((L, -1.0), (R, 1.0)):
        Re = np.asarray(eye["R"])
        for depth in (0.5, 3.0, 40.0):
            for v in (-ty, 0.0, ty):
                x = eye["pos"] + depth * (Re[2] + sgn * tx * Re[0] + v * Re[1])
                t = cam_coords(U, x[None])[0]
                assert abs(t[0] / t[2] - sgn * tx) < 1e-12
    # containment of random points of both frusta
    rng = np.random.default_rng(0)
    for eye in (L, R):
        Re = np.asarray(eye["R"])
        n = 2000
        z = rng.uniform(eye["znear"], 100, n)
        a = rng.uniform(-tx, tx, n); b = rng.uniform(-ty, ty, n)
        x = eye["pos"] + z[:, None] * (Re[2] + a[:, None] * Re[0] + b[:, None] * Re[1])
        t = cam_coords(U, x)
        assert np.all(t[:, 2] >= U["znear"])
        assert np.all(np.abs(t[:, 0] / t[:, 2]) <= tx * (1 + 1e-12))
        assert np.all(np.abs(t[:, 1] / t[:, 2]) <= ty * (1 + 1e-12))


def _scene_with(pos, level, radius, d_ref):
    n = len(pos)
    s = synth.tiny_scene(n=n)
    s.pos = np.asarray(pos, np.float32)
    s.level = np.asarray(level, np.uint8)
    s.radius = np.asarray(radius, np.float32)
    s.d_ref = d_ref
    return s


def test_lod_rule_matches_log2_form():
    rng = np.random.default_rng(1)
    n = 20000
    pos = rng.uniform(-3000, 3000, (n, 3))
    level = rng.integers(0, 11, n)
    cam = synth.look_camera((0, 0, 0), (1, 0, 0), (0, 0, 1), 64, 64, math.radians(90))
    s = _scene_with(pos, level, np.full(n, 1e9), 2.0 ** 19)  # huge spheres: frustum never culls
    ids, band = oracle.select(s, cam)
    dist = np.linalg.norm(s.pos.astype(np.float64), axis=1)
    lmax_ok = np.floor(np.log2(s.d_ref / dist))
    keep = (level == 0) | (level <= lmax_ok)
    ok = band == 0
    got = np.zeros(n, bool); got[ids] = True
    assert np.array_equal(got[ok], keep[ok])
    assert np.all(np.diff(ids) > 0)


def test_frustum_test_matches_corner_ray_planes():
    rng = np.random.default_rng(2)
    n = 20000
    cam = synth.look_camera((5, -3, 1), (0.3, 1.0, -0.2), (0, 0, 1), 300, 200, math.radians(75))
    pos = rng.uniform(-60, 60, (n, 3)) + np.array([5, 25, 1])
    rad = rng.uniform(0, 8, n)
    s = _scene_with(pos, np.zeros(n), rad, 1e30)
    ids, band = oracle.select(s, cam)
    R = np.asarray(cam["R"]); p = np.asarray(cam["pos"])
    tx, ty = math.tan(cam["fovx"] / 2), math.tan(cam["fovy"] / 2)
    corners = [R.T @ np.array([sx * tx, sy * ty, 1.0]) for sx, sy in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
    planes = []
    for i in range(4):
        nrm = np.cross(corners[i], corners[(i + 1) % 4])
        if nrm @ R[2] < 0:
            nrm = -nrm
        planes.append((nrm / np.linalg.norm(nrm), p))
    planes.append((R[2], p + cam["znear"] * R[2]))
    x = s.pos.astype(np.float64)
    keep = np.ones(n, bool)
    for nrm, q in planes:
        keep &= (x - q) @ nrm >= -s.radius.astype(np.float64)
    got = np.zeros(n, bool); got[ids] = True
    ok = band == 0
    assert np.array_equal(got[ok], keep[ok])
    assert 0.05 < keep.mean() < 0.95


def torch_mlp_reference(scene, ids, pu):
    """Independent float64 torch evaluation of the three 2-layer MLPs."""
    x = torch.tensor(scene.pos[ids], dtype=torch.float64)
    v = x - torch.tensor(pu, dtype=torch.float64)
    d = v / v.norm(dim=1, keepdim=True)
    z = torch.cat([torch.tensor(scene.feat[ids], dtype=torch.float64), d], 1)
    outs = {}
    for name in ("alpha", "color", "cov"):
        W1, b1, W2, b2 = [torch.tensor(w, dtype=torch.float64) for w in scene.mlp[name]]
        h = torch.relu(torch.nn.functional.linear(z, W1, b1))
        outs[name] = torch.nn.functional.linear(h, W2, b2).numpy()
    return outs


def test_derive_matches_torch_mlp(tiny):
    ids = np.arange(0, 2000, 7, dtype=np.int32)
    pu = np.array([0.3, -0.1, -15.2])
    der = oracle.derive(tiny, ids, pu)
    ref = torch_mlp_reference(tiny, ids, pu)
    k = tiny.k
    m = len(ids)
    assert np.allclose(der["alpha_pre"].reshape(m, k), ref["alpha"], rtol=0, atol=1e-12)
    assert np.allclose(der["alpha"].reshape(m, k), np.tanh(ref["alpha"]), atol=1e-12)
    assert np.allclose(der["rgb"].reshape(m, k, 3), 1 / (1 + np.exp(-ref["color"].reshape(m, k, 3))), atol=1e-12)
    o = ref["cov"].reshape(m, k, 7)
    sc = tiny.scale[ids, 3:6].astype(np.float64)[:, None, :] / (1 + np.exp(-o[..., 0:3]))
    q = o[..., 3:7] / np.linalg.norm(o[..., 3:7], axis=-1, keepdims=True)
    Rm = Rotation.from_quat(np.concatenate([q[..., 1:4], q[..., 0:1]], -1).reshape(-1, 4)).as_matrix()
    S = np.einsum("nij,nj,nkj->nik", Rm, sc.reshape(-1, 3) ** 2, Rm)
    cov = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]], 1)
    assert np.allclose(der["cov"], cov, atol=1e-12)
    mu = tiny.pos[ids].astype(np.float64)[:, None, :] + tiny.scale[ids, None, 0:3] * tiny.offsets[ids].astype(np.float64)
    assert np.allclose(der["mu"], mu.reshape(-1, 3), atol=1e-12)


def test_derive_zero_weights_closed_form(tiny):
    s = tiny.subset(np.arange(5))
    k = s.k
    mlp = {}
    rng = np.random.default_rng(0)
    for name, c in synth.HEADS:
        W1, b1, W2, b2 = s.mlp[name]
        nb2 = rng.uniform(-1, 1, c * k).astype(np.float32)
        mlp[name] = (W1, b1, np.zeros_like(W2), nb2)
    q = np.array([1.0, 0.0, 0.0, 0.0], np.float32)
    for j in range(k):
        mlp["cov"][3][7 * j + 3:7 * j + 7] = q
    s.mlp = mlp
    der = oracle.derive(s, np.arange(5, dtype=np.int32), np.zeros(3))
    b2a, b2c, b2s = mlp["alpha"][3].astype(np.float64), mlp["color"][3].astype(np.float64), mlp["cov"][3].astype(np.float64)
    assert np.allclose(der["alpha"].reshape(5, k), np.tanh(b2a)[None], atol=1e-15)
    assert np.allclose(der["rgb"].reshape(5, k, 3), (1 / (1 + np.exp(-b2c))).reshape(k, 3)[None], atol=1e-15)
    sc = s.scale[:, None, 3:6].astype(np.float64) / (1 + np.exp(-b2s.reshape(k, 7)[None, :, 0:3]))
    cov = der["cov"].reshape(5, k, 6)
    assert np.allclose(cov[..., 0], sc[..., 0] ** 2, atol=1e-15)
    assert np.allclose(cov[..., 3], sc[..., 1] ** 2, atol=1e-15)
    assert np.allclose(cov[..., 5], sc[..., 2] ** 2, atol=1e-15)
    assert np.all(cov[..., [1, 2, 4]] == 0)


def test_derive_rotation_and_layout_against_scipy(tiny):
    s = tiny.subset(np.arange(3))
    k = s.k
    rng = np.random.default_rng(7)
    quats = rng.standard_normal((k, 4))  # (w, x, y, z), unnormalised
    mlp = dict(s.mlp)
    W1, b1, W2, b2 = s.mlp["cov"]
    nb2 = np.zeros(7 * k, np.float32)
    for j in range(k):
        nb2[7 * j:7 * j + 3] = 0.1 * (j + 1)
        nb2[7 * j + 3:7 * j + 7] = quats[j]
    mlp["cov"] = (W1, b1, np.zeros_like(W2), nb2)
    W1, b1, W2, b2 = s.mlp["alpha"]
    mlp["alpha"] = (W1, b1, np.zeros_like(W2), (0.05 * np.arange(1, k + 1)).astype(np.float32))
    s.mlp = mlp
    der = oracle.derive(s, np.arange(3, dtype=np.int32), np.zeros(3))
    assert np.allclose(der["alpha"].reshape(3, k), np.tanh(0.05 * np.arange(1, k + 1, dtype=np.float32).astype(np.float64)), atol=1e-15)
    q32 = nb2.reshape(k, 7)[:, 3:7].astype(np.float64)
    Rm = Rotation.from_quat(np.concatenate([q32[:, 1:4], q32[:, 0:1]], 1)).as_matrix()
    for a in range(3):
        for j in range(k):
            sc = s.scale[a, 3:6].astype(np.float64) / (1 + np.exp(-np.float64(np.float32(0.1 * (j + 1)))))
            S = Rm[j] @ np.diag(sc ** 2) @ Rm[j].T
            c = der["cov"][a * k + j]
            got = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
            assert np.allclose(got, S, atol=1e-14)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        np.array([1.00390625, 1.01171875, 1.0 + 3 * 2 ** -8, -2.0 - 2 ** -7])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)


def test_e4m3_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 3000), rng.standard_normal(3000) * 2.0 ** rng.uniform(-11, 4, 3000),
                        np.array([2 ** -10, 3 * 2 ** -10, 0.3, 17.0, 240.0, 464.0 - 1e-3])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([oracle.round_e4m3(float(v)) for v in x])
    assert np.array_equal(got, ref)
    assert oracle.round_e4m3(1000.0) == 448.0 and oracle.round_e4m3(-1000.0) == -448.0


def test_emulated_precision_is_close_but_not_exact(tiny):
    ids = np.arange(0, 2000, 11, dtype=np.int32)
    pu = np.array([0.0, 0.0, -15.0])
    ex = oracle.derive(tiny, ids, pu, 0)
    for prec, tol in ((1, 0.05), (2, 0.1)):
        em = oracle.derive(tiny, ids, pu, prec)
        d = np.abs(em["alpha"] - ex["alpha"]).max()
        assert 0 < d < tol
