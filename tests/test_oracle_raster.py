"""Pins of the oracle's rasteriser (projection, tile lists, sort, blend).

Each test checks the oracle against something it does not itself compute:
  * the closed-form image of one isotropic Gaussian on the optical axis
    (EWA with a vanishing third Jacobian column: Sigma2D = (f s / z)^2 I + 0.3 I);
  * the closed form of two on-axis Gaussians, front over back;
  * a brute-force NumPy renderer that uses no tiles and no sort keys: every
    Gaussian at every pixel, depth order in float64, and a 2D covariance
    built from a central-difference Jacobian of the perspective map;
  * transmittance bounds; mirror symmetry of a stereo pair;
  * a dense grid search for the rectangle minimum behind the tile test;
  * numpy.lexsort for the stable (tile, depth) order.
"""
import math

import numpy as np
import pytest

import oracle
import synth

MIN_A = 1.0 / 255.0


def cam_at_origin(W=64, H=64, fov=60.0):
    return synth.look_camera((0, 0, 0), (0, 0, 1), (0, -1, 0), W, H, math.radians(fov), math.radians(fov))


def test_single_isotropic_gaussian_closed_form():
    W = H = 64
    cam = cam_at_origin(W, H)
    f = W / (2 * math.tan(math.radians(30)))
    z, s, a0 = 5.0, 0.1, 0.8
    rgb = np.array([[0.2, 0.5, 0.9]])
    mu = np.array([[0.0, 0.0, z]])
    cov = np.array([[s * s, 0, 0, s * s, 0, s * s]])
    out = oracle.render_gaussians(mu, cov, rgb, np.array([a0]), cam)
    sig2 = (f * s / z) ** 2 + 0.3
    u = np.arange(W) + 0.5
    r2 = (u[None, :] - W / 2) ** 2 + (u[:, None] - H / 2) ** 2
    a = np.minimum(0.99, a0 * np.exp(-r2 / (2 * sig2)))
    a = np.where(a >= MIN_A, a, 0.0)
    expect = rgb[0][:, None, None] * a[None]
    assert np.max(np.abs(out["image"] - expect)) < 1e-12
    assert np.max(np.abs(out["T"] - (1 - a))) < 1e-12


def test_two_on_axis_gaussians_closed_form():
    W = H = 48
    cam = cam_at_origin(W, H)
    f = W / (2 * math.tan(math.radians(30)))
    mu = np.array([[0.0, 0.0, 8.0], [0.0, 0.0, 4.0]])  # listed back-first: the sort must reorder
    s = np.array([0.3, 0.08])
    cov = np.stack([[q * q, 0, 0, q * q, 0, q * q] for q in s])
    rgb = np.array([[0.9, 0.1, 0.1], [0.1, 0.8, 0.3]])
    al = np.array([0.7, 0.6])
    out = oracle.render_gaussians(mu, cov, rgb, al, cam)
    u = np.arange(W) + 0.5
    r2 = (u[None, :] - W / 2) ** 2 + (u[:, None] - H / 2) ** 2
    def alpha_at(i):
        sig2 = (f * s[i] / mu[i, 2]) ** 2 + 0.3
        a = np.minimum(0.99, al[i] * np.exp(-r2 / (2 * sig2)))
        return np.where(a >= MIN_A, a, 0.0)
    a_front, a_back = alpha_at(1), alpha_at(0)
    expect = rgb[1][:, None, None] * a_front + rgb[0][:, None, None] * a_back * (1 - a_front)
    assert np.max(np.abs(out["image"] - expect)) < 1e-12


def brute_force(mu, cov, rgb, alpha, cam):
    """Every Gaussian at every pixel centre, float64 depth order (ties by index),
    2D covariance from a central-difference Jacobian of the projection.
    Returns the image, the transmittance and, per pixel, the Gaussian whose
    opacity ended it (-1 where none did)."""
    W, H = cam["width"], cam["height"]
    R, p = np.asarray(cam["R"]), np.asarray(cam["pos"])
    fx = W / (2 * math.tan(cam["fovx"] / 2)); fy = H / (2 * math.tan(cam["fovy"] / 2))

    def proj(x):
        t = R @ (x - p)
        return np.array([fx * t[0] / t[2] + W / 2, fy * t[1] / t[2] + H / 2])

    recs = []
    for i in range(len(alpha)):
        t = R @ (mu[i] - p)
        if t[2] <= cam["znear"] or alpha[i] < MIN_A:
            continue
        J = np.zeros((2, 3))
        h = 1e-5 * max(1.0, abs(t[2]))
        for c in range(3):
            e = np.zeros(3); e[c] = h
            J[:, c] = (proj(mu[i] + e) - proj(mu[i] - e)) / (2 * h)
        S = np.array([[cov[i, 0], cov[i, 1], cov[i, 2]], [cov[i, 1], cov[i, 3], cov[i, 4]],
                      [cov[i, 2], cov[i, 4], cov[i, 5]]])
        S2 = J @ S @ J.T + 0.3 * np.eye(2)
        if np.linalg.det(S2) <= 0:
            continue
        recs.append((t[2], i, proj(mu[i]), np.linalg.inv(S2)))
    recs.sort(key=lambda r: (r[0], r[1]))
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    T = np.ones((H, W)); Cimg = np.zeros((3, H, W)); done = np.zeros((H, W), bool)
    stopper = np.full((H, W), -1)
    for depth, i, m, Ci in recs:
        dx, dy = px - m[0], py - m[1]
        q = Ci[0, 0] * dx * dx + 2 * Ci[0, 1] * dx * dy + Ci[1, 1] * dy * dy
        a = np.minimum(0.99, alpha[i] * np.exp(-0.5 * q))
        use = (a >= MIN_A) & ~done
        stop = use & (T * (1 - a) < 1e-4)
        stopper[stop] = i
        done |= stop
        add = use & ~stop
        Cimg += np.where(add, a * T, 0.0)[None] * rgb[i][:, None, None]
        T = np.where(add, T * (1 - a), T)
    return Cimg, T, stopper


@pytest.mark.parametrize("seed,W,H", [(1, 72, 56), (2, 40, 33), (3, 96, 64)])
def test_oracle_matches_brute_force(seed, W, H):
    # Gaussians kept inside the Jacobian clamp cone (|t_x / t_z| < 1.3 tan(fov/2)).
    mu, cov, rgb, al = synth.random_gaussians(300, seed=seed, box=2.0, zc=9.0)
    cam = synth.look_camera((0.1, -0.2, 0), (0.02, 0.01, 1), (0, -1, 0), W, H, math.radians(50))
    out = oracle.render_gaussians(mu, cov, rgb, al, cam, debug=True)
    ref, Tref, stopper = brute_force(mu.astype(np.float64), cov.astype(np.float64), rgb.astype(np.float64),
                                     al.astype(np.float64), cam)
    ok = out["band"] == 0
    assert ok.mean() > 0.99
    diff = np.abs(out["image"] - ref).max(0)
    # The brute force's Jacobian is a central difference (error ~1e-9 relative).
    assert diff[ok].max() < 1e-6, diff[ok].max()
    assert np.abs(out["T"] - Tref)[ok].max() < 1e-6
    # visit counts: a pixel nothing ended visits its whole tile list; otherwise
    # the last Gaussian it visited is the one the brute force saw end it
    ntx = (W + 15) // 16
    ty, tx = np.divmod(np.arange(H * W).reshape(H, W), W)
    tile = (ty // 16) * ntx + (tx // 16)
    ne = out["n_eval"]
    length = out["ends"][tile] - out["starts"][tile]
    assert np.all(ne >= out["n_contrib"]) and np.all(ne <= length)
    free = ok & (stopper < 0)
    assert np.array_equal(ne[free], length[free])
    ended = ok & (stopper >= 0)
    assert ended.any() and free.any()
    last = out["sorted_g"][out["starts"][tile[ended]] + ne[ended] - 1]
    assert np.array_equal(last, stopper[ended])


def test_transmittance_bounds_and_monotone(tiny, tiny_cams):
    L, R = tiny_cams
    fr = oracle.render_frame(tiny, L, R)
    for eye in ("left", "right"):
        T = fr[eye]["T"]
        assert T.min() >= 1e-4 and T.max() <= 1.0
        # T = prod(1 - a) over added Gaussians <= 0.99^n... and n = 0 iff T = 1
        nc = fr[eye]["n_contrib"]
        assert np.all((nc == 0) == (T == 1.0))
        assert np.all(T <= 0.99 ** 0 + 1e-15)
    # adding a Gaussian never raises T: blending a prefix of a list leaves T >= full-list T
    mu, cov, rgb, al = synth.random_gaussians(200, seed=5, box=2.0, zc=8.0)
    cam = cam_at_origin(48, 48)
    full = oracle.render_gaussians(mu, cov, rgb, al, cam)
    part = oracle.render_gaussians(mu[:100], cov[:100], rgb[:100], al[:100], cam)
    assert np.all(part["T"] >= full["T"] - 1e-15) or (full["band"].any())


def test_mirror_symmetry_of_stereo_pair():
    W, H = 72, 40
    mu, cov, rgb, al = synth.random_gaussians(250, seed=11, box=2.0, zc=7.0)
    L, R = synth.stereo_pair((0, 0, 0), (0, 0, 1), (0, -1, 0), W, H, math.radians(60), ipd=0.3)
    mm = mu.copy(); mm[:, 0] *= -1
    mc = cov.copy(); mc[:, 1] *= -1; mc[:, 2] *= -1
    a = oracle.render_gaussians(mm, mc, rgb, al, L)
    b = oracle.render_gaussians(mu, cov, rgb, al, R)
    ok = (a["band"] == 0) & (b["band"][:, ::-1] == 0)
    d = np.abs(a["image"] - b["image"][:, :, ::-1]).max(0)
    assert d[ok].max() < 1e-12


def test_rect_min_q_against_grid_search():
    rng = np.random.default_rng(0)
    for _ in range(200):
        A = rng.standard_normal((2, 2)); S = A @ A.T + 0.3 * np.eye(2)
        Ci = np.linalg.inv(S)
        m = rng.uniform(-30, 30, 2)
        x0, y0 = rng.uniform(-20, 20, 2); x1, y1 = x0 + rng.uniform(0, 15), y0 + rng.uniform(0, 15)
        q = oracle.rect_min_q(m[0], m[1], Ci[0, 0], Ci[0, 1], Ci[1, 1], x0, x1, y0, y1)
        gx, gy = np.meshgrid(np.linspace(x0, x1, 301), np.linspace(y0, y1, 301))
        dx, dy = gx - m[0], gy - m[1]
        qq = Ci[0, 0] * dx * dx + 2 * Ci[0, 1] * dx * dy + Ci[1, 1] * dy * dy
        assert q <= qq.min() + 1e-9
        assert qq.min() - q <= 1e-3 * (1 + qq.min())


def test_tile_lists_cover_every_contributing_pixel():
    W, H = 80, 45
    mu, cov, rgb, al = synth.random_gaussians(120, seed=4, box=2.0, zc=7.0)
    cam = cam_at_origin(W, H)
    out = oracle.render_gaussians(mu, cov, rgb, al, cam, debug=True)
    pre = out["pre"]
    listed = set(zip(out["pairs_tile"][out["pairs_flags"] & 1 == 1].tolist(),
                     out["pairs_g"][out["pairs_flags"] & 1 == 1].tolist()))
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    ntx = (W + 15) // 16
    tile_of = (np.arange(H)[:, None] // 16) * ntx + np.arange(W)[None, :] // 16
    for g in np.nonzero(pre["keep"])[0]:
        m = pre["mean2d"][g]; cn = pre["conic"][g]
        dx, dy = px - m[0], py - m[1]
        q = cn[0] * dx * dx + 2 * cn[1] * dx * dy + cn[2] * dy * dy
        a = al[g] * np.exp(-0.5 * q)
        need = set(np.unique(tile_of[a >= MIN_A * (1 + 1e-9)]).tolist())
        have = {t for (t, gg) in listed if gg == g}
        assert need <= have
        tau = 2 * math.log(255 * al[g])
        for t in have:  # every listed tile's rectangle reaches the footprint
            tx, ty = t % ntx, t // ntx
            x1 = min(16 * tx + 15, W - 1) + 0.5; y1 = min(16 * ty + 15, H - 1) + 0.5
            gx, gy = np.meshgrid(np.linspace(16 * tx + 0.5, x1, 121), np.linspace(16 * ty + 0.5, y1, 121))
            ddx, ddy = gx - m[0], gy - m[1]
            qq = cn[0] * ddx * ddx + 2 * cn[1] * ddx * ddy + cn[2] * ddy * ddy
            assert qq.min() <= tau + 1e-3 * (1 + tau)


def test_sort_matches_lexsort():
    rng = np.random.default_rng(3)
    n = 5000
    tile = rng.integers(0, 50, n).astype(np.int32)
    g = rng.integers(0, 400, n).astype(np.int32)
    depth = rng.choice(rng.uniform(0.5, 30, 300), 400)  # many exact ties
    order = oracle.sort_pairs(tile, g, depth)
    ref = np.lexsort((np.arange(n), depth.astype(np.float32)[g], tile))
    assert np.array_equal(order, ref)


def test_psnr_and_maxabs_definitions():
    a = np.random.default_rng(0).uniform(0.1, 0.9, (3, 8, 8))
    assert abs(oracle.psnr(a + 0.01, a) - 40.0) < 1e-9
    assert abs(oracle.max_abs(a + 0.01, a) - 0.01) < 1e-12


# ---------------------------------------------------------------- SSIM

def test_ssim_identical_is_one():
    rng = np.random.default_rng(3)
    x = rng.random((3, 17, 23))
    assert abs(oracle.ssim(x, x) - 1.0) < 1e-12


def test_ssim_constant_images_closed_form():
    # constant images: zero variances, so SSIM = (2ab + C1) / (a^2 + b^2 + C1) at every window
    a, b = 0.3, 0.7
    c1 = 1e-4
    want = (2 * a * b + c1) / (a * a + b * b + c1)
    got = oracle.ssim(np.full((2, 12, 15), a), np.full((2, 12, 15), b))
    assert abs(got - want) < 1e-12


def test_ssim_window_sums_to_one_and_is_gaussian():
    w = oracle.ssim_window()
    assert len(w) == 11 and abs(w.sum() - 1.0) < 1e-15
    assert abs(w[6] / w[5] - math.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-12


def test_ssim_matches_direct_windows():
    # brute force: every 11 x 11 window with the 2-D Gaussian weights, no separability
    rng = np.random.default_rng(5)
    x, y = rng.random((1, 13, 14)), rng.random((1, 13, 14))
    w = oracle.ssim_window()
    w2 = np.outer(w, w)
    c1, c2 = 1e-4, 9e-4
    vals = []
    for i in range(13 - 10):
        for j in range(14 - 10):
            px, py = x[0, i:i + 11, j:j + 11], y[0, i:i + 11, j:j + 11]
            mx, my = (w2 * px).sum(), (w2 * py).sum()
            vx = (w2 * (px - mx) ** 2).sum()
            vy = (w2 * (py - my) ** 2).sum()
            cxy = (w2 * (px - mx) * (py - my)).sum()
            vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    assert abs(oracle.ssim(x, y) - float(np.mean(vals))) < 1e-12
    assert abs(oracle.ssim(x, y) - oracle.ssim(y, x)) < 1e-15
