"""GPU parity of the raster-only entry (gsc_render_gaussians) against the
FP64 oracle: closed-form image, random anisotropic scenes with ragged tiles,
tile lists and their order, empty and fully culled inputs, and the
full-64-bit-key sort mode."""
import math

import numpy as np
import pytest

import oracle
import synth
from parity import assert_image, assert_pairs, assert_ranges_from_keys, mask_tiles

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    assert torch.cuda.is_available()
    return gs


def run(gs, mu, cov, rgb, al, cam, full_key=False):
    W, H = cam["width"], cam["height"]
    r = gs.Renderer(max_width=W, max_height=H, full_key_sort=full_key)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    out = torch.zeros(3, H, W, device="cuda")
    T = torch.zeros(H, W, device="cuda")
    nc = torch.zeros(H, W, dtype=torch.int32, device="cuda")
    r.render_gaussians(dev(mu), dev(cov), dev(rgb), dev(al), cam, out, T, nc)
    torch.cuda.synchronize()
    r.sync()
    pairs = r.debug("pairs") if len(al) else np.zeros((0, 2), np.int32)
    return out.cpu().numpy(), T.cpu().numpy(), nc.cpu().numpy(), pairs, r


def test_single_gaussian_closed_form(gs):
    cam = synth.look_camera((0, 0, 0), (0, 0, 1), (0, -1, 0), 64, 64, math.radians(60), math.radians(60))
    mu = np.array([[0.0, 0.0, 5.0]]); cov = np.array([[0.01, 0, 0, 0.01, 0, 0.01]])
    rgb = np.array([[0.2, 0.5, 0.9]]); al = np.array([0.8])
    img, T, nc, pairs, _ = run(gs, mu, cov, rgb, al, cam)
    ref = oracle.render_gaussians(mu, cov, rgb, al, cam)
    assert np.abs(img - ref["image"]).max() < 1e-5
    assert np.abs(T - ref["T"]).max() < 1e-5


@pytest.mark.parametrize("n,seed,W,H", [(300, 1, 72, 56), (2000, 2, 130, 97), (5000, 3, 256, 256), (1, 4, 17, 9)])
def test_random_scene_matches_oracle(gs, n, seed, W, H):
    mu, cov, rgb, al = synth.random_gaussians(n, seed=seed, box=3.0, zc=8.0)
    cam = synth.look_camera((0.1, -0.2, 0), (0.05, 0.02, 1), (0, -1, 0), W, H, math.radians(60))
    img, T, nc, pairs, _ = run(gs, mu, cov, rgb, al, cam)
    ref = oracle.render_gaussians(mu, cov, rgb, al, cam, debug=True)
    rep = assert_image(img, ref)
    ok = ref["band"] == 0
    assert np.abs(T - ref["T"])[ok].max() <= 1e-4
    assert np.array_equal(nc[ok], ref["n_contrib"][ok])
    assert_pairs(pairs, ref, ref["pre"]["depth"])
    print(rep)


def test_empty_and_culled(gs):
    cam = synth.look_camera((0, 0, 0), (0, 0, 1), (0, -1, 0), 40, 24, math.radians(60))
    img, T, nc, pairs, _ = run(gs, np.zeros((0, 3)), np.zeros((0, 6)), np.zeros((0, 3)), np.zeros(0), cam)
    assert np.all(img == 0) and np.all(T == 1) and np.all(nc == 0)
    mu, cov, rgb, al = synth.random_gaussians(100, seed=9, box=1.0, zc=-5.0)  # all behind the camera
    img, T, nc, pairs, _ = run(gs, mu, cov, rgb, al, cam)
    assert np.all(img == 0) and np.all(T == 1) and len(pairs) == 0


def test_full_key_sort_gives_same_order(gs):
    mu, cov, rgb, al = synth.random_gaussians(3000, seed=5, box=3.0, zc=8.0)
    cam = synth.look_camera((0, 0, 0), (0, 0, 1), (0, -1, 0), 200, 150, math.radians(60))
    a = run(gs, mu, cov, rgb, al, cam, full_key=False)
    b = run(gs, mu, cov, rgb, al, cam, full_key=True)
    assert np.array_equal(a[3], b[3])
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("seed", [21, 22])
def test_large_footprints_match_oracle(gs, seed):
    # Gaussians 0.3-3 m in front of the camera with metre-scale covariances:
    # footprints span tens of tiles, many cross the image border, the image
    # is 200x120 so the last tile column and row are clipped.
    mu, cov, rgb, al = synth.random_gaussians(400, seed=seed, box=2.5, zc=1.8, s_lo=0.05, s_hi=1.2)
    cam = synth.look_camera((0, 0, 0), (0, 0, 1), (0, -1, 0), 200, 120, math.radians(90))
    img, T, nc, pairs, _ = run(gs, mu, cov, rgb, al, cam)
    ref = oracle.render_gaussians(mu, cov, rgb, al, cam, debug=True)
    assert ref["n_pairs"] > 20 * 400 * 0.2
    assert_image(img, ref)
    assert_pairs(pairs, ref, ref["pre"]["depth"])


def test_many_tiles_two_pass_sort_and_ranges(gs):
    # 1000x560: 63 x 35 tiles, 32 x 18 = 576 super tiles, so the sort takes
    # two radix passes (8 + 2 bits); the item count is not a multiple of
    # 1024, so the ranges see both their full 1024-key steps and the ragged
    # tail; the odd tile counts leave a half-filled super tile at the right
    # and bottom edges
    mu, cov, rgb, al = synth.random_gaussians(40000, seed=6, box=6.0, zc=12.0, s_hi=0.25)
    cam = synth.look_camera((0.1, -0.2, 0), (0.05, 0.02, 1), (0, -1, 0), 1000, 560, math.radians(70))
    img, T, nc, pairs, r = run(gs, mu, cov, rgb, al, cam)
    keys = r.debug("sort_keys")
    vals = r.debug("sort_vals")
    ranges = r.debug("raw_ranges")
    ref = oracle.render_gaussians(mu, cov, rgb, al, cam, debug=True)
    assert len(ranges) == 32 * 18 and keys.max() >= 256
    assert len(vals) == len(keys) and mask_tiles(vals) == len(pairs)
    assert len(keys) % 1024 != 0 and len(pairs) > 100000, (len(keys), len(pairs))
    assert_ranges_from_keys(keys, ranges)
    assert_pairs(pairs, ref, ref["pre"]["depth"])
    assert_image(img, ref)
    r.close()
