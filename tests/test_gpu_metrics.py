"""GPU parity of the device SSIM (gsc_ssim) with the FP64 oracle: seeded
random images of several sizes, from the 11 x 11 minimum to sizes that leave
ragged 16 x 16 tiles of window positions; identical images; constant images
against the closed form; two rendered frames; the size limit."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    return gs


@pytest.fixture(scope="module")
def r(gs):
    rr = gs.Renderer(k=10, max_width=64, max_height=64)
    yield rr
    rr.close()


@pytest.mark.parametrize("shape", [(3, 11, 11), (1, 12, 27), (3, 37, 53), (1, 64, 64), (3, 100, 129)])
def test_ssim_matches_oracle(r, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.random(shape, dtype=np.float32)
    # a correlated second image (SSIM well inside (0, 1))
    y = np.clip(x + 0.1 * rng.standard_normal(shape).astype(np.float32), 0, 1).astype(np.float32)
    got = r.ssim(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    want = oracle.ssim(x, y)
    assert abs(got - want) < 1e-9, (shape, got, want)
    assert 0.0 < want < 1.0


def test_ssim_identical_and_constant(r):
    rng = np.random.default_rng(9)
    x = torch.from_numpy(rng.random((3, 40, 50), dtype=np.float32)).cuda()
    assert abs(r.ssim(x, x) - 1.0) < 1e-12
    a, b = float(np.float32(0.3)), float(np.float32(0.7))  # the values the float32 images hold
    want = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    ca = torch.full((2, 20, 30), a, device="cuda")
    cb = torch.full((2, 20, 30), b, device="cuda")
    assert abs(r.ssim(ca, cb) - want) < 1e-9


def test_ssim_of_rendered_frames(gs, tiny, tiny_cams):
    L, R = tiny_cams
    W, H = L["width"], L["height"]
    rr = gs.Renderer(k=tiny.k, max_width=W, max_height=H)
    rr.load(tiny)
    oL = torch.zeros(3, H, W, device="cuda"); oR = torch.zeros(3, H, W, device="cuda")
    rr.frame(L, R, oL, oR)
    rr.sync()
    torch.cuda.synchronize()
    got = rr.ssim(oL, oR)
    want = oracle.ssim(oL.cpu().numpy(), oR.cpu().numpy())
    assert abs(got - want) < 1e-9, (got, want)
    rr.close()


def test_ssim_size_limit(gs, r):
    x = torch.zeros(3, 10, 20, device="cuda")
    with pytest.raises(gs.GscError):
        r.ssim(x, x)
