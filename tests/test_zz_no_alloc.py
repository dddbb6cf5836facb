"""The allocation-free raster-only entry (gsc_render_gaussians_noalloc)
against the allocating one (gsc_render_gaussians) on the same inputs: two
calls in a row on the shared static buffer, the second with fewer
Gaussians and a smaller image, each checked against the context path's
image and transmittance (the same kernels, so the same values) and its
overflow status; plus the FP64 oracle on the first call."""
import math

import numpy as np
import pytest

import oracle
import synth
from parity import assert_image

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    return gs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def test_noalloc_matches_context_entry_twice(gs):
    cases = [(6000, 11, 200, 152), (700, 12, 96, 72)]   # second call smaller
    for i, (n, seed, W, H) in enumerate(cases):
        print("noalloc case %d: n=%d seed=%d %dx%d" % (i, n, seed, W, H), flush=True)
        mu, cov, rgb, al = synth.random_gaussians(n, seed=seed, box=3.0, zc=8.0)
        cam = synth.look_camera((0.1, -0.2, 0), (0.05, 0.02, 1), (0, -1, 0), W, H, math.radians(60))
        args = [dev(x) for x in (mu, cov, rgb, al)]
        out = torch.full((3, H, W), -1.0, device="cuda")
        T = torch.full((H, W), -1.0, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        gs.render_gaussians_noalloc(*args, cam, out, T, status)
        torch.cuda.synchronize()
        r = gs.Renderer(max_width=W, max_height=H)
        ref_out = torch.zeros(3, H, W, device="cuda")
        ref_T = torch.zeros(H, W, device="cuda")
        r.render_gaussians(*args, cam, ref_out, ref_T)
        torch.cuda.synchronize()
        r.sync()
        r.close()
        a, b = out.cpu().numpy(), ref_out.cpu().numpy()
        assert int(status.item()) == 0
        d = float(np.abs(a - b).max())
        dT = float(np.abs(T.cpu().numpy() - ref_T.cpu().numpy()).max())
        print("  max-abs vs gsc_render_gaussians: image %.3g, T %.3g" % (d, dT))
        assert d <= 1e-6 and dT <= 1e-6
        if i == 0:
            assert_image(a, oracle.render_gaussians(mu, cov, rgb, al, cam))
