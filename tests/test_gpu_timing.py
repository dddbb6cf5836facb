"""GPU checks of the library's own stage timing (gsc_timing,
gsc_timing_stages, gsc_timing_read) on the tiny scene: with every stage
timed, the stage times partition each frame; with a subset, only that
subset is timed while the frame times stay available; images do not depend
on whether or what is timed."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    return gs


def run(gs, tiny, cams, frames, **timing):
    L, R = cams
    W, H = L["width"], L["height"]
    r = gs.Renderer(k=tiny.k, reuse=True, d_max=10, max_width=W, max_height=H)
    r.load(tiny)
    oL = torch.zeros(3, H, W, device="cuda"); oR = torch.zeros(3, H, W, device="cuda")
    r.timing(True, **timing)
    for _ in range(frames):
        r.frame(L, R, oL, oR)
    torch.cuda.synchronize()
    stages, frame_ms, n = r.timing_read(max_frames=frames)
    r.timing(False)
    img = (oL.cpu().numpy(), oR.cpu().numpy())
    r.close()
    return stages, frame_ms, n, img


def test_all_stages_partition_the_frame(gs, tiny, tiny_cams):
    stages, frame_ms, n, _ = run(gs, tiny, tiny_cams, 4)
    assert n == 4 and len(frame_ms) == 4
    assert set(stages) == set(gs.STAGES)
    assert all(v >= 0.0 for v in stages.values())
    assert (frame_ms > 0).all()
    # consecutive events: the stage times add up to the frames' times
    total = sum(stages.values())
    assert abs(total - float(frame_ms.sum())) <= 1e-3 * max(1.0, float(frame_ms.sum())), (total, frame_ms.sum())
    assert stages["blend"] > 0.0 and stages["preprocess"] > 0.0


def test_selected_stages_only(gs, tiny, tiny_cams):
    stages, frame_ms, n, img_sel = run(gs, tiny, tiny_cams, 3, stages=["blend"])
    assert n == 3 and (frame_ms > 0).all()
    assert stages["blend"] > 0.0
    assert all(v == 0.0 for k, v in stages.items() if k != "blend"), stages
    # the blend lies inside each frame
    assert stages["blend"] <= float(frame_ms.sum()) + 1e-6
    # what is timed does not change the images
    _, _, _, img_all = run(gs, tiny, tiny_cams, 3)
    np.testing.assert_array_equal(img_sel[0], img_all[0])
    np.testing.assert_array_equal(img_sel[1], img_all[1])
