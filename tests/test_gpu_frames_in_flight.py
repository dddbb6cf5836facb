"""GPU checks of two frames in flight (gsc_pipeline): along a walk on the
tiny scene, frames rendered with each blend overlapping the next frame's
earlier stages give images bit-identical to the sequential order (each frame
into buffers of its own, one synchronisation at the end), for the
direct-mapped and the evicting cache; the last frame's statistics and the
frame timing agree; switching the mode off restores the sequential path."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H = 128, 96


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    return gs


def walk(n, step=0.3, turn=0.03):
    out = []
    for i in range(n):
        ang = turn * i
        out.append(synth.stereo_pair((step * i, 0.1 * math.sin(i), -15.0 + 0.05 * i), (math.sin(ang), 0.0, math.cos(ang)),
                                     (0, -1, 0), W, H, math.radians(60), math.radians(50)))
    return out


def pan(n, fov=20.0, step=0.2):
    # with 1004 lines the pan must evict, while every visible anchor still fits
    out = []
    for i in range(n):
        ang = -0.9 + step * i
        out.append(synth.stereo_pair((0, 0, -12.0), (math.sin(ang), 0, math.cos(ang)), (0, -1, 0), W, H,
                                     math.radians(fov), math.radians(fov * 0.75)))
    return out


def renderer(gs, tiny, capacity):
    r = gs.Renderer(k=tiny.k, reuse=True, d_max=10, max_width=W, max_height=H, cache_capacity=capacity)
    r.load(tiny)
    r.count_work(True)
    return r


def render_all(r, traj, sync_each):
    outs = []
    for L, R in traj:
        oL = torch.zeros(3, H, W, device="cuda"); oR = torch.zeros(3, H, W, device="cuda")
        r.frame(L, R, oL, oR)
        if sync_each:
            r.sync()
        outs.append((oL, oR))
    r.sync()
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in outs]


STAT_KEYS = ("n_visible", "n_miss", "n_gauss", "n_pairs", "n_eval", "n_contrib", "depth_used", "depth_next")


@pytest.mark.parametrize("path,capacity", [("walk", 0), ("pan", 1004)], ids=["direct", "evicting"])
def test_frames_in_flight_match_sequential(gs, tiny, path, capacity):
    traj = walk(9) if path == "walk" else pan(10)
    r = renderer(gs, tiny, capacity)
    seq = render_all(r, traj, sync_each=True)
    st_seq = r.stats()
    r.close()

    r = renderer(gs, tiny, capacity)
    r.pipeline(True)
    pipe = render_all(r, traj, sync_each=False)
    st_pipe = r.stats()
    r.close()
    for i, ((a, b), (c, d)) in enumerate(zip(seq, pipe)):
        assert np.array_equal(a, c) and np.array_equal(b, d), i
    assert any(img.max() > 0 for img, _ in seq)
    for k in STAT_KEYS:
        assert np.array_equal(np.asarray(st_seq[k]), np.asarray(st_pipe[k])), k
    if capacity:
        assert st_seq["overflow"] == 0


def test_timing_and_switch_off(gs, tiny):
    traj = walk(6)
    r = renderer(gs, tiny, 0)
    r.pipeline(True)
    r.timing(True)
    render_all(r, traj[:4], sync_each=False)
    stages, frame_ms, n = r.timing_read(max_frames=4)
    r.timing(False)
    assert n == 4 and (frame_ms > 0).all(), frame_ms
    assert stages["blend"] > 0.0 and stages["preprocess"] > 0.0
    # the rest of the walk sequentially, against a renderer that never pipelined
    r.pipeline(False)
    tail = render_all(r, traj[4:], sync_each=True)
    r.close()
    ref = renderer(gs, tiny, 0)
    want = render_all(ref, traj, sync_each=True)[4:]
    ref.close()
    for (a, b), (c, d) in zip(tail, want):
        assert np.array_equal(a, c) and np.array_equal(b, d)


def test_needs_a_scene(gs, tiny):
    r = gs.Renderer(k=tiny.k, max_width=W, max_height=H)
    with pytest.raises(Exception):
        r.pipeline(True)
    r.close()
