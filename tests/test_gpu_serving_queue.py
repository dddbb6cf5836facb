"""GPU tests of the serving queue policy (Section 5's shared queue and
display rule): the pose gate queues a request only when the unified camera
moved or turned past its threshold; requests older than the timeout are
dropped unrendered (their outputs untouched) and reported as such; with
ordered delivery a frame finishing after a newer frame of its viewer was
delivered is reported expired; with the policy off nothing changes."""
import math
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W, H = 96, 64


@pytest.fixture(scope="module")
def gs():
    import paper_2502_14938_amd as gs
    gs.lib()
    return gs


@pytest.fixture(scope="module")
def scene_r(gs, tiny):
    r = gs.Renderer(k=tiny.k, reuse=True, max_width=256, max_height=256)
    r.load(tiny)
    yield r
    r.close()


def pose(x=0.0, z=-15.0, yaw=0.0):
    return synth.stereo_pair((x, 0.0, z), (math.sin(yaw), 0.0, math.cos(yaw)), (0, -1, 0), W, H,
                             math.radians(60), 2 * math.atan(math.tan(math.radians(30)) * H / W))


def outs():
    return torch.zeros(3, H, W, device="cuda"), torch.zeros(3, H, W, device="cuda")


def drain(srv):
    recs = []
    while srv.pending() > 0:
        srv.step()
        torch.cuda.synchronize()
        recs += srv.poll()
    torch.cuda.synchronize()
    return recs + srv.poll()


def test_pose_gate(gs, scene_r):
    srv = gs.Server(scene_r, 1 << 34)
    v = srv.admit(W, H)
    srv.policy(pose_m=0.01, pose_rad=0.01)
    a, b = outs()
    assert srv.submit(v, *pose(), time.monotonic(), a, b) is not None
    # the same pose and a move below the threshold are not queued
    assert srv.submit(v, *pose(), time.monotonic(), *outs()) is None
    assert srv.submit(v, *pose(x=0.005), time.monotonic(), *outs()) is None
    # a move or a turn past it is (each against the last queued pose)
    assert srv.submit(v, *pose(x=0.05), time.monotonic(), *outs()) is not None
    assert srv.submit(v, *pose(x=0.05, yaw=0.02), time.monotonic(), *outs()) is not None
    recs = drain(srv)
    assert len(recs) == 3 and all(st == gs.GSC_OK for _, _, st in recs)
    # policy off: every request is queued
    srv.policy()
    assert srv.submit(v, *pose(x=0.05, yaw=0.02), time.monotonic(), *outs()) is not None
    assert len(drain(srv)) == 1
    srv.close()


def test_timeout_drops_unrendered(gs, scene_r):
    srv = gs.Server(scene_r, 1 << 34)
    v = srv.admit(W, H)
    srv.policy(timeout_s=0.5)
    old_l, old_r = outs()
    rid_old = srv.submit(v, *pose(), time.monotonic() - 5.0, old_l, old_r)
    new_l, new_r = outs()
    rid_new = srv.submit(v, *pose(x=0.1), time.monotonic() + 5.0, new_l, new_r)
    recs = {rid: st for rid, _, st in drain(srv)}
    assert recs == {rid_old: gs.GSC_E_TIMEOUT, rid_new: gs.GSC_OK}
    assert float(old_l.abs().sum()) == 0.0 and float(old_r.abs().sum()) == 0.0  # never rendered
    assert float(new_l.abs().sum()) > 0.0
    srv.close()


def test_ordered_delivery_discards_older_frames(gs, scene_r):
    srv = gs.Server(scene_r, 1 << 34)
    v = srv.admit(W, H)
    srv.policy(ordered=True)
    t0 = time.monotonic()
    # queued in this order (FIFO per viewer) but stamped newer first: the
    # second finishes after a newer frame was delivered
    r1 = srv.submit(v, *pose(), t0 + 1.0, *outs())
    r2 = srv.submit(v, *pose(x=0.1), t0, *outs())
    r3 = srv.submit(v, *pose(x=0.2), t0 + 2.0, *outs())
    recs = {rid: st for rid, _, st in drain(srv)}
    assert recs == {r1: gs.GSC_OK, r2: gs.GSC_E_EXPIRED, r3: gs.GSC_OK}
    srv.close()


def test_policy_off_matches_plain_serving(gs, scene_r):
    # the default policy changes nothing: same images as with explicit "off"
    imgs = []
    for explicit in (False, True):
        srv = gs.Server(scene_r, 1 << 34)
        v = srv.admit(W, H)
        if explicit:
            srv.policy(pose_m=0.0, pose_rad=0.0, timeout_s=0.0, ordered=False)
        bufs = [outs() for _ in range(3)]
        t0 = time.monotonic()
        for i, (a, b) in enumerate(bufs):
            assert srv.submit(v, *pose(x=0.1 * i), t0 - 10.0 + i, a, b) is not None
        recs = drain(srv)
        assert len(recs) == 3 and all(st == gs.GSC_OK for _, _, st in recs)
        imgs.append([(a.cpu().numpy(), b.cpu().numpy()) for a, b in bufs])
        srv.close()
    for (a, b), (c, d) in zip(*imgs):
        assert np.array_equal(a, c) and np.array_equal(b, d)
