"""GPU tests of the multi-viewer server (continuous batching).

  * every viewer's frames are bit-identical whether it is served alone or
    batched with viewers of other resolutions and trajectories, and equal to
    the single-viewer entry points (gsc_derive + gsc_render_stereo);
  * more viewers than one batch holds: all requests complete, FIFO by arrival;
  * admission against the device-memory budget: refused when it does not
    fit, admitted after a viewer leaves;
  * completion times come after submission; a batch that runs out of cache
    lines reports GSC_E_CAPACITY for its requests;
  * a mixed batch on the city scene at the serving resolutions (1280x720,
    2048x1080 and 2560x1440 per eye, each viewer on its own walk and cache),
    two batches in flight, against the FP64 oracle with its cache model,
    every frame and eye;
  * with two batches in flight the images are the same as with one.
"""
import math
import time

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


SIZES = [(128, 96), (96, 64), (160, 112), (80, 80)]


def walk(n, W, H, seed):
    rng = np.random.default_rng(seed)
    pos = np.array([rng.uniform(-2, 2), rng.uniform(-1, 1), -15.0 + rng.uniform(-2, 2)])
    ang = rng.uniform(-0.3, 0.3)
    out = []
    for _ in range(n):
        out.append(synth.stereo_pair(pos.copy(), (math.sin(ang), 0.0, math.cos(ang)), (0, -1, 0), W, H,
                                     math.radians(60), 2 * math.atan(math.tan(math.radians(30)) * H / W)))
        pos = pos + np.array([rng.uniform(-0.3, 0.3), 0.0, rng.uniform(0.0, 0.4)])
        ang += rng.uniform(-0.05, 0.05)
    return out


def scene_renderer(gs, scene, **kw):
    r = gs.Renderer(k=scene.k, reuse=True, max_width=256, max_height=256, **kw)
    r.load(scene)
    return r


def serve(gs, scene_r, viewers, budget=1 << 34, order="interleaved", overlap=False):
    """viewers: list of (W, H, frames). Submits every frame (interleaved over
    viewers, arrival times increasing), steps until all complete; returns the
    images per viewer and the completion records.  overlap: two batches in
    flight."""
    srv = gs.Server(scene_r, budget)
    if overlap:
        srv.overlap(True)
    ids, outs, arrive = [], [], {}
    for W, H, _ in viewers:
        vid = srv.admit(W, H)
        assert vid is not None
        ids.append(vid)
        outs.append([])
    n = max(len(f) for _, _, f in viewers)
    req = {}
    for t in range(n):
        for i, (W, H, frames) in enumerate(viewers):
            if t >= len(frames):
                continue
            L, R = frames[t]
            oL = torch.full((3, H, W), -1.0, device="cuda")
            oR = torch.full((3, H, W), -1.0, device="cuda")
            ta = time.monotonic()
            rid = srv.submit(ids[i], L, R, ta, oL, oR)
            arrive[rid] = ta
            req[rid] = (i, t)
            outs[i].append((oL, oR))
    done = []
    while len(done) < len(req):
        launched = srv.step()
        if launched == 0:
            torch.cuda.synchronize()
        done += srv.poll()
    torch.cuda.synchronize()
    done += srv.poll()
    assert srv.pending() == 0
    srv.close()
    return outs, done, arrive, req


@pytest.mark.parametrize("overlap", [False, True])
def test_alone_equals_mix_equals_single_viewer_path(gs, tiny, overlap):
    torch.cuda.set_device(0)
    viewers = [(W, H, walk(6, W, H, seed=10 + i)) for i, (W, H) in enumerate(SIZES[:3])]
    base = scene_renderer(gs, tiny)
    mixed, done, arrive, req = serve(gs, base, viewers, overlap=overlap)
    assert all(s == 0 for _, _, s in done)
    for i, v in enumerate(viewers):
        alone, d1, _, _ = serve(gs, base, [v], overlap=overlap)
        assert all(s == 0 for _, _, s in d1)
        ref = scene_renderer(gs, tiny)
        W, H, frames = v
        for t, (L, R) in enumerate(frames):
            a = torch.zeros(3, H, W, device="cuda"); b = torch.zeros(3, H, W, device="cuda")
            ref.frame(L, R, a, b)
            torch.cuda.synchronize()
            for eye in range(2):
                m, al = mixed[i][t][eye], alone[0][t][eye]
                assert torch.equal(m, al), (i, t, eye, (m - al).abs().max().item())
                assert torch.equal(al, (a, b)[eye]), (i, t, eye)
            assert float(mixed[i][t][0].min()) >= 0.0  # every pixel written


@pytest.mark.parametrize("overlap", [False, True])
def test_more_viewers_than_a_batch(gs, tiny, overlap):
    viewers = [(SIZES[i % 4][0], SIZES[i % 4][1], walk(3, *SIZES[i % 4], seed=40 + i)) for i in range(11)]
    base = scene_renderer(gs, tiny)
    outs, done, arrive, req = serve(gs, base, viewers, overlap=overlap)
    assert len(done) == sum(len(f) for _, _, f in viewers)
    assert all(s == 0 for _, _, s in done)
    for rid, t, s in done:
        assert t >= arrive[rid]
    # a viewer's frames complete in order
    per = {}
    for rid, t, s in sorted(done, key=lambda d: d[1]):
        i, f = req[rid]
        per.setdefault(i, []).append(f)
    for i, fs in per.items():
        assert fs == sorted(fs)
    # batches hold at most 8 viewers: with 11 viewers the first frame of the
    # three youngest viewers completes after the oldest eight's
    first = {req[rid][0]: t for rid, t, s in done if req[rid][1] == 0}
    assert max(first[i] for i in range(8)) <= min(first[i] for i in range(8, 11))


def test_budget_admission(gs, tiny):
    base = scene_renderer(gs, tiny)
    probe = gs.Server(base, 1 << 40)
    vb = probe.viewer_bytes(128, 96)
    assert vb > 0 and probe.viewer_bytes(160, 112) >= vb
    probe.overlap(True)                    # two raster sets: a larger share per viewer
    assert probe.viewer_bytes(128, 96) > vb
    probe.admit(128, 96)
    with pytest.raises(gs.GscError):       # only before viewers are admitted
        probe.overlap(False)
    probe.close()
    srv = gs.Server(base, int(1.5 * vb))
    a = srv.admit(128, 96)
    assert a is not None
    assert srv.admit(128, 96) is None  # does not fit beside the first
    srv.leave(a)
    b = srv.admit(128, 96)
    assert b is not None
    L, R = walk(1, 128, 96, seed=3)[0]
    oL = torch.zeros(3, 96, 128, device="cuda"); oR = torch.zeros(3, 96, 128, device="cuda")
    srv.submit(b, L, R, time.monotonic(), oL, oR)
    assert srv.step() == 1
    torch.cuda.synchronize()
    got = []
    for _ in range(1000):
        got += srv.poll()
        if got:
            break
        time.sleep(0.001)
    assert len(got) == 1 and got[0][2] == 0
    # a request larger than the admitted size is refused
    big = walk(1, 160, 112, seed=4)[0]
    with pytest.raises(gs.GscError):
        srv.submit(b, big[0], big[1], 0.0, oL, oR)
    srv.close()


def test_capacity_overflow_reported(gs, tiny):
    base = gs.Renderer(k=tiny.k, reuse=True, max_width=256, max_height=256, cache_capacity=64)
    base.load(tiny)
    (W, H) = SIZES[0]
    outs, done, _, _ = serve(gs, base, [(W, H, walk(2, W, H, seed=5))])
    assert [s for _, _, s in done] == [gs.GSC_E_CAPACITY] * 2


def test_mixed_city_batch_matches_oracle(gs):
    city = synth.city_scene()
    base = gs.Renderer(k=city.k, reuse=True, max_width=2560, max_height=1440)
    base.load(city)
    viewers = [(W, H, synth.city_walk(3, seed=100 + i, start=(-500.0 + 150.0 * i, -520.0 + 90.0 * i, 10.0 + 6.0 * i),
                                      width=W, height=H))
               for i, (W, H) in enumerate(synth.SERVING_RESOLUTIONS)]
    outs, done, _, _ = serve(gs, base, viewers, budget=64 << 30, overlap=True)  # the serving config's budget
    base.close()
    assert all(s == 0 for _, _, s in done)
    for i, (W, H, frames) in enumerate(viewers):
        sim = oracle.CacheSim(city.n, city.n, 10)
        lines = {}
        for t, (L, R) in enumerate(frames):
            ref = oracle.render_frame(city, L, R, cache=sim, cache_lines=lines)
            for eye, key in ((0, "left"), (1, "right")):
                rep = assert_image(outs[i][t][eye].cpu().numpy(), ref[key])
                print("\nviewer %d (%dx%d) frame %d %s: %s" % (i, W, H, t, key, rep))
