"""Pins of the oracle's derived-Gaussian cache (Section 4, Alg. 1, eq. 4).

  * a hand-worked seven-frame script (tests/golden/cache_script.json) fixes
    hits, misses, evictions and the depth sequence;
  * a static camera makes every cached frame bit-identical to the uncached
    render (the view, hence every derivation, is unchanged);
  * reuse switched off is identical to no cache;
  * |hits| + |misses| = |visible| and depths stay in [1, D_max] on a walk.
"""
import json
import os

import numpy as np

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cache_script.json")


def test_cache_hand_script():
    spec = json.load(open(GOLD))
    sim = oracle.CacheSim(spec["n_anchors"], spec["capacity"], spec["d_max"])
    for fr in spec["frames"]:
        vis = np.array(fr["visible"], np.int64)
        stale = np.isin(vis, fr["stale"]) if fr["stale"] else None
        r = sim.frame(vis, stale)
        assert sorted(vis[r["hit"]].tolist()) == fr["hits"], fr["why"]
        assert r["misses"].tolist() == fr["misses"], fr["why"]
        assert sorted(r["evicted"].tolist()) == fr["evicted"], fr["why"]
        assert r["d_used"] == fr["d_used"] and r["d_next"] == fr["d_next"], fr["why"]


def test_static_camera_cache_is_identical(tiny, tiny_cams):
    L, R = tiny_cams
    ref = oracle.render_frame(tiny, L, R)
    sim = oracle.CacheSim(tiny.n, tiny.n, 10)
    lines = {}
    for f in range(3):
        fr = oracle.render_frame(tiny, L, R, cache=sim, cache_lines=lines)
        assert np.array_equal(fr["left"]["image"], ref["left"]["image"])
        assert np.array_equal(fr["right"]["image"], ref["right"]["image"])
        if f > 0:
            assert fr["cache"]["n_miss"] == 0


def test_reuse_off_equals_no_cache(tiny):
    traj = [synth.stereo_pair((0.05 * i, 0.0, -15.0), (0.01 * i, 0, 1), (0, -1, 0), 128, 96, 1.0) for i in range(3)]
    sim = oracle.CacheSim(tiny.n, tiny.n, 10, reuse=False)
    lines = {}
    for L, R in traj:
        fr = oracle.render_frame(tiny, L, R, cache=sim, cache_lines=lines)
        ref = oracle.render_frame(tiny, L, R)
        assert fr["cache"]["n_miss"] == fr["cache"]["n_visible"]
        assert np.array_equal(fr["left"]["image"], ref["left"]["image"])


def test_cache_counts_and_depth_range():
    rng = np.random.default_rng(0)
    n, C = 400, 260
    sim = oracle.CacheSim(n, C, 10)
    centre = 100
    for t in range(60):
        centre += int(rng.integers(0, 6))
        vis = np.unique(np.clip(rng.integers(centre - 100, centre + 100, 220), 0, n - 1))
        r = sim.frame(vis)
        assert r["hit"].sum() + r["n_miss"] == len(vis)
        assert 1 <= r["d_next"] <= 10
        used = sim.line_anchor >= 0
        assert np.all(sim.tau[used] <= t)
        assert np.all(t - sim.tau[used] <= r["d_used"])
        # every visible anchor now owns a line that maps back to it
        assert np.all(sim.line_anchor[sim.slot_of[vis]] == vis)
