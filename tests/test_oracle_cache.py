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
import pytest

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


@pytest.mark.parametrize("guide,cases", [
    # (nx, nm) -> next depth with D_max = 10, worked by hand
    ("linear", [((100, 0), 10), ((100, 25), 8), ((100, 5), 10), ((100, 15), 9), ((100, 100), 1), ((3, 1), 7)]),
    # halved per eighth of update rate: r = 0.12 -> 10, 0.13 -> 5, 0.25 -> 2, 0.375 -> 1, 1 -> 1
    ("exp", [((100, 0), 10), ((100, 12), 10), ((100, 13), 5), ((100, 25), 2), ((8, 3), 1), ((100, 100), 1)]),
    # steps at r = 1/8 and 3/8
    ("staged", [((100, 12), 10), ((8, 1), 5), ((100, 13), 5), ((100, 37), 5), ((8, 3), 1), ((100, 38), 1)]),
])
def test_guide_functions_worked_values(guide, cases):
    for (nx, nm), want in cases:
        assert oracle.guide_depth(guide, 10, nx, nm) == want, (guide, nx, nm)


@pytest.mark.parametrize("guide", ["linear", "exp", "staged"])
def test_guide_functions_monotone_and_bounded(guide):
    for D in (1, 2, 7, 10, 63):
        prev = D
        for nm in range(0, 201):
            d = oracle.guide_depth(guide, D, 200, nm)
            assert 1 <= d <= D and d <= prev, (guide, D, nm)
            prev = d
        assert oracle.guide_depth(guide, D, 200, 0) == D  # nothing decoded: full depth
