"""Host-side logic of the benchmark (no GPU): the algorithmic work per method
row reproduces the measurement table's per-stage byte counts at its
estimate for the city workload (|X_t| = 2.2e5 visible anchors, all missed,
|G_t| = 1.1e6 Gaussians, K = 6.6e6 tile pairs per eye, 2048x1080 per eye,
1M anchors, k = 10), and the radix pass count of a 64-bit (tile | depth)
key."""
import pytest

import bench


def test_radix_passes():
    assert bench.radix_passes(2048, 1080) == (6, 128 * 68)    # 8,704 tiles -> 14 bits -> 46 -> 6 passes
    assert bench.radix_passes(1280, 720)[0] == 6               # 3,600 tiles -> 12 bits -> 44
    assert bench.radix_passes(16, 16) == (5, 1)                # one tile: 33 bits


def test_algorithmic_work_matches_estimate_table():
    c = {"n_visible": 220000, "n_miss": 220000, "n_gauss": 1100000, "n_pairs": [6600000, 6600000],
         "n_eval": [0, 0]}
    w = bench.algorithmic_work([c], 1, 2048, 1080, 1000000, 10)
    mb = {k: v[0] / 1e6 for k, v in w.items()}
    expect = {"select": 18, "schedule": 5, "derive": 177, "compose": 13, "preprocess": 185, "scan": 18,
              "duplicate": 255, "sort": 1900, "ranges": 106, "blend": 581}
    for k, v in expect.items():
        assert mb[k] == pytest.approx(v, rel=0.06), (k, mb[k])  # the table rounds to whole MB
    assert sum(mb.values()) == pytest.approx(3300, rel=0.03)
    # all rows are HBM-bound at this size: ~0.41 ms at 8 TB/s
    t = sum(bench.row_bound_s(k, *w[k]) for k in w)
    assert t == pytest.approx(0.41e-3, rel=0.03)


def test_blend_alu_bound_when_visits_dominate():
    c = {"n_visible": 1, "n_miss": 0, "n_gauss": 1, "n_pairs": [1, 1], "n_eval": [10 ** 10, 0]}
    w = bench.algorithmic_work([c], 1, 16, 16, 1, 10)
    b, f = w["blend"]
    assert f == 20 * 10 ** 10
    assert bench.row_bound_s("blend", b, f) == pytest.approx(f / 157.3e12)
