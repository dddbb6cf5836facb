"""Comparison helpers shared by the GPU parity tests (test-side only)."""
import numpy as np

IMG_TOL = 1e-4


def image_report(gpu, ora, tol=IMG_TOL):
    """gpu: [3,H,W] float32; ora: oracle eye dict.  Returns a dict with the
    max-abs over unflagged pixels, the count of pixels over tol, and whether
    every such pixel is flagged by the oracle."""
    d = np.abs(np.asarray(gpu, np.float64) - ora["image"]).max(0)
    band = ora["band"] != 0
    bad = d > tol
    return {"max_unflagged": float(d[~band].max()) if (~band).any() else 0.0, "max_all": float(d.max()),
            "n_bad": int(bad.sum()), "bad_unflagged": int((bad & ~band).sum()), "n_band": int(band.sum()),
            "npx": int(d.size)}


def assert_image(gpu, ora, tol=IMG_TOL, frac=1e-4):
    r = image_report(gpu, ora, tol)
    assert r["bad_unflagged"] == 0, r
    assert r["n_bad"] <= max(2, frac * r["npx"]), r
    return r


def pairs_by_tile(pairs):
    out = {}
    for t, g in pairs:
        out.setdefault(int(t), []).append(int(g))
    return out


def assert_pairs(gpu_pairs, ora, depth):
    """gpu_pairs: [n,2] (tile, g) in sorted order.  Oracle lists decide the set
    (marginal pairs may go either way); order must be non-decreasing in depth
    except between depths within 4 float32 ulps."""
    fl = ora["pairs_flags"]
    sure = ((fl & 1) == 1) & ((fl & 2) == 0)
    must = set(zip(ora["pairs_tile"][sure].tolist(), ora["pairs_g"][sure].tolist()))
    may = set(zip(ora["pairs_tile"].tolist(), ora["pairs_g"].tolist()))
    got = set(map(tuple, np.asarray(gpu_pairs).tolist()))
    assert len(got) == len(gpu_pairs), "duplicate pairs"
    assert must <= got, "missing pairs: %s" % sorted(must - got)[:10]
    assert got <= may, "extra pairs: %s" % sorted(got - may)[:10]
    # tiles ascending
    tiles = np.asarray(gpu_pairs)[:, 0]
    assert np.all(np.diff(tiles) >= 0)
    for t, gs in pairs_by_tile(gpu_pairs).items():
        d = depth[np.asarray(gs)]
        d32 = d.astype(np.float32)
        ulp = np.spacing(d32).astype(np.float64)
        step = np.diff(d)
        ok = (step >= 0) | (np.abs(step) <= 4 * ulp[1:])
        assert ok.all(), (t, np.nonzero(~ok)[0][:5])


# ------------------------------------------------ vectorised, large inputs

def gauss_codes(G, visible, k):
    """Render-buffer entries (visible position * k + j) as anchor * k + j, an
    id that does not depend on which other anchors are visible."""
    G = np.asarray(G, np.int64)
    return np.asarray(visible, np.int64)[G // k] * k + G % k


def excluded_codes(ref, k):
    """Codes whose presence the oracle leaves open: every Gaussian of an
    anchor whose selection is in band, and every Gaussian whose opacity mask
    is in band."""
    vis = np.asarray(ref["visible"], np.int64)
    band_anchor = np.nonzero(ref["select_band"])[0].astype(np.int64)
    mb = np.nonzero(ref["mask_band"])[0].astype(np.int64)
    mask_codes = vis[mb // k] * k + mb % k
    j = np.arange(k, dtype=np.int64)
    return np.unique(np.concatenate([(band_anchor[:, None] * k + j[None, :]).reshape(-1), mask_codes]))


def assert_visible_and_buffer(vis_gpu, G_gpu, ref, k):
    """Selection (LOD + frustum) and render buffer, bit-exact outside the
    oracle's bands.  Returns the GPU's render-buffer codes."""
    band = ref["select_band"]
    ov = np.asarray(ref["visible"])
    vis_gpu = np.asarray(vis_gpu)
    assert np.all(np.diff(vis_gpu) > 0)
    assert np.array_equal(vis_gpu[band[vis_gpu] == 0], ov[band[ov] == 0])
    cg = gauss_codes(G_gpu, vis_gpu, k)
    co = gauss_codes(ref["G"], ov, k)
    assert np.all(np.diff(cg) > 0)
    ex = excluded_codes(ref, k)
    assert np.array_equal(cg[~np.isin(cg, ex)], co[~np.isin(co, ex)])
    return cg


def assert_pairs_large(gpu_pairs, codes_gpu, ora_eye, codes_ora, excluded, depth_ora):
    """Per-eye sorted tile pairs at any size.  gpu_pairs [n,2] (tile, render
    buffer index) in sorted order; the oracle's debug lists of the same eye.
    Pairs are compared as (tile, code) with code = anchor * k + j; pairs of
    excluded codes and the oracle's marginal pairs may go either way, every
    other pair must be on both sides.  Order: tiles ascending; within a tile
    the oracle's FP64 depths non-decreasing except between depths within 4
    float32 ulps (the GPU keys its sort by FP32 depth).  Returns counts."""
    gp = np.asarray(gpu_pairs, np.int64)
    tiles = gp[:, 0]
    assert np.all(np.diff(tiles) >= 0), "tiles not ascending"
    gcode = np.asarray(codes_gpu, np.int64)[gp[:, 1]]
    key_g = (tiles << 40) | gcode
    assert len(np.unique(key_g)) == len(key_g), "duplicate pairs"
    fl = ora_eye["pairs_flags"]
    ocode = np.asarray(codes_ora, np.int64)[np.asarray(ora_eye["pairs_g"], np.int64)]
    key_o = (np.asarray(ora_eye["pairs_tile"], np.int64) << 40) | ocode
    sure = ((fl & 1) == 1) & ((fl & 2) == 0) & ~np.isin(ocode, excluded)
    free_g = ~np.isin(gcode, excluded)
    missing = ~np.isin(key_o[sure], key_g)
    assert not missing.any(), ("missing pairs", int(missing.sum()), key_o[sure][missing][:5])
    extra = free_g & ~np.isin(key_g, key_o)
    assert not extra.any(), ("extra pairs", int(extra.sum()), key_g[extra][:5])
    # order within each tile, on the pairs whose Gaussian both sides hold
    pos = np.searchsorted(codes_ora, gcode)
    pos = np.minimum(pos, len(codes_ora) - 1)
    known = np.asarray(codes_ora, np.int64)[pos] == gcode
    t, d = tiles[known], np.asarray(depth_ora, np.float64)[pos[known]]
    same = t[1:] == t[:-1]
    step = d[1:] - d[:-1]
    ulp = np.spacing(d[1:].astype(np.float32)).astype(np.float64)
    bad = same & (step < 0) & (np.abs(step) > 4 * ulp)
    assert not bad.any(), ("order", int(bad.sum()), np.nonzero(bad)[0][:5])
    return {"pairs": int(len(gp)), "sure": int(sure.sum()), "marginal_or_excluded": int(len(gp) - free_g.sum())}


def mask_tiles(sort_vals) -> int:
    """Tiles the sorted (super tile, entry) items cover: the set bits of
    their 4-bit masks (value bits 28-31)."""
    m = (np.asarray(sort_vals, np.uint32) >> 28).astype(np.int64)
    return int(((m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1)).sum())


def assert_ranges_from_keys(raw_keys, raw_ranges):
    """Ranges of the sorted keys (global super-tile ids, cleared to [0, 0)
    for an empty one) against the run boundaries of the keys."""
    keys = np.asarray(raw_keys, np.int64)
    rg = np.asarray(raw_ranges, np.int64).reshape(-1, 2)
    assert np.all(np.diff(keys) >= 0), "sorted keys not ascending"
    assert len(keys) == 0 or keys[-1] < len(rg)
    t = np.arange(len(rg))
    st = np.searchsorted(keys, t, side="left")
    en = np.searchsorted(keys, t, side="right")
    nonempty = en > st
    assert np.array_equal(rg[nonempty, 0], st[nonempty])
    assert np.array_equal(rg[nonempty, 1], en[nonempty])
    assert np.all(rg[~nonempty] == 0)
    return int(nonempty.sum())
