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
