"""Pins of the oracle's reuse-predictor maths.

The analytic float64 gradients of the weighted BCE loss are checked against
central finite differences of the loss (h = 1e-6); Adam against its
closed-form first step (every parameter moves by lr * sign(grad)); the
features against hand-computable geometric cases.
"""
import numpy as np

import oracle
import synth


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = synth.predictor_init(seed=3)
    for i in range(1, 6, 2):
        params[i] = rng.uniform(-0.1, 0.1, params[i].shape)  # non-zero biases
    X = rng.standard_normal((64, oracle.PRED_FEATURES))
    y = (rng.uniform(size=64) < 0.3).astype(np.float64)
    loss, grads = oracle.pred_loss_grad(params, X, y, pos_weight=2.5)
    h = 1e-6
    for pi, P in enumerate(params):
        flat = P.reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
        for j in idx:
            old = flat[j]
            flat[j] = old + h
            lp, _ = oracle.pred_loss_grad(params, X, y, 2.5)
            flat[j] = old - h
            lm, _ = oracle.pred_loss_grad(params, X, y, 2.5)
            flat[j] = old
            num = (lp - lm) / (2 * h)
            ana = grads[pi].reshape(-1)[j]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (pi, j, num, ana)


def test_adam_first_step_is_signed_lr():
    params = [np.array([1.0, -2.0, 3.0])]
    grads = [np.array([0.5, -1e-3, 20.0])]
    m, v = [np.zeros(3)], [np.zeros(3)]
    out = oracle.adam_step(params, grads, m, v, step=1, lr=1e-3, eps=0.0)
    assert np.allclose(out[0], np.array([1.0, -2.0, 3.0]) - 1e-3 * np.sign(grads[0]), atol=1e-15)


def test_features_geometry():
    s = synth.tiny_scene(n=4)
    s.pos = np.array([[0, 0, 10], [10, 0, 0], [0, 0, 5], [3, 4, 0]], np.float32)
    s.level = np.array([0, 0, 0, 0], np.uint8)
    f = oracle.reuse_features(s, np.arange(4), pu_now=np.zeros(3), pu_then=np.zeros((4, 3)), age=np.array([1, 2, 3, 10]),
                              d_max=10, fx=100.0)
    assert np.allclose(f[:, 0], 0) and np.allclose(f[:, 1], 0) and np.allclose(f[:, 4], 0)
    assert np.allclose(f[:, 2], [0.1, 0.2, 0.3, 1.0])
    # viewing anchor (10,0,0) from (0,0,0) then from (10,0,-10): 90 degrees -> 1 - cos = 1
    f2 = oracle.reuse_features(s, np.array([1]), np.zeros(3), np.array([[10.0, 0.0, -10.0]]), [1], 10, 100.0)
    assert abs(f2[0, 0] - 1.0) < 1e-12
    assert abs(f2[0, 1] - 0.0) < 1e-12
    assert abs(f2[0, 4] - np.sqrt(200.0) / 10.0) < 1e-12
    assert abs(f2[0, 5] - np.log2(0.5 * 100.0 / 10.0)) < 1e-12


def _gauss(alpha, rgb, cov):
    return {"alpha": np.array(alpha, np.float64), "rgb": np.array(rgb, np.float64),
            "cov": np.array(cov, np.float64)}


def test_reuse_label_hand_worked():
    """Two Gaussians per anchor; each row changes one quantity by a hand-picked
    amount, so the drift and the 16/255 (~0.0627) bound are read off by eye."""
    eye = [1, 0, 0, 1, 0, 1]
    base_rgb = [[0.2, 0.4, 0.6], [0.1, 0.1, 0.1]]
    # anchor 0: nothing changes
    # anchor 1: opacity 0.30 -> 0.31 (drift 0.01)
    # anchor 2: red 0.2 -> 0.4 at opacity 0.5 (drift 0.1); its twin at 0.2 (drift 0.04)
    # anchor 3: Sigma_xx 1.0 -> 1.1 at opacity 1 (relative 0.1, drift 0.05)
    cached = _gauss([0.5, 0.5, 0.30, 0.5, 0.5, 0.5, 1.0, 0.5],
                    base_rgb * 4,
                    [eye] * 8)
    fresh = _gauss([0.5, 0.5, 0.31, 0.5, 0.5, 0.5, 1.0, 0.5],
                   base_rgb * 4,
                   [eye] * 8)
    fresh["rgb"][4, 0] = 0.4
    cached["cov"][6, 0] = 1.1
    lab = oracle.reuse_label(cached, fresh, 2, size_px=[1.0, 1.0, 1.0, 1.0])
    assert lab.tolist() == [0, 0, 1, 0]
    # footprint 3x3 px: 0.01 * 9 = 0.09 > 0.0627; 2x2 px: 0.05 * 4 = 0.2
    lab = oracle.reuse_label(cached, fresh, 2, size_px=[5.0, 3.0, 0.5, 2.0])
    assert lab.tolist() == [0, 1, 1, 1]
    # below one pixel the area counts as one: 0.04 stays below the bound
    cached["alpha"][4] = fresh["alpha"][4] = 0.2
    assert oracle.reuse_label(cached, fresh, 2, size_px=[1.0, 0.1, 0.1, 0.1]).tolist() == [0, 0, 0, 0]
    assert oracle.reuse_label(cached, fresh, 2, size_px=[1.0, 1.0, 1.3, 1.0]).tolist() == [0, 0, 1, 0]
