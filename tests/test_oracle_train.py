"""Pins of the training-step oracle (Section 3.4 "Loss function"; Supplement
"Hyperparameters"): the SSIM map against closed forms (identical images,
constant images in the interior and at a zero-padded corner), the loss
gradient against central finite differences of the loss value, the score
weights summing to the loss, and Adam / VectorAdam against closed-form steps
and rotation equivariance. CPU only."""
import math

import numpy as np
import pytest

from oracle import train as TR

torch = pytest.importorskip("torch")


def test_window_is_a_normalised_symmetric_gaussian():
    w = TR.gaussian_window()
    assert w.shape == (11, 11)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    # ratio of centre to an axis neighbour is exp(1 / (2 sigma^2))
    assert w[5, 5] / w[5, 6] == pytest.approx(math.exp(1 / (2 * 1.5 ** 2)), rel=1e-12)


def test_ssim_of_an_image_with_itself_is_one():
    x = np.random.default_rng(0).random((23, 17, 3))
    np.testing.assert_allclose(TR.ssim_map(x, x), 1.0, atol=1e-12)


def test_ssim_of_constant_images_interior_and_corner():
    a, b = 0.7, 0.3
    x = np.full((20, 20, 3), a)
    y = np.full((20, 20, 3), b)
    S = TR.ssim_map(x, y)
    interior = (2 * a * b + TR.C1) / (a * a + b * b + TR.C1)   # sigmas vanish
    np.testing.assert_allclose(S[5:15, 5:15], interior, rtol=1e-12)
    # corner: zero padding keeps the window mass s inside the image
    g = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    g /= g.sum()
    s = g[5:].sum() ** 2
    mx, my = a * s, b * s
    vx, vy, cxy = a * a * s * (1 - s), b * b * s * (1 - s), a * b * s * (1 - s)
    corner = ((2 * mx * my + TR.C1) * (2 * cxy + TR.C2)) / ((mx * mx + my * my + TR.C1) * (vx + vy + TR.C2))
    np.testing.assert_allclose(S[0, 0], corner, rtol=1e-12)


def _loss_value(cols, tgts, lam):
    P = sum(c.shape[0] * c.shape[1] for c in cols)
    tot = 0.0
    for c, t in zip(cols, tgts):
        tot += lam * np.abs(c - t).sum() + (1 - lam) * (1 - TR.ssim_map(c, t)).sum()
    return tot / (3 * P)


def test_loss_gradient_equals_finite_differences():
    rng = np.random.default_rng(3)
    cols = [rng.random((9, 13, 3)), rng.random((7, 6, 3))]
    tgts = [rng.random((9, 13, 3)), rng.random((7, 6, 3))]
    lam = 0.8
    loss, gc, gl = TR.loss_l1_ssim(cols, tgts, lam)
    assert loss == pytest.approx(_loss_value(cols, tgts, lam), rel=1e-12)
    assert gl.sum() == pytest.approx(loss, rel=1e-12)
    h = 1e-6
    offs = [0, 9 * 13]
    for (v, y, x, c) in [(0, 0, 0, 0), (0, 4, 6, 1), (0, 8, 12, 2), (1, 3, 2, 0), (1, 6, 5, 1)]:
        if abs(cols[v][y, x, c] - tgts[v][y, x, c]) < 10 * h:
            continue
        cp = [a.copy() for a in cols]
        cm = [a.copy() for a in cols]
        cp[v][y, x, c] += h
        cm[v][y, x, c] -= h
        fd = (_loss_value(cp, tgts, lam) - _loss_value(cm, tgts, lam)) / (2 * h)
        p = offs[v] + y * cols[v].shape[1] + x
        assert gc[p, c] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_pure_l1_gradient_is_the_sign():
    rng = np.random.default_rng(4)
    c, t = rng.random((6, 5, 3)), rng.random((6, 5, 3))
    loss, gc, _ = TR.loss_l1_ssim([c], [t], lam=1.0)
    assert loss == pytest.approx(np.abs(c - t).mean(), rel=1e-12)
    np.testing.assert_allclose(gc, np.sign(c - t).reshape(-1, 3) / (3 * 30), rtol=1e-12)


def test_adam_constant_gradient_steps_are_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        p0 = p.copy()
        p, m, v = TR.adam(p, g, m, v, lr=0.01, t=t)
        # bias correction makes m_hat = g and v_hat = g^2 exactly
        np.testing.assert_allclose(p - p0, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_vector_adam_first_step_uses_the_vector_norm():
    g = np.array([3.0, 4.0, 0.0, 0.0, -1.0, 0.0])
    p, m, v = TR.adam(np.zeros(6), g, np.zeros(6), np.zeros(2), lr=0.1, t=1, vec=3)
    np.testing.assert_allclose(p, -0.1 * g / (np.repeat([5.0, 1.0], 3) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * np.array([25.0, 1.0]), rtol=1e-12)


def test_vector_adam_is_rotation_equivariant():
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    gs = [rng.standard_normal((4, 3)) for _ in range(6)]
    p1, m1, v1 = np.zeros(12), np.zeros(12), np.zeros(4)
    p2, m2, v2 = np.zeros(12), np.zeros(12), np.zeros(4)
    for t, g in enumerate(gs, start=1):
        p1, m1, v1 = TR.adam(p1, g.ravel(), m1, v1, lr=0.05, t=t, vec=3)
        p2, m2, v2 = TR.adam(p2, (g @ q.T).ravel(), m2, v2, lr=0.05, t=t, vec=3)
    np.testing.assert_allclose(p2.reshape(4, 3), p1.reshape(4, 3) @ q.T, atol=1e-12)


def test_learning_rate_decays_by_100_over_training():
    assert TR.lr_at(0.05, 0, 1000) == pytest.approx(0.05)
    assert TR.lr_at(0.05, 999, 1000) == pytest.approx(0.0005)
    assert TR.lr_at(0.05, 500, 1001) == pytest.approx(0.005)
