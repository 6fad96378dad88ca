"""Pins of the FP64 warm-start network reference and the feature reference (CPU)."""
from __future__ import annotations

import numpy as np

import synth
from oracle import features, mlp, wls


def _theta(F, H, rng, scale=0.5):
    return rng.normal(scale=scale, size=sum(int(np.prod(s)) for _, s in mlp.shapes(F, H)))


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    F, H, B = 5, 7, 9
    th = _theta(F, H, rng)
    X = rng.normal(size=(B, F))
    t = rng.uniform(0, 2, size=B)
    L, g = mlp.loss_and_grad(th, X, t, 0.3, 0.7, F, H)
    h = 1e-6
    fd = np.empty_like(th)
    for j in range(th.size):
        e = np.zeros_like(th)
        e[j] = h
        fd[j] = (mlp.loss_and_grad(th + e, X, t, 0.3, 0.7, F, H)[0] -
                 mlp.loss_and_grad(th - e, X, t, 0.3, 0.7, F, H)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_forward_closed_form_single_unit():
    """F = H = 1 with positive weights: every relu passes, so
    y = softplus(w3 (W2 (W1 x + b1) + b2) + b3) and lr = mean(h2) wr + br."""
    F = H = 1
    W1, b1, W2, b2, w3, b3, wr, br = 2.0, 0.5, 3.0, 0.25, 0.5, -1.0, 4.0, 0.1
    th = np.array([W1, b1, W2, b2, w3, b3, wr, br])
    X = np.array([[1.0], [2.0]])
    y, lr, _ = mlp.forward(th, X, F, H)
    h2 = W2 * (W1 * X[:, 0] + b1) + b2
    assert np.allclose(y, np.log1p(np.exp(w3 * h2 + b3)), rtol=1e-14)
    assert abs(lr - (h2.mean() * wr + br)) <= 1e-13


def test_adam_first_step_is_signed_learning_rate():
    """After one Adam step from zero moments the bias-corrected update is
    lr g / (|g| + eps): each parameter moves by almost exactly lr against the sign of g."""
    rng = np.random.default_rng(1)
    th = rng.normal(size=20)
    g = rng.normal(size=20)
    new, m, v = mlp.adam(th, g, np.zeros(20), np.zeros(20), 1, lr=1e-2)
    assert np.allclose(th - new, 1e-2 * np.sign(g), rtol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_matches_closed_form_for_constant_gradient():
    """With a constant gradient g the moments are m_k = (1-b1^k) g and
    v_k = (1-b2^k) g^2, so every bias-corrected step is lr g / (|g| + eps)."""
    th = np.array([1.0, -2.0])
    g = np.array([0.3, -0.2])
    m = v = np.zeros(2)
    x = th.copy()
    for k in range(1, 6):
        x, m, v = mlp.adam(x, g, m, v, k, lr=0.1)
    assert np.allclose(x, th - 5 * 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_spot_features_on_a_hand_built_problem():
    """Two scenarios, two spots, three voxels (target, OAR, other)."""
    from tests._helpers import problem_from_dense
    A0 = np.array([[1.0, 0.0], [1.0, 2.0], [2.0, 0.0]])
    A1 = np.array([[2.0, 0.0], [0.0, 1.0], [2.0, 1.0]])
    P = problem_from_dense([A0, A1], w=[1.0, 0.5, 0.1], p=[1.0, 0.0, 0.0])
    W = wls.from_problem(P)
    f = features.spot_features(W, np.array([1, 2, 0]))
    # spot 0: target shares 1/4 and 2/4; OAR shares 1/4 and 0; masses 4 and 4
    assert np.allclose(f[0, :5], [0.375, 0.25, 0.5, 0.125, 0.25])
    assert np.isclose(f[0, 5], np.log1p(4.0))
    # b_0 = sum_s sum_i w_i p_i a_si0 = 1 + 2; gdiag_0 = (1 + 0.5 + 0.4) + (4 + 0 + 0.4)
    assert np.isclose(f[0, 6], 3.0 / 6.3)
    # spot 1 never reaches the target: b = 0
    assert np.allclose(f[1, [0, 1, 2]], 0.0) and f[1, 6] == 0.0
    assert np.allclose(f[1, [3, 4]], [(1.0 + 0.5) / 2, 1.0])


def test_spot_features_ideal_intensity_is_single_spot_minimiser():
    """Feature 6 is the minimiser of f over spot j alone (others at zero):
    f(t e_j) is a parabola whose vertex is b_j / g_jj."""
    P = synth.make_tiny(0)
    W = wls.from_problem(P)
    vc = np.zeros(P.m, dtype=np.uint8)
    f = features.spot_features(W, vc)
    for j in (0, 17, P.n - 1):
        e = np.zeros(P.n)
        e[j] = 1.0
        t = f[j, 6]
        fm = [wls.objective(W, (t + d) * e) for d in (-1e-3, 0.0, 1e-3)]
        assert fm[1] <= fm[0] and fm[1] <= fm[2]
