"""Pins of the FP64 surrogate reference: backpropagation against central finite
differences, the softmax cross-entropy gradient against its closed form, and
Adam against the minimum of a convex quadratic."""
import numpy as np

from oracle import surrogate_oracle as S


def _small(seed=3):
    sizes = (6, 9, 7, 51)
    ps = S.init_params(seed, sizes)
    g = np.random.default_rng(seed)
    ps = [p + 0.1 * g.standard_normal(p.shape) for p in ps]  # non-zero biases too
    X = g.standard_normal((5, 6))
    lab = g.integers(0, 3, 5)
    tr = g.standard_normal((5, 48))
    return ps, X, lab, tr


def test_backprop_matches_finite_differences():
    ps, X, lab, tr = _small()
    grads, L = S.gradients(ps, X, lab, tr, w_traj=0.7)
    h = 1e-6
    for k, p in enumerate(ps):
        flat = p.reshape(-1)
        idx = np.random.default_rng(k).choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = S.loss(S.forward(ps, X)[0], lab, tr, 0.7)
            flat[i] = old - h
            lm = S.loss(S.forward(ps, X)[0], lab, tr, 0.7)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (k, i)


def test_cross_entropy_gradient_closed_form():
    # two classes equal, one larger: p = softmax; dCE/dz = p - onehot
    y = np.zeros((1, 51))
    y[0, :3] = [0.0, 0.0, np.log(2.0)]
    g = S.output_gradient(y, np.array([2]), np.zeros((1, 48)))
    assert np.allclose(g[0, :3], [0.25, 0.25, -0.5], atol=1e-15)
    # the loss at the same point: -log(1/2)
    assert abs(S.loss(y, np.array([2]), np.zeros((1, 48))) - np.log(2.0)) < 1e-15


def test_relu_network_is_piecewise_linear():
    # positive homogeneity of a bias-free ReLU network: f(a x) = a f(x), a > 0
    ps = S.init_params(5)
    ps = [p if k % 2 == 0 else np.zeros_like(p) for k, p in enumerate(ps)]
    X = np.random.default_rng(1).standard_normal((4, 6))
    y1, _ = S.forward(ps, X)
    y2, _ = S.forward(ps, 3.5 * X)
    assert np.allclose(y2, 3.5 * y1, rtol=1e-12, atol=1e-12)


def test_adam_reaches_quadratic_minimum():
    # minimise 0.5 (p - c)^T D (p - c): Adam converges to c
    c = np.array([1.5, -2.0, 0.25])
    D = np.array([1.0, 10.0, 0.1])
    p = [np.zeros(3)]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    for t in range(1, 5001):
        g = [D * (p[0] - c)]
        p, m, v = S.adam_step(p, g, m, v, t, lr=0.01)
    assert np.abs(p[0] - c).max() < 1e-3


def test_adam_first_step_is_lr_sign():
    # bias correction makes the first step exactly lr * g / (|g| + eps)
    g = [np.array([3.0, -0.5])]
    p, _, _ = S.adam_step([np.zeros(2)], g, [np.zeros(2)], [np.zeros(2)], 1, lr=0.1)
    assert np.allclose(p[0], -0.1 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
