"""Pins of the warm-start network oracle (CPU, float64): its gradient against
central finite differences of its loss, its optimiser against closed forms of
the Adam update, and its encodings against their definitions."""
import numpy as np

from oracle import mlp


def _net(seed, n_in=3, n_hidden=5, n_out=6, B=7):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.param_count(n_in, n_hidden, n_out)) * 0.7
    x = rng.standard_normal((B, n_in))
    t = rng.standard_normal((B, n_out))
    return p, x, t


def test_gradient_finite_differences():
    """Every component of the gradient against a central difference of the
    loss (truncation error O(h^2) ~ 1e-12 at h = 1e-6)."""
    p, x, t = _net(0)
    L, g = mlp.loss_and_grad(p, x, t, 5, 6)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(p + e, x, t, 5, 6)[0] - mlp.loss_and_grad(p - e, x, t, 5, 6)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())
    # the loss is the mean squared error of the forward pass
    y, _ = mlp.forward(p, x, 5, 6)
    assert abs(L - np.mean((y - t) ** 2)) < 1e-15


def test_forward_layers_by_hand():
    """One sample written out with explicit sums over the weights."""
    p, x, t = _net(1, n_in=2, n_hidden=3, n_out=2, B=1)
    W1, b1, W2, b2, W3, b3 = mlp.split(p, 2, 3, 2)
    h1 = [np.tanh(sum(x[0, i] * W1[i, j] for i in range(2)) + b1[j]) for j in range(3)]
    h2 = [np.tanh(sum(h1[i] * W2[i, j] for i in range(3)) + b2[j]) for j in range(3)]
    y = [sum(h2[i] * W3[i, j] for i in range(3)) + b3[j] for j in range(2)]
    got, _ = mlp.forward(p, x, 3, 2)
    assert np.allclose(got[0], y, rtol=0, atol=1e-15)


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p0, g = rng.standard_normal(11), rng.standard_normal(11)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(11), np.zeros(11), 1, 0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient():
    """With a constant gradient both bias-corrected moments are exact, so every
    step moves by the same -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p, g = rng.standard_normal(5), rng.standard_normal(5)
    m = v = np.zeros(5)
    q = p.copy()
    for s in range(1, 21):
        q, m, v = mlp.adam_step(q, g, m, v, s, 0.003)
    assert np.allclose(q, p - 20 * 0.003 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_encodings():
    spec = np.array([[[0.5, 0.3, 0.2, 0.0]] * 4])
    t = mlp.spectra_to_targets(spec)
    assert t.shape == (1, 16)
    assert t[0, 3] == np.log10(mlp.FLOOR) and abs(t[0, 0] - np.log10(0.5)) < 1e-16
    back = mlp.targets_to_spectra(t, 4)
    assert np.allclose(back[0, :, :3], spec[0, :, :3], rtol=1e-15)
    x = mlp.features(np.array([[0.0, 0.25], [np.pi / 2, -0.5]]))
    assert np.allclose(x, [[1.0, 0.0, 0.25], [0.0, 1.0, -0.5]], atol=1e-16)


def test_training_reduces_loss():
    """Full-batch Adam on a smooth target of the features fits it."""
    rng = np.random.default_rng(4)
    theta = np.stack([rng.uniform(0, 2 * np.pi, 64), rng.uniform(-0.5, 0.5, 64)], axis=1)
    x = mlp.features(theta)
    t = np.stack([np.sin(2 * theta[:, 0]), theta[:, 1] ** 2, np.cos(theta[:, 0]) * theta[:, 1]], axis=1)
    n_h = 16
    p = rng.standard_normal(mlp.param_count(3, n_h, 3)) * 0.3
    m = v = np.zeros_like(p)
    L0, _ = mlp.loss_and_grad(p, x, t, n_h, 3)
    for s in range(1, 1501):
        L, g = mlp.loss_and_grad(p, x, t, n_h, 3)
        p, m, v = mlp.adam_step(p, g, m, v, s, 0.01)
    assert L < 1e-2 * L0
