"""Warm-start network kernels (include/ctm_mlp.h) against the float64 oracle
(oracle/mlp.py) on the same seeded parameters and inputs: forward pass,
loss and gradient, one Adam step, a short training run, and the feature and
target encodings.  A ragged batch (37 rows) and the real output width (4 chi
= 256) are used.  Tolerance: 1e-12 relative (float64 on both sides; the GPU
sums in another order)."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

N_IN, N_H, N_OUT, B = 3, 64, 256, 37


def _inputs(seed):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(omlp.param_count(N_IN, N_H, N_OUT)) * 0.2
    theta = np.stack([rng.uniform(0, 2 * np.pi, B), rng.uniform(-0.5, 0.5, B)], axis=1)
    t = rng.standard_normal((B, N_OUT))
    return p, theta, t


def _net(p):
    from paper_1711_04798_amd import MLP
    return MLP(N_IN, N_H, N_OUT, p, max_batch=B)


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


def test_features_and_targets(gpu):
    p, theta, _ = _inputs(0)
    net = _net(p)
    x = net.features(theta).cpu().numpy()
    assert _rel(x, omlp.features(theta)) < 1e-15
    spec = np.abs(np.random.default_rng(1).standard_normal((5, 4, 64))) * 1e-3
    spec[:, :, 50:] = 0.0
    t = net.targets(spec).cpu().numpy()
    assert np.allclose(t, omlp.spectra_to_targets(spec), rtol=0, atol=1e-14)
    t = net.targets(spec, 1e-10).cpu().numpy()
    assert np.allclose(t, omlp.spectra_to_targets(spec, 1e-10), rtol=0, atol=1e-14)


def test_forward(gpu):
    p, theta, _ = _inputs(2)
    net = _net(p)
    x = net.features(theta)
    y = net.forward(x).cpu().numpy()
    yo, _ = omlp.forward(p, omlp.features(theta), N_H, N_OUT)
    assert _rel(y, yo) < 1e-12
    ye = net.forward(x, exp10=True).cpu().numpy()
    assert _rel(ye, 10.0 ** yo) < 1e-12


def test_loss_and_gradient(gpu):
    p, theta, t = _inputs(3)
    net = _net(p)
    x = net.features(theta)
    L, g = net.loss_grad(x, net._dev(t))
    Lo, go = omlp.loss_and_grad(p, omlp.features(theta), t, N_H, N_OUT)
    assert abs(L - Lo) <= 1e-12 * Lo
    assert _rel(g.cpu().numpy(), go) < 1e-12


def test_adam_and_training(gpu):
    p, theta, t = _inputs(4)
    net = _net(p)
    x = net.features(theta)
    td = net._dev(t)
    # one explicit step
    net.loss_grad(x, td)
    net.adam(1e-3)
    _, go = omlp.loss_and_grad(p, omlp.features(theta), t, N_H, N_OUT)
    po, mo, vo = omlp.adam_step(p, go, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    assert _rel(net.p.cpu().numpy(), po) < 1e-12
    # then 25 fused steps on the device
    hist = net.train(x, td, 25, 1e-3)
    xo = omlp.features(theta)
    losses = []
    for s in range(2, 27):
        L, go = omlp.loss_and_grad(po, xo, t, N_H, N_OUT)
        losses.append(L)
        po, mo, vo = omlp.adam_step(po, go, mo, vo, s, 1e-3)
    assert _rel(hist, losses) < 1e-10
    assert _rel(net.p.cpu().numpy(), po) < 1e-10
    assert hist[-1] < hist[0]
