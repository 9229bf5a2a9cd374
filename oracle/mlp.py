"""Oracle: the warm-start network (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; the warm start is a form beyond it.  A
three-layer perceptron maps the parameters theta = (t1, t2) of a family of
PEPS tensors to the log10 of the normalised singular values of the four
corner matrices of the converged environment, which then initialise diagonal
corners (the CTM_INIT_DIAG start of the library).

Definitions used here (the GPU kernels implement the same ones):
* input features x = (cos t1, sin t1, t2): t1 is an angle, so it enters
  through its cosine and sine;
* layers h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3, with
  W_l stored [fan_in][fan_out] and all parameters in one flat vector in the
  order W1, b1, W2, b2, W3, b3;
* loss L = mean over the batch and the outputs of (y - target)^2;
* optimiser: Adam (Kingma & Ba, "Adam: a method for stochastic optimization",
  ICLR 2015, Algorithm 1) with bias-corrected moment estimates, on the full
  training set each step;
* targets: t = log10(max(s, floor)) for the normalised spectrum s of each
  corner, chi values per corner, corners C1..C4 in order (4 chi outputs);
  the floor (1e-16 by default) hides values below the resolution of the
  environment.
"""
import numpy as np

__all__ = [
    "features", "param_count", "split", "forward", "loss_and_grad", "adam_step",
    "spectra_to_targets", "targets_to_spectra", "FLOOR",
]

FLOOR = 1e-16


def features(theta):
    """theta [B, 2] -> x [B, 3] = (cos t1, sin t1, t2)."""
    theta = np.asarray(theta, dtype=np.float64)
    return np.stack([np.cos(theta[:, 0]), np.sin(theta[:, 0]), theta[:, 1]], axis=1)


def param_count(n_in, n_hidden, n_out):
    return n_in * n_hidden + n_hidden + n_hidden * n_hidden + n_hidden + n_hidden * n_out + n_out


def split(p, n_in, n_hidden, n_out):
    """Views W1, b1, W2, b2, W3, b3 into the flat parameter vector."""
    shapes = [(n_in, n_hidden), (n_hidden,), (n_hidden, n_hidden), (n_hidden,), (n_hidden, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    assert o == p.size
    return out


def forward(p, x, n_hidden, n_out):
    """Returns y and the activations (h1, h2) needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = split(p, x.shape[1], n_hidden, n_out)
    h1 = np.tanh(x @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    y = h2 @ W3 + b3
    return y, (h1, h2)


def loss_and_grad(p, x, t, n_hidden, n_out):
    """Mean squared error and its gradient with respect to p (chain rule,
    layer by layer from the output back)."""
    B = x.shape[0]
    W1, b1, W2, b2, W3, b3 = split(p, x.shape[1], n_hidden, n_out)
    y, (h1, h2) = forward(p, x, n_hidden, n_out)
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / (B * n_out)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dz2 = (dy @ W3.T) * (1.0 - h2 * h2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 * h1)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
    return L, g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def spectra_to_targets(spec, floor=FLOOR):
    """Normalised spectra [..., 4, chi] -> log10 targets [..., 4 chi]."""
    spec = np.asarray(spec, dtype=np.float64)
    t = np.log10(np.maximum(spec, floor))
    return t.reshape(t.shape[:-2] + (-1,))


def targets_to_spectra(y, chi):
    """log10 outputs [..., 4 chi] -> spectra [..., 4, chi]."""
    y = np.asarray(y, dtype=np.float64)
    return (10.0 ** y).reshape(y.shape[:-1] + (4, chi))
