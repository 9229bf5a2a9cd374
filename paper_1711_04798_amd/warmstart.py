"""Learned warm start of the CTM environment (argument marshalling only).

A three-layer perceptron (include/ctm_mlp.h) maps the parameters theta of a
family of PEPS tensors to the normalised corner spectra of the converged
environment.  Plain CTM from the trivial start produces the training targets;
the predicted spectra then start diagonal corners (CTM_INIT_DIAG).  Every
computation runs in libctm.so; this module only batches the calls.
"""
import numpy as np

from .binding import CTM, MLP

# converged-environment runs: float64 contractions, fixed-count warm-started
# subspace iteration (so that a sweep can be one captured graph), relative
# cutoff 1e-8 (below it the kept directions are float64 noise and the
# spectra never settle to 1e-10)
DEFAULT_SOLVER = dict(prec="fp64", max_iters=3, resid_tol=0.0, cutoff=1e-8)


def converge_batch(tensors, chi, tol, max_sweeps, spectra=None, batch=256, use_graph=True, device="cuda:0",
                   **solver):
    """Converge the 1x1-cell environment of every tensor, `batch` instances per
    context.  spectra [N, 4, chi] (optional) starts diagonal corners.

    Returns (spectra [N, 4, chi], sweeps [N], deltas [N], kappa [N])."""
    opts = dict(DEFAULT_SOLVER)
    opts.update(solver)
    N = len(tensors)
    out_s = np.zeros((N, 4, chi))
    out_sw = np.zeros(N, dtype=np.int64)
    out_d = np.zeros(N)
    out_k = np.zeros(N)
    for i0 in range(0, N, batch):
        part = tensors[i0:i0 + batch]
        n = len(part)
        kw = {}
        if spectra is not None:
            kw = dict(init="diag", spectrum=np.asarray(spectra[i0:i0 + n], dtype=np.float64).reshape(n, 1, 4, chi))
        g = CTM([[A] for A in part], chi=chi, use_graph=use_graph, device=device, **kw, **opts)
        sw, dl, _ = g.converge(tol=tol, max_sweeps=max_sweeps)
        for j in range(n):
            out_s[i0 + j] = g.spectra(j)[0]
            out_k[i0 + j] = g.norm(j)
        out_sw[i0:i0 + n] = sw
        out_d[i0:i0 + n] = dl
        g.close()
    return out_s, out_sw, out_d, out_k


def converge_injected(tensors, chi, tol, max_sweeps, spectra, pre_sweeps=1, batch=256, use_graph=True,
                      device="cuda:0", **solver):
    """The other reading of a spectrum warm start: every run starts trivially,
    takes `pre_sweeps` sweeps, then its corners get the given singular values
    (vectors kept, ctm_set_corner_spectra) and it converges from there.

    Returns (spectra, sweeps including the pre-sweeps, deltas, kappa)."""
    opts = dict(DEFAULT_SOLVER)
    opts.update(solver)
    N = len(tensors)
    out_s = np.zeros((N, 4, chi))
    out_sw = np.zeros(N, dtype=np.int64)
    out_d = np.zeros(N)
    out_k = np.zeros(N)
    for i0 in range(0, N, batch):
        part = tensors[i0:i0 + batch]
        n = len(part)
        g = CTM([[A] for A in part], chi=chi, use_graph=use_graph, device=device, **opts)
        g.converge(tol=0.0, max_sweeps=pre_sweeps)
        for j in range(n):
            g.set_corner_spectra(np.asarray(spectra[i0 + j], dtype=np.float64).reshape(1, 4, chi), inst=j)
        sw, dl, _ = g.converge(tol=tol, max_sweeps=max_sweeps)
        for j in range(n):
            out_s[i0 + j] = g.spectra(j)[0]
            out_k[i0 + j] = g.norm(j)
        out_sw[i0:i0 + n] = np.asarray(sw) + pre_sweeps
        out_d[i0:i0 + n] = dl
        g.close()
    return out_s, out_sw, out_d, out_k


def init_params(seed, n_in, n_hidden, n_out):
    """Initial parameters drawn on the host (normal, scaled by 1/sqrt(fan_in);
    biases zero), in the flat order W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
        parts.append(rng.standard_normal(fi * fo) / np.sqrt(fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


# corner-spectrum values below this fraction of the total are at the noise
# level of a float64 environment with relative cutoff 1e-8 and are not fitted
TARGET_FLOOR = 1e-10


def train(theta, spectra, hidden=128, steps=4000, lr=2e-3, seed=0, floor=TARGET_FLOOR, device="cuda:0"):
    """Full-batch Adam on the device; returns (network, loss history)."""
    theta = np.asarray(theta, dtype=np.float64)
    N, _, chi = spectra.shape
    net = MLP(3, hidden, 4 * chi, init_params(seed, 3, hidden, 4 * chi), max_batch=N, device=device)
    x = net.features(theta)
    t = net.targets(spectra, floor)
    hist = net.train(x, t, steps, lr)
    return net, hist


def converge_with_fallback(tensors, chi, tol, max_sweeps, spectra, warm_budget, **kw):
    """Warm-started runs (diagonal corners from `spectra`) limited to
    `warm_budget` sweeps; every instance that has not converged by then is
    run again from the trivial start (the plain method is the fallback).

    Returns (spectra, sweeps spent in total, converged-from-warm mask, kappa)."""
    s_w, sw_w, d_w, k_w = converge_batch(tensors, chi, tol, warm_budget, spectra=spectra, **kw)
    ok = d_w < tol
    total = sw_w.astype(np.int64).copy()
    out_s, out_k = s_w.copy(), k_w.copy()
    bad = np.nonzero(~ok)[0]
    if bad.size:
        s_t, sw_t, d_t, k_t = converge_batch([tensors[i] for i in bad], chi, tol, max_sweeps, **kw)
        out_s[bad], out_k[bad] = s_t, k_t
        total[bad] += sw_t
    return out_s, total, ok, out_k


def predict(net, theta):
    """Predicted normalised spectra [N, 4, chi] for parameters theta [N, 2]."""
    theta = np.asarray(theta, dtype=np.float64)
    x = net.features(theta)
    y = net.forward(x, exp10=True).cpu().numpy()
    return y.reshape(len(theta), 4, -1)
