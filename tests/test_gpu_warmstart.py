"""Learned warm start, end to end on the GPU: plain CTM runs from the trivial
start produce converged corner spectra for a training set of the family
A(theta) = normalize(cos t1 A0 + sin t1 A1 + t2 A2) (d=8, D=4, chi=64); the
network is trained on them by the library's kernels; held-out members are
then converged from diagonal corners with the predicted spectra, falling back
to the trivial start where the warm start does not converge.

Asserted: training lowers the loss; the predictions beat the training-set
mean spectrum on held-out members; with the fallback every member converges
to the same environment as from the trivial start (kappa to 1e-8).  The
sweep counts with and without the warm start are printed: they are a
measurement, not a pass condition.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_warm_start_pipeline(gpu):
    from paper_1711_04798_amd import warmstart as ws
    chi, D, tol = 64, 4, 1e-10
    base = synth.warm_family(0, d=8, D=D)
    th_tr, th_te = synth.warm_thetas(1, 512), synth.warm_thetas(2, 16)
    T_tr = [synth.warm_member(base, t) for t in th_tr]
    T_te = [synth.warm_member(base, t) for t in th_te]
    print("case warm start", flush=True)
    s_tr, sw_tr, d_tr, _ = ws.converge_batch(T_tr, chi, tol, 60)
    assert (d_tr < tol).all()
    net, hist = ws.train(th_tr, s_tr, hidden=128, steps=4000, lr=2e-3)
    assert hist[-1] < 0.1 * hist[0]
    pred = ws.predict(net, th_te)
    s_tv, sw_tv, d_tv, k_tv = ws.converge_batch(T_te, chi, tol, 60)
    lg = lambda a: np.log10(np.maximum(a, ws.TARGET_FLOOR))
    err_net = np.abs(lg(pred) - lg(s_tv))[:, :, :8].mean()
    err_mean = np.abs(lg(s_tr).mean(axis=0)[None] - lg(s_tv))[:, :, :8].mean()
    s_w, sw_w, ok_w, k_w = ws.converge_with_fallback(T_te, chi, tol, 60, pred, warm_budget=2 * int(sw_tv.max()))
    print("warm start: trivial sweeps %s; warm(+fallback) sweeps %s; warm converged %d/%d; "
          "log10 spectrum error (top 8) net %.4f vs training mean %.4f"
          % (sw_tv.tolist(), sw_w.tolist(), int(ok_w.sum()), len(ok_w), err_net, err_mean), flush=True)
    assert err_net < err_mean
    assert np.max(np.abs(k_w - k_tv) / np.abs(k_tv)) < 1e-8
