"""The learned warm start's negative result, reproduced in the oracle.

The warm start predicts corner singular spectra (the targets of the learned
network).  These tests show, on the 1x1 cell with d = 2, D = 2, chi = 16,
what the spectra alone are worth, using the exact converged spectra as the
best any predictor could give:

* the diagonal start (C_i = diag(s_i), T = delta_ab delta_uu') with the exact
  spectra does not converge: it starts on a product of the auxiliary space
  with a traced physical boundary, which carries none of the lattice beyond
  the spectrum, and the corner spectra keep changing by 1e-2 per sweep;
* injecting the exact spectra into the corners of a trivial run after its
  first sweep (C <- U diag(s) V^T, singular vectors kept) saves no sweeps.
"""
import numpy as np

import synth
from oracle import ctm, obs

CUT = 1e-8


def _converged():
    A = synth.cell_tensors(0, 2, 2, 1)[0]
    cell = ctm.Cell(1, 1, [0], [A])
    env = ctm.init_trivial(cell, 16)
    sweeps, delta, ok = ctm.converge(cell, env, tol=1e-10, max_sweeps=60, cutoff=CUT)
    assert ok
    return cell, env, sweeps


def test_diag_start_with_exact_spectra_does_not_converge():
    cell, env, _ = _converged()
    spec = ctm.corner_spectra(env)
    envd = ctm.init_diag(cell, 16, spec)
    s_old = ctm.corner_spectra(envd)
    deltas = []
    for _ in range(40):
        ctm.sweep(cell, envd, cutoff=CUT)
        s_new = ctm.corner_spectra(envd)
        deltas.append(ctm.spectra_delta(s_new, s_old))
        s_old = s_new
    assert min(deltas) > 1e-3
    # and it is not at the right fixed point
    k0, kd = obs.kappa(cell, env), obs.kappa(cell, envd)
    assert abs(kd - k0) > 1e-4 * abs(k0)


def test_exact_spectrum_injection_saves_no_sweeps():
    cell, env, sweeps_plain = _converged()
    spec = ctm.corner_spectra(env)[(0, 0)]
    envi = ctm.init_trivial(cell, 16)
    ctm.sweep(cell, envi, cutoff=CUT)
    for i in range(4):
        U, _, Vh = np.linalg.svd(envi.C[i][(0, 0)])
        C = U @ np.diag(spec[i]) @ Vh
        envi.C[i][(0, 0)] = C / np.linalg.norm(C)
    sweeps, _, ok = ctm.converge(cell, envi, tol=1e-10, max_sweeps=60, cutoff=CUT)
    assert ok
    assert 1 + sweeps >= sweeps_plain - 1
    k0, ki = obs.kappa(cell, env), obs.kappa(cell, envi)
    assert abs(ki - k0) < 1e-9 * abs(k0)
