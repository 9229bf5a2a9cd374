"""Boundary density operator on an infinite cylinder (Sec. IV, Eq. "Eq:rho")
through the C ABI, against the CPU oracle on the same environments and
against the closed form of the dimer state.

* dimer state (maximally entangled pairs on the horizontal bonds): every
  eigenvalue of sigma_L^T sigma_R / Tr is 1 / D^nv and S = nv ln D, on a
  1x1 and a 2x2 cell, with a flat spectrum that a single Krylov sequence
  could not resolve (every product lies in the span);
* an oracle environment imported into the GPU context (both sides then use
  the same edges): the whole spectrum (Krylov dimension D^nv) element by
  element, and the leading eigenvalues of a partial Krylov space within
  their residual estimates;
* each side's own converged environment of the same tensors: the whole
  spectrum to the convergence level.

Tolerances: on eigenvalues divided by the trace and on S, 1e-10 or ten
times the relative asymmetry of the two rings (the Lanczos treats them as
symmetric, which the exact fixed point is), whichever is larger.
"""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import boundary as obd

from test_gpu_stages import env_to_flat

pytestmark = pytest.mark.gpu


def _dimer_peps(D):
    A = np.zeros((D * D, D, D, D, D))
    for sl in range(D):
        for sr in range(D):
            A[sl * D + sr, 0, sl, 0, sr] = 1.0
    return A


@pytest.mark.parametrize("cell_kind,D,nv", [("1x1", 2, 4), ("1x1", 2, 8), ("1x1", 3, 4), ("2x2", 2, 6)])
def test_dimer_state(gpu, cell_kind, D, nv):
    from paper_1711_04798_amd import CTM
    A = _dimer_peps(D)
    print("case boundary dimer", cell_kind, D, nv, flush=True)
    if cell_kind == "1x1":
        g = CTM([[A]], chi=4)
    else:
        g = CTM([[A, A]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=4)
    g.sweep(3)
    ev, res, S, wt = g.boundary_spectrum(nv)
    g.close()
    assert np.abs(ev - D ** -nv).max() < 1e-12, ev[:4]
    assert abs(S - nv * np.log(D)) < 1e-10 and abs(wt - 1.0) < 1e-12


def _tol(cell, env, x0, nv):
    asym = 0.0
    for sg in (obd.sigma_left(cell, env, x0, nv), obd.sigma_right(cell, env, x0, nv)):
        asym = max(asym, np.abs(sg - sg.T).max() / np.abs(sg).max())
    return max(1e-10, 10 * asym)


def _oracle_env(seed, d, D, chi, sweeps):
    A, B = synth.cell_tensors(seed, d, D, 2)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, chi)
    for _ in range(sweeps):
        octm.sweep(cell, env, cutoff=1e-10)
    return [A, B], cell, env


@pytest.mark.parametrize("d,D,chi,nvs", [(2, 2, 16, (2, 4, 6)), (8, 3, 24, (2, 4))])
def test_imported_env_full_spectrum(gpu, d, D, chi, nvs):
    from paper_1711_04798_amd import CTM
    tens, cell, env = _oracle_env(40, d, D, chi, 30)
    print("case boundary imported", d, D, chi, flush=True)
    g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi)
    g.import_env(env_to_flat(env, 2, 2))
    for nv in nvs:
        for x0 in (0, 1):
            po, _ = obd.boundary_spectrum(cell, env, x0, nv)
            ev, res, S, wt = g.boundary_spectrum(nv, column=x0)
            err = np.abs(np.sort(ev)[::-1] - po).max()
            tol = _tol(cell, env, x0, nv)
            print("nv %d column %d: dim %d, max |dp| %.2e (bound %.1e), S gpu %.12f oracle %.12f, weight %.15f"
                  % (nv, x0, len(po), err, tol, S, obd.entropy(po), wt))
            assert err < tol
            assert abs(S - obd.entropy(po)) < tol
    # a partial Krylov space: the leading eigenvalues within their residuals
    nv = nvs[-1]
    po, _ = obd.boundary_spectrum(cell, env, 0, nv)
    ev, res, S, wt = g.boundary_spectrum(nv, krylov=min(len(po), 24), nev=4)
    print("partial: leading %s (oracle %s), residuals %s" % (ev, po[:4], res))
    assert np.all(np.abs(ev - po[:4]) <= res + _tol(cell, env, 0, nv))
    g.close()


@pytest.mark.parametrize("cap", [10, 100])
def test_ring_split_launches(gpu, cap):
    """The ring GEMMs split into launches of at most `cap` rows (pieces of one
    row group at cap = 10 < 27, several groups per launch at cap = 100): the
    whole spectrum against the unsplit run (the split does not change any
    element's summation) and against the oracle on the same imported
    environment (d = 8, D = 3, chi = 24, N_v = 4)."""
    import ctypes
    from paper_1711_04798_amd import CTM, binding
    lib = binding.load()
    lib.ctm_debug_set_ring_rows.argtypes = [ctypes.c_int64]
    tens, cell, env = _oracle_env(40, 8, 3, 24, 30)
    print("case boundary split", cap, flush=True)
    g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24)
    g.import_env(env_to_flat(env, 2, 2))
    ev0, _, S0, _ = g.boundary_spectrum(4)
    try:
        assert lib.ctm_debug_set_ring_rows(cap) == 0
        ev, _, S, _ = g.boundary_spectrum(4)
    finally:
        lib.ctm_debug_set_ring_rows(0)
    g.close()
    po, _ = obd.boundary_spectrum(cell, env, 0, 4)
    d_split = np.abs(ev - ev0).max()
    err = np.abs(np.sort(ev)[::-1] - po).max()
    print("cap %d: max |split - unsplit| %.2e, max |dp| vs oracle %.2e" % (cap, d_split, err))
    assert d_split <= 1e-14 and abs(S - S0) <= 1e-13
    assert err < _tol(cell, env, 0, 4)


def test_gpu_env_full_spectrum(gpu):
    """Each side converges its own environment from the same tensors (2x2,
    d = 2, D = 3, chi = 24, float64, to a change of 1e-12 per sweep), then
    the whole spectrum at nv = 4 (dimension 81): the two agree to the
    convergence level (1e-8), the GPU's own float64 CTM feeding the GPU
    boundary operator."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(41, 2, 3, 2)
    print("case boundary own environments", flush=True)
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24, cutoff=1e-10)
    sw, dl, ok = g.converge(tol=1e-12, max_sweeps=200)
    assert ok, (sw, dl)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, 24)
    so, do, oko = octm.converge(cell, env, tol=1e-12, max_sweeps=200, cutoff=1e-10)
    assert oko
    po, _ = obd.boundary_spectrum(cell, env, 0, 4)
    ev, res, S, wt = g.boundary_spectrum(4)
    g.close()
    err = np.abs(np.sort(ev)[::-1] - po).max()
    tol = max(_tol(cell, env, 0, 4), 1e-8)
    print("own environments nv 4: sweeps gpu %d oracle %d; max |dp| %.2e (bound %.1e), S gpu %.12f oracle %.12f"
          % (sw[0], so, err, tol, S, obd.entropy(po)))
    assert err < tol and abs(S - obd.entropy(po)) < tol
