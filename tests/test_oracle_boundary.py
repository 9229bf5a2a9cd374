"""Pins of the oracle's boundary density operator (Sec. IV, Eq. "Eq:rho") to
facts other than itself:

* a PEPS of maximally entangled pairs on the horizontal bonds (vertical
  bonds trivial): the half-cylinder state is exactly N_v such pairs across
  the cut, so the spectrum is flat, 1 / D^N_v, and S = N_v ln D;
* a product state (D = 1): one eigenvalue 1, S = 0;
* the similarity behind Eq. "Eq:rho": sqrt(sigma_L^T) sigma_R sqrt(sigma_L^T)
  has the spectrum of sigma_L^T sigma_R (sigma_L positive semidefinite);
* random orthogonal gauges on the four bond types of the checkerboard leave
  the spectrum unchanged: both rings transform by the same orthogonal map
  on ket and bra indices.  A ring taken at the wrong column pairs edges of
  different bond types and breaks this.
"""
import numpy as np
import pytest

import synth
from oracle import ctm, models
from oracle import boundary as bd


def _dimer_peps(D):
    """A[(s_l, s_r), u, l, d, r] = delta(s_l, l) delta(s_r, r) e0_u e0_d."""
    A = np.zeros((D * D, D, D, D, D))
    for sl in range(D):
        for sr in range(D):
            A[sl * D + sr, 0, sl, 0, sr] = 1.0
    return A


def _env(cell, chi, sweeps, cutoff=1e-12):
    env = ctm.init_trivial(cell, chi)
    for _ in range(sweeps):
        ctm.sweep(cell, env, cutoff=cutoff)
    return env


@pytest.mark.parametrize("D,nv", [(2, 2), (2, 4), (3, 2), (3, 4), (2, 6)])
def test_dimer_state_entropy(D, nv):
    cell = ctm.Cell(1, 1, [0], [_dimer_peps(D)])
    env = _env(cell, 4, 3)
    p, im = bd.boundary_spectrum(cell, env, 0, nv)
    assert np.abs(im).max() == 0.0
    assert np.abs(p - D ** -nv).max() < 1e-14
    assert abs(bd.entropy(p) - nv * np.log(D)) < 1e-12


def test_dimer_state_checkerboard():
    """The same state on the 2x2 cell (A = B): both cut columns."""
    A = _dimer_peps(2)
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [A, A])
    env = _env(cell, 4, 3)
    for x0 in (0, 1):
        p, _ = bd.boundary_spectrum(cell, env, x0, 4)
        assert abs(bd.entropy(p) - 4 * np.log(2)) < 1e-12


def test_product_state_entropy():
    rng = np.random.default_rng(30)
    cell = ctm.Cell(1, 1, [0], [models.product_peps(rng.standard_normal(3))])
    env = _env(cell, 2, 2)
    p, _ = bd.boundary_spectrum(cell, env, 0, 4)
    assert p.shape == (1,) and abs(p[0] - 1.0) < 1e-14 and bd.entropy(p) == 0.0


def test_similarity_of_eq_rho():
    """For a positive semidefinite sigma_L, sqrt(sigma_L) sigma_R sqrt(sigma_L)
    and sigma_L sigma_R share their spectrum.  The CTM sigma_L is symmetric and
    positive semidefinite up to the truncation error (here ~1e-4 relative at
    chi = 12): the identity is checked on its symmetric part, and the
    oracle's spectrum of sigma_L^T sigma_R agrees with it to that level."""
    A, B = synth.cell_tensors(31, 2, 2, 2)
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = _env(cell, 12, 15)
    sl, sr = bd.sigma_left(cell, env, 0, 4), bd.sigma_right(cell, env, 0, 4)
    asym = np.abs(sl - sl.T).max() / np.abs(sl).max()
    assert asym < 1e-3
    w, V = np.linalg.eigh(0.5 * (sl + sl.T))
    assert w.min() > -1e-3 * w.max()
    ws = np.maximum(w, 0.0)
    a = V @ np.diag(ws) @ V.T
    root = V @ np.diag(np.sqrt(ws)) @ V.T
    # spec(X Y) = spec(Y X) with X = sqrt(sigma_L), Y = sqrt(sigma_L) sigma_R
    ev_sym = np.sort(np.linalg.eigvals(root @ sr @ root).real)[::-1]
    ev_prod = np.sort(np.linalg.eigvals(a @ sr).real)[::-1]
    assert np.abs(ev_sym - ev_prod).max() < 1e-12 * ev_sym.max()
    p, _ = bd.boundary_spectrum(cell, env, 0, 4)
    assert np.abs(ev_sym / ev_sym.sum() - p).max() < 10 * asym


def _orth(rng, n):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q


@pytest.mark.parametrize("x0", [0, 1])
def test_gauge_invariance_checkerboard(x0):
    A, B = synth.cell_tensors(32, 2, 2, 2)
    rng = np.random.default_rng(33)
    O1, O2, O3, O4 = [_orth(rng, 2) for _ in range(4)]
    Ag = np.einsum("suldr,uU,lL,dE,rR->sULER", A, O4, O2, O3, O1)
    Bg = np.einsum("suldr,uU,lL,dE,rR->sULER", B, O3, O1, O4, O2)
    c1 = ctm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    c2 = ctm.Cell(2, 2, [0, 1, 1, 0], [Ag, Bg])
    e1, e2 = _env(c1, 12, 8), _env(c2, 12, 8)
    for nv in (2, 4):
        p1, _ = bd.boundary_spectrum(c1, e1, x0, nv)
        p2, _ = bd.boundary_spectrum(c2, e2, x0, nv)
        assert np.abs(p1 - p2).max() < 1e-10, (nv, np.abs(p1 - p2).max())
