"""Pins of the oracle's simple update (oracle/su.py) to facts other than
itself: an untruncated bond update is the gate applied to the two-site state
(brute force); the Heisenberg chain reaches the Bethe-ansatz energy within
the truncation error of its bond dimension, from above (the energy is that
of the state, evaluated by CTM); the classical ferromagnet ends in a product
state of energy -1 per bond; a bond whose Hamiltonian is zero (the ruby
model's B -> A horizontal link) keeps a rank-1 leg rank 1 (the trivial legs
of Fig. 2)."""
import numpy as np
import pytest

from oracle import ctm as octm
from oracle import models, obs, su

SX, SZ = models.SX, models.SZ
SYSY = np.real(np.kron(models.SY, models.SY))
HEIS = 0.25 * (np.kron(SX, SX) + SYSY + np.kron(SZ, SZ))
E_BETHE = 0.25 - np.log(2.0)  # energy per bond of the spin-1/2 Heisenberg chain


def _two_site(T, lam, bond):
    """Psi[(s, other legs) of the first site, (s, other legs) of the second]
    with every weight multiplied in (brute force over the bond index)."""
    (t1, p1), (t2, p2) = su.ENDS[bond]
    parts = []
    for t, p in ((t1, p1), (t2, p2)):
        X = T[t]
        for leg in range(1, 5):
            if leg == p:
                continue
            shape = [1] * 5
            shape[leg] = -1
            X = X * lam[su.LEG_BOND[t][leg]].reshape(shape)
        parts.append(np.moveaxis(X, p, -1))
    X, Y = parts
    return np.einsum("abcdp,p,efghp->abcdefgh", X, lam[bond], Y)


def test_untruncated_update_is_the_gate():
    """A bond of rank 1 (a product state across it) gains rank at most d^2 <= D
    from one gate: no truncation, and the new two-site state is exactly the
    gate applied to the old one (up to normalisation)."""
    rng = np.random.default_rng(1)
    d, D = 2, 4
    T = [rng.standard_normal((d, D, D, D, D)) for _ in range(2)]
    lam = {b: np.sort(rng.uniform(0.2, 1.0, D))[::-1] for b in su.BONDS}
    lam["h0"] = np.array([1.0, 0.0, 0.0, 0.0])
    T[0][:, :, :, :, 1:] = 0.0   # A.r restricted to index 0
    T[1][:, :, 1:, :, :] = 0.0   # B.l restricted to index 0
    G = rng.standard_normal((d * d, d * d))
    old = _two_site(T, lam, "h0")
    # Psi axes: (s, three other legs) of A, then of B; the gate acts on the two s
    want = np.einsum("ijkl,kbcdlfgh->ibcdjfgh", G.reshape(d, d, d, d), old)
    su.bond_update(T, lam, "h0", G, D)
    new = _two_site(T, lam, "h0")
    err = np.abs(new / np.linalg.norm(new) - want / np.linalg.norm(want)).max()
    assert err < 1e-12
    assert np.count_nonzero(lam["h0"]) <= d * d


def _chain_state(D, seed=3):
    rng = np.random.default_rng(seed)
    T = [rng.standard_normal((2, D, D, D, D)) for _ in range(2)]
    for X in T:
        X[:, 1:, :, :, :] = 0.0   # vertical legs of dimension one
        X[:, :, :, 1:, :] = 0.0
    lam = su.init_weights(D, {"v0": 1, "v1": 1})
    return T, lam


def _cell_energy(T, lam, bond_h, chi, sweeps):
    cell = octm.Cell(2, 2, [0, 1, 1, 0], su.peps_tensors(T, lam))
    env = octm.init_trivial(cell, chi)
    # the corner spectra of decoupled rows do not move: a fixed number of sweeps
    octm.converge(cell, env, tol=0.0, max_sweeps=sweeps, cutoff=1e-10, min_sweeps=sweeps)
    return obs.energy(cell, env, bond_h)


@pytest.mark.slow
def test_heisenberg_chain_bethe_energy():
    """Horizontal Heisenberg bonds only, vertical legs of dimension one: every
    row is an infinite chain in matrix-product form with bond dimension D = 4.
    Its energy per bond, evaluated by CTM, lies above the Bethe-ansatz value
    1/4 - ln 2 and within 4e-3 of it."""
    D = 4
    T, lam = _chain_state(D)
    bh = lambda x, y, v: np.zeros((4, 4)) if v else HEIS
    for dtau, n in ((0.1, 200), (0.03, 300), (0.01, 500), (0.003, 1000)):
        su.evolve(T, lam, su.gates_from(bh, dtau), D, n, tol=1e-10)
    e, vals = _cell_energy(T, lam, bh, 24, 40)
    per_bond = e / 4
    print("Heisenberg chain D=%d: E/bond %.6f (Bethe %.6f)" % (D, per_bond, E_BETHE))
    assert E_BETHE - 1e-9 <= per_bond <= E_BETHE + 4e-3
    # the vertical weights stay those of dimension-one legs
    assert np.count_nonzero(lam["v0"]) == 1 and np.count_nonzero(lam["v1"]) == 1


def test_classical_ferromagnet():
    """h = -sigma^z sigma^z on every bond: imaginary time ends in a fully
    polarised product state, energy -1 per bond and weights (1, 0)."""
    rng = np.random.default_rng(4)
    D = 2
    T = [rng.standard_normal((2, D, D, D, D)) for _ in range(2)]
    # break the up/down symmetry slightly so one polarisation wins
    T[0][0] += 0.5
    T[1][0] += 0.5
    lam = su.init_weights(D)
    h = -np.kron(SZ, SZ)
    bh = lambda x, y, v: h
    su.evolve(T, lam, su.gates_from(bh, 0.1), D, 300, tol=1e-12)
    e, vals = _cell_energy(T, lam, bh, 8, 10)
    print("ferromagnet: E/bond %.12f, weights %s" % (e / 8, lam["h0"]))
    assert abs(e / 8 + 1.0) < 1e-9
    for b in su.BONDS:
        assert abs(lam[b][0] - 1.0) < 1e-9 and abs(lam[b][1]) < 1e-6


def test_zero_bond_keeps_trivial_leg():
    """Ruby model, D = 2: the B -> A horizontal link (H_l = 0, identity gate)
    starts with weight (1, 0) and A.l, B.r restricted to index 0; after
    Trotter steps it is still exactly rank one."""
    rng = np.random.default_rng(6)
    D = 2
    T = [rng.standard_normal((8, D, D, D, D)) for _ in range(2)]
    T[0][:, :, 1:, :, :] = 0.0   # A.l
    T[1][:, :, :, :, 1:] = 0.0   # B.r
    lam = su.init_weights(D, {"h1": 1})
    su.evolve(T, lam, su.gates_from(models.ruby_bond_h(), 0.05), D, 20)
    assert np.array_equal(lam["h1"], np.array([1.0, 0.0]))
    assert not np.any(T[0][:, :, 1:, :, :]) and not np.any(T[1][:, :, :, :, 1:])
    assert np.count_nonzero(lam["h0"]) == 2
