"""Simple update on the GPU (ctm_su_*) against the oracle's (oracle/su.py) on
the same seeded inputs.

Compared quantities do not depend on the gauge of the bond indices (the SVD
fixes singular vectors only up to sign, and degenerate ones up to a
rotation): the bond weights, and the one-site and two-site densities of the
weighted tensors.  Tolerances: weights and densities 1e-10 after one Trotter
step, 1e-8 after ten (the GPU factors each tensor through the eigenvalues
of its Gram matrix where the oracle takes a QR decomposition, and above
d^2 D = 80 takes the leading singular triplets of theta by subspace
iteration where the oracle takes a full SVD: both agree to rounding
relative to the smallest kept singular value).  (8, 3) and (8, 4) run the
subspace-iteration path.
"""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import models, obs, su

pytestmark = pytest.mark.gpu

SX, SZ = models.SX, models.SZ
SYSY = np.real(np.kron(models.SY, models.SY))
HEIS = 0.25 * (np.kron(SX, SX) + SYSY + np.kron(SZ, SZ))
E_BETHE = 0.25 - np.log(2.0)


def _weighted(T, lam, t):
    X = T[t]
    for leg in range(1, 5):
        shape = [1] * 5
        shape[leg] = -1
        X = X * lam[su.LEG_BOND[t][leg]].reshape(shape)
    return X


def _densities(T, lam):
    """One-site densities of A and B and the two-site density of every bond
    type (the weighted tensors contracted over all virtual indices), each
    divided by its trace."""
    out = []
    W = [_weighted(T, lam, t) for t in (0, 1)]
    for t in (0, 1):
        r = np.einsum("sabcd,tabcd->st", W[t], W[t])
        out.append(r / np.trace(r))
    for b in su.BONDS:
        (t1, p1), (t2, p2) = su.ENDS[b]
        # the bond index carries lambda once: divide one copy out of each side
        X = np.moveaxis(W[t1], p1, -1)
        Y = np.moveaxis(W[t2], p2, -1)
        lb = lam[b]
        inv = np.where(lb > 0, 1.0 / np.where(lb > 0, lb, 1.0), 0.0)
        Psi = np.einsum("sabcp,p,tefgp->sabctefg", X, inv, Y)
        r = np.einsum("sabctefg,uabcvefg->stuv", Psi, Psi)
        d = r.shape[0]
        r = r.reshape(d * d, d * d)
        out.append(r / np.trace(r))
    return out


def _random_state(seed, d, D):
    rng = np.random.default_rng(seed)
    T = [synth.peps_tensor(rng, d, D) for _ in range(2)]
    lam = {b: np.sort(rng.uniform(0.3, 1.0, D))[::-1] / 1.0 for b in su.BONDS}
    for b in su.BONDS:
        lam[b] = lam[b] / np.linalg.norm(lam[b])
    return T, lam


def _random_h(seed, d):
    rng = np.random.default_rng(seed)
    hs = []
    for _ in range(4):
        h = rng.standard_normal((d * d, d * d))
        hs.append(0.5 * (h + h.T))
    return hs


def _gpu(states, hs, dtau):
    from paper_1711_04798_amd import SimpleUpdate
    D = states[0][0][0].shape[1]
    g = SimpleUpdate([[T[0], T[1]] for T, _ in states],
                     np.array([[lam[b] for b in su.BONDS] for _, lam in states]))
    g.set_gates(np.array([[h[b] for b in range(4)] for h in hs]), dtau)
    return g


def _compare(gT, gL, T, lam, tol, what):
    glam = {b: gL[i] for i, b in enumerate(su.BONDS)}
    werr = max(np.abs(glam[b] - lam[b]).max() for b in su.BONDS)
    derr = max(np.abs(a - c).max() for a, c in zip(_densities([gT[0], gT[1]], glam), _densities(T, lam)))
    print("%s: weights %.2e densities %.2e" % (what, werr, derr))
    assert werr < tol and derr < tol


@pytest.mark.parametrize("d,D", [(2, 3), (2, 6), (8, 2), (3, 4), (8, 3), (8, 4)])
def test_su_matches_oracle(gpu, d, D):
    """Random states and random symmetric bond Hamiltonians: one Trotter step
    (1e-10), then nine more (1e-8)."""
    T, lam = _random_state(10 + d + D, d, D)
    hl = _random_h(20 + d + D, d)
    print("case su parity", d, D, flush=True)
    g = _gpu([(T, lam)], [hl], 0.05)
    gates = {b: None for b in su.BONDS}
    bh_list = dict(zip(su.BONDS, hl))
    for b in su.BONDS:
        w, V = np.linalg.eigh(0.5 * (bh_list[b] + bh_list[b].T))
        gates[b] = (V * np.exp(-0.05 * w)) @ V.T
    To = [t.copy() for t in T]
    lo = {b: v.copy() for b, v in lam.items()}
    su.step(To, lo, gates, D)
    steps, ch = g.evolve(1, 0.0, 1)
    assert steps == 1
    gT, gL = g.state()
    _compare(gT[0], gL[0], To, lo, 1e-10, "d=%d D=%d one step" % (d, D))
    for _ in range(9):
        su.step(To, lo, gates, D)
    g.evolve(9, 0.0, 3)
    gT, gL = g.state()
    _compare(gT[0], gL[0], To, lo, 1e-8, "d=%d D=%d ten steps" % (d, D))
    g.close()


def test_su_batched_ruby(gpu):
    """Five ruby-model instances with different couplings (d = 8, D = 2), each
    against its own oracle run after five Trotter steps."""
    Js = [(1.0, 1.0, 1.0), (0.8, 0.8, 0.4), (1.2, 0.5, 0.3), (0.3, 0.3, 1.4), (1.0, 0.2, 0.8)]
    states, hs, ref = [], [], []
    for i, J in enumerate(Js):
        T, lam = _random_state(40 + i, 8, 2)
        bh = models.ruby_bond_h(J)
        h = [bh(0, 0, False), bh(1, 0, False), bh(0, 0, True), bh(1, 0, True)]
        states.append((T, lam))
        hs.append(h)
        To = [t.copy() for t in T]
        lo = {b: v.copy() for b, v in lam.items()}
        su.evolve(To, lo, su.gates_from(bh, 0.05), 2, 5)
        ref.append((To, lo))
    print("case su batched ruby", flush=True)
    g = _gpu(states, hs, 0.05)
    g.evolve(5, 0.0, 5)
    gT, gL = g.state()
    for i in range(len(Js)):
        _compare(gT[i], gL[i], ref[i][0], ref[i][1], 1e-8, "J=%s" % (Js[i],))
    g.close()


def test_su_zero_bond_trivial_leg(gpu):
    """The ruby model's B -> A link (zero Hamiltonian, identity gate) started
    at rank one stays exactly rank one on the GPU."""
    rng = np.random.default_rng(6)
    D = 2
    T = [rng.standard_normal((8, D, D, D, D)) for _ in range(2)]
    T[0][:, :, 1:, :, :] = 0.0
    T[1][:, :, :, :, 1:] = 0.0
    lam = su.init_weights(D, {"h1": 1})
    bh = models.ruby_bond_h()
    h = [bh(0, 0, False), bh(1, 0, False), bh(0, 0, True), bh(1, 0, True)]
    print("case su trivial leg", flush=True)
    g = _gpu([(T, lam)], [h], 0.05)
    g.evolve(20, 0.0, 10)
    gT, gL = g.state()
    g.close()
    assert np.array_equal(gL[0][1], np.array([1.0, 0.0]))
    assert not np.any(gT[0][0][:, :, 1:, :, :]) and not np.any(gT[0][1][:, :, :, :, 1:])


def test_su_heisenberg_chain_gpu(gpu):
    """The Heisenberg-chain pin through the GPU path: simple update on the GPU
    with the oracle pin's schedule, then the GPU CTM of its iPEPS: the energy
    per bond lies above the Bethe-ansatz value and within 4e-3 of it, and the
    weights match the oracle's run."""
    from paper_1711_04798_amd import CTM
    D = 4
    rng = np.random.default_rng(3)
    T = [rng.standard_normal((2, D, D, D, D)) for _ in range(2)]
    for X in T:
        X[:, 1:, :, :, :] = 0.0
        X[:, :, :, 1:, :] = 0.0
    lam = su.init_weights(D, {"v0": 1, "v1": 1})
    z = np.zeros((4, 4))
    h = [HEIS, HEIS, z, z]
    print("case su heisenberg chain", flush=True)
    g = _gpu([(T, lam)], [h], 0.1)
    To = [t.copy() for t in T]
    lo = {b: v.copy() for b, v in lam.items()}
    bh = lambda x, y, v: z if v else HEIS
    for dtau, n in ((0.1, 200), (0.03, 300), (0.01, 500), (0.003, 1000)):
        g.set_gates(np.array([h]), dtau)
        g.evolve(n, 1e-10, 10)
        su.evolve(To, lo, su.gates_from(bh, dtau), D, n, tol=1e-10)
    gT, gL = g.state()
    A, B = g.peps()[0]
    g.close()
    werr = max(np.abs(gL[0][i] - lo[b]).max() for i, b in enumerate(su.BONDS))
    c = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24, cutoff=1e-10)
    c.converge(tol=0.0, max_sweeps=40)
    e = sum(c.expect(x, y, False, HEIS) for y in range(2) for x in range(2)) / 4
    c.close()
    print("GPU simple update: weights vs oracle %.2e; E/bond %.6f (Bethe %.6f)" % (werr, e, E_BETHE))
    assert werr < 1e-6
    assert E_BETHE - 1e-9 <= e <= E_BETHE + 4e-3
