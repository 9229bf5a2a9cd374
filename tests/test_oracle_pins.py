"""Pins of the CPU float64 oracle against results fixed by mathematics, not by
the oracle itself: the Onsager solution of the 2D Ising model, brute-force
contraction of finite open patches, exact D = 1 product states, the
Eckart-Young property of the projectors, gauge / padding / rotation
invariances, and the ruby block Hamiltonian built a second, independent way.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate, special

import synth
from oracle import ctm, models, obs


# ---------------------------------------------------------------------------
# double layer
# ---------------------------------------------------------------------------
def test_double_layer_brute_force():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((3, 2, 3, 2, 1))
    B = rng.standard_normal((3, 2, 3, 2, 1))
    a = ctm.double_layer(A, B)
    for u, v, l, m, d, e, r, q in itertools.product(range(2), range(2), range(3), range(3),
                                                    range(2), range(2), range(1), range(1)):
        ref = sum(A[s, u, l, d, r] * B[s, v, m, e, q] for s in range(3))
        assert abs(a[u * 2 + v, l * 3 + m, d * 2 + e, r * 1 + q] - ref) < 1e-14


def test_double_layer_psd_rank():
    """a viewed as (ket legs) x (bra legs) is A^T A: PSD with rank <= d."""
    A = synth.cell_tensors(2, 3, 2, 1)[0]
    a = ctm.double_layer(A).reshape(2, 2, 2, 2, 2, 2, 2, 2)
    M = a.transpose(0, 2, 4, 6, 1, 3, 5, 7).reshape(16, 16)
    w = np.linalg.eigvalsh(M)
    assert np.abs(M - M.T).max() < 1e-15
    assert w.min() > -1e-14
    assert np.sum(w > 1e-12) <= 3


def test_rotation_of_double_layer():
    A = synth.cell_tensors(5, 2, 2, 1)[0]
    a = ctm.double_layer(A)
    assert np.array_equal(ctm.rot_a(a, 1), ctm.double_layer(ctm.rot_phys(A, 1)))
    assert np.array_equal(ctm.rot_a(a, 4), a)


# ---------------------------------------------------------------------------
# projectors
# ---------------------------------------------------------------------------
def test_projectors_full_rank_identity():
    rng = np.random.default_rng(7)
    n = 12
    Qs = [rng.standard_normal((n, n)) + 3 * np.eye(n) for _ in range(4)]
    P1, P2 = ctm.projectors(*Qs, chi=n, cutoff=0.0)
    assert np.abs(P1 @ P2 - np.eye(n)).max() < 1e-11


def test_projectors_eckart_young():
    """With truncation, Uh^T P1 P2 Lh^T is the best rank-chi approximation of
    N: its spectral-norm error is sigma_{chi+1} and its Frobenius error the
    root of the discarded sigma^2 (Eckart-Young-Mirsky)."""
    rng = np.random.default_rng(8)
    n, chi = 20, 7
    Qs = [rng.standard_normal((n, n)) for _ in range(4)]
    P1, P2 = ctm.projectors(*Qs, chi=chi, cutoff=0.0)
    Uh, Lh = Qs[0] @ Qs[1], Qs[2] @ Qs[3]
    N = (Lh @ Uh).T
    approx = Uh.T @ P1 @ P2 @ Lh.T
    s = np.linalg.svd(N, compute_uv=False)
    E = N - approx
    assert abs(np.linalg.norm(E, 2) - s[chi]) < 1e-10 * s[0]
    assert abs(np.linalg.norm(E) - np.sqrt(np.sum(s[chi:] ** 2))) < 1e-10 * s[0]
    assert np.linalg.matrix_rank(P1 @ P2, tol=1e-10) == chi


def test_projector_cutoff_zero_rank():
    """Exactly rank-deficient N: only the nonzero singular values are kept."""
    rng = np.random.default_rng(9)
    n, r = 10, 3
    X = rng.standard_normal((n, r)) @ rng.standard_normal((r, n))
    Qs = [X, np.eye(n), np.eye(n), np.eye(n)]
    P1, P2, info = ctm.projectors(*Qs, chi=6, cutoff=1e-12, return_info=True)
    assert info["keep"] == r
    assert np.all(P1[:, r:] == 0) and np.all(P2[r:, :] == 0)


# ---------------------------------------------------------------------------
# finite patches: brute force vs CTM from the trivial start, no truncation
# ---------------------------------------------------------------------------
def _dl(A):
    """Double layer built here from the definition, for the brute force."""
    D = A.shape[1]
    out = np.zeros((D * D,) * 4)
    for s in range(A.shape[0]):
        ket = A[s].reshape(D, 1, D, 1, D, 1, D, 1)
        bra = A[s].reshape(1, D, 1, D, 1, D, 1, D)
        out += (ket * bra).reshape((D * D,) * 4)
    return out


def _patch_Z(a, w, h, Dk):
    """Open w x h patch of double-layer tensors a[U,L,Dn,R]; every boundary leg
    carries delta_uu' (ket and bra bond traced).  Row-by-row contraction."""
    D2 = a.shape[0]
    b = np.eye(Dk).reshape(D2)
    state = b
    for _ in range(w - 1):
        state = np.multiply.outer(state, b)
    state = state.reshape((D2,) * w) if w > 1 else state.reshape(D2)
    for _ in range(h):
        carry = b
        st = state.reshape((D2,) * w)
        # contract columns left to right; st legs: [U_0..U_{w-1}] -> [Dn_0..Dn_{w-1}]
        cur = np.tensordot(st, carry, axes=0)              # [..U.., L]
        for j in range(w):
            # cur legs: Dn_0..Dn_{j-1}, U_j..U_{w-1}, L
            cur = np.tensordot(cur, a, axes=([j, cur.ndim - 1], [0, 1]))  # [.., Dn, R]
            cur = np.moveaxis(cur, -2, j)
        state = np.tensordot(cur, b, axes=([cur.ndim - 1], [0]))
    tot = state
    for _ in range(w):
        tot = np.tensordot(tot, b, axes=([0], [0]))
    return float(tot)


@pytest.mark.parametrize("k", [1, 2])
def test_finite_patch_brute_force(k):
    """k sweeps from the trivial start with nothing truncated: Z11, Z00, Z10,
    Z01 are the open patches (2k+1)^2, (2k)^2, (2k+1) x 2k and 2k x (2k+1).
    (At k = 3 the exact half-system spectrum of the unnormalised 7x7 patch
    spans more than 15 decades, so float64 cannot keep it whole.)"""
    A = synth.cell_tensors(11, 2, 2, 1)[0]
    cell = ctm.Cell(1, 1, [0], [A])
    env = ctm.init_trivial(cell, 64)
    for _ in range(k):
        ctm.sweep(cell, env, cutoff=1e-12, normalize=False)
    Z11, Z00, Z10, Z01 = obs.cell_Z(cell, env)
    a = _dl(A)
    n = 2 * k
    ref = {
        "Z11": _patch_Z(a, n + 1, n + 1, 2), "Z00": _patch_Z(a, n, n, 2),
        "Z10": _patch_Z(a, n + 1, n, 2), "Z01": _patch_Z(a, n, n + 1, 2),
    }
    for name, val in zip(["Z11", "Z00", "Z10", "Z01"], [Z11, Z00, Z10, Z01]):
        assert abs(val - ref[name]) <= 1e-11 * abs(ref[name]), (name, val, ref[name])


def test_uniform_checkerboard_matches_single_site():
    """A 2x2 cell holding the same tensor everywhere describes the same state
    as the 1x1 cell: kappa and all four bond density matrices agree (the two
    runs reach their chi-limited fixed points along different paths)."""
    A = synth.cell_tensors(12, 2, 2, 1)[0]
    c1 = ctm.Cell(1, 1, [0], [A])
    c4 = ctm.Cell(2, 2, [0, 0, 0, 0], [A])
    e1, e4 = _converged(c1, 16, 60), _converged(c4, 16, 60)
    k1, k4 = obs.kappa(c1, e1), obs.kappa(c4, e4)
    assert abs(k1 - k4) < 1e-6 * k1
    for v in (False, True):
        r1 = obs.rdm(c1, e1, 0, 0, v)
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            assert np.abs(obs.rdm(c4, e4, x, y, v) - r1).max() < 1e-6


def test_checkerboard_translation():
    """Swapping A and B is a translation by one site: the bond from (0,0) of
    one cell is the bond from (1,0) of the other (chi-limited)."""
    A, B = synth.cell_tensors(13, 2, 2, 2)
    cab = ctm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    cba = ctm.Cell(2, 2, [0, 1, 1, 0], [B, A])
    eab, eba = _converged(cab, 16, 60), _converged(cba, 16, 60)
    assert abs(obs.kappa(cab, eab) - obs.kappa(cba, eba)) < 1e-6 * obs.kappa(cab, eab)
    for v in (False, True):
        assert np.abs(obs.rdm(cab, eab, 0, 0, v) - obs.rdm(cba, eba, 1, 0, v)).max() < 1e-6


# ---------------------------------------------------------------------------
# Onsager
# ---------------------------------------------------------------------------
def onsager_lnz(K):
    """ln Z per site: ln 2 + (1/(8 pi^2)) int int ln[cosh^2 2K - sinh 2K (cos a + cos b)]."""
    f = lambda b_, a_: np.log(np.cosh(2 * K) ** 2 - np.sinh(2 * K) * (np.cos(a_) + np.cos(b_)))
    val, _ = integrate.dblquad(f, 0, 2 * np.pi, 0, 2 * np.pi, epsabs=1e-13, epsrel=1e-13)
    return np.log(2.0) + val / (8 * np.pi ** 2)


def onsager_lnz_1d(K):
    """Second, independent form: ln(2 cosh 2K) + (1/pi) int_0^{pi/2}
    ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt, k = 2 sinh 2K / cosh^2 2K."""
    kk = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    f = lambda t: np.log(0.5 * (1 + np.sqrt(1 - kk ** 2 * np.sin(t) ** 2)))
    val, _ = integrate.quad(f, 0, np.pi / 2, epsabs=1e-14, epsrel=1e-14)
    return np.log(2 * np.cosh(2 * K)) + val / np.pi


def onsager_zz(K):
    """Nearest-neighbour <s s'> = coth(2K)/2 [1 + (2/pi)(2 tanh^2 2K - 1) K(k)]."""
    kk = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    return (1 / np.tanh(2 * K)) / 2 * (1 + (2 / np.pi) * (2 * np.tanh(2 * K) ** 2 - 1) * special.ellipk(kk ** 2))


def test_onsager_forms_agree():
    for K in (0.3, 0.6):
        assert abs(onsager_lnz(K) - onsager_lnz_1d(K)) < 1e-11
        # <zz> = (1/2) d lnZ/dK (two bonds per site), central difference
        h = 1e-5
        dz = (onsager_lnz_1d(K + h) - onsager_lnz_1d(K - h)) / (2 * h) / 2
        assert abs(dz - onsager_zz(K)) < 1e-8


@pytest.mark.parametrize("K", [0.3, 0.6])
def test_onsager_ctm(K):
    """Ising PEPS (d = D = 2): kappa = Z per site and <zz> match the exact
    solution at chi = 32, far from K_c = 0.4407."""
    A = models.ising_peps(K)
    cell = ctm.Cell(1, 1, [0], [A])
    env = ctm.init_trivial(cell, 32)
    for _ in range(60):
        ctm.sweep(cell, env)
    lnk = np.log(obs.kappa(cell, env))
    rho = obs.rdm(cell, env, 0, 0)
    zz = np.trace(rho @ np.kron(models.SZ, models.SZ))
    assert abs(lnk - onsager_lnz_1d(K)) < 1e-9
    assert abs(zz - onsager_zz(K)) < 1e-9
    # both bond directions agree (the model is isotropic)
    rv = obs.rdm(cell, env, 0, 0, vertical=True)
    assert abs(np.trace(rv @ np.kron(models.SZ, models.SZ)) - zz) < 1e-9


# ---------------------------------------------------------------------------
# D = 1 product states
# ---------------------------------------------------------------------------
def test_product_state_exact():
    rng = np.random.default_rng(3)
    phi = rng.standard_normal(3)
    A = models.product_peps(phi)
    cell = ctm.Cell(1, 1, [0], [A])
    env = ctm.init_trivial(cell, 4)
    for _ in range(3):
        ctm.sweep(cell, env)
    nrm = phi @ phi
    assert abs(obs.kappa(cell, env) - nrm) < 1e-13 * nrm
    rho = obs.rdm(cell, env, 0, 0)
    pp = np.kron(phi, phi)
    assert np.abs(rho - np.outer(pp, pp) / nrm ** 2).max() < 1e-13


def test_product_state_fidelity():
    rng = np.random.default_rng(4)
    p1, p2 = rng.standard_normal(4), rng.standard_normal(4)
    A1, A2 = models.product_peps(p1), models.product_peps(p2)
    ks = []
    for kets, bras in [([A1], [A1]), ([A2], [A2]), ([A1], [A2])]:
        cell = ctm.Cell(1, 1, [0], kets, bras)
        env = ctm.init_trivial(cell, 4)
        for _ in range(3):
            ctm.sweep(cell, env)
        ks.append(obs.kappa(cell, env))
    d = obs.fidelity(ks[2], ks[0], ks[1])
    assert abs(d - abs(p1 @ p2) / np.sqrt((p1 @ p1) * (p2 @ p2))) < 1e-13


# ---------------------------------------------------------------------------
# ruby Hamiltonian
# ---------------------------------------------------------------------------
def _pauli_apply(alpha, bit):
    """(new bit, amplitude) of sigma^alpha acting on basis state bit (0: up)."""
    if alpha == "z":
        return bit, (1.0 if bit == 0 else -1.0)
    if alpha == "x":
        return 1 - bit, 1.0
    return 1 - bit, (1j if bit == 0 else -1j)


def _term_bitloop(ops, nspins=6):
    """Matrix of a product of Paulis on a 6-spin register (spins 1..3 block one,
    4..6 block two; spin 1 the most significant bit), by explicit action on
    basis states."""
    dim = 2 ** nspins
    M = np.zeros((dim, dim), dtype=complex)
    for col in range(dim):
        bits = [(col >> (nspins - 1 - j)) & 1 for j in range(nspins)]
        amp = 1.0
        for spin, alpha in ops:
            nb, a = _pauli_apply(alpha, bits[spin - 1])
            bits[spin - 1] = nb
            amp *= a
        row = sum(b << (nspins - 1 - j) for j, b in enumerate(bits))
        M[row, col] += amp
    return M


def test_ruby_terms_two_ways():
    J = (0.7, 1.3, 0.4)
    t = models.ruby_terms(J)
    Jx, Jy, Jz = J
    # H_r: -Jx s^x_A1 s^x_B1 - Jy s^y_A3 s^y_B3 (A spins 1..3, B spins 4..6)
    Hr = -Jx * _term_bitloop([(1, "x"), (4, "x")]) - Jy * _term_bitloop([(3, "y"), (6, "y")])
    assert np.abs(t["Hr"] - Hr).max() < 1e-14
    zzA = sum(_term_bitloop([(i, "z"), (j, "z")]) for i, j in [(1, 2), (1, 3), (2, 3)])
    zzB = sum(_term_bitloop([(i, "z"), (j, "z")]) for i, j in [(4, 5), (4, 6), (5, 6)])
    # H_u: A above B: (h_A + h_B)/2 - Jx s^x_A3 s^x_B2 - Jy s^y_A2 s^y_B1
    Hu = 0.5 * (-Jz) * (zzA + zzB) - Jx * _term_bitloop([(3, "x"), (5, "x")]) \
        - Jy * _term_bitloop([(2, "y"), (4, "y")])
    assert np.abs(t["Hu"] - Hu).max() < 1e-14
    # H_d: B above A: -Jx s^x_B3 s^x_A2 - Jy s^y_B2 s^y_A1 with B first
    Hd = 0.5 * (-Jz) * (zzA + zzB) - Jx * _term_bitloop([(3, "x"), (5, "x")]) \
        - Jy * _term_bitloop([(2, "y"), (4, "y")])
    assert np.abs(t["Hd"] - Hd).max() < 1e-14
    assert np.abs(t["Hl"]).max() == 0.0


def test_ruby_onsite_spectrum():
    h = models.ruby_terms((1, 1, 1))["hA"]
    w = np.sort(np.linalg.eigvalsh(h))
    assert np.allclose(w, [-3, -3, 1, 1, 1, 1, 1, 1], atol=1e-14)


@pytest.mark.parametrize("state,expected", [("up", -1.0), ("plus", -0.5)])
def test_ruby_product_state_energy(state, expected):
    """All spins up: only the z bonds contribute, -J_z per spin; all spins in
    |+>: only the x bonds, -J_x / 2 per spin (3 x-bonds per 6 spins)."""
    s1 = np.array([1.0, 0.0]) if state == "up" else np.array([1.0, 1.0]) / np.sqrt(2)
    phi = np.kron(np.kron(s1, s1), s1)
    A = models.product_peps(phi)
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [A, A])
    env = ctm.init_trivial(cell, 2)
    for _ in range(2):
        ctm.sweep(cell, env)
    E, _ = obs.energy(cell, env, models.ruby_bond_h((1, 1, 1)))
    assert abs(E / 12 - expected) < 1e-13


# ---------------------------------------------------------------------------
# invariances
# ---------------------------------------------------------------------------
def _converged(cell, chi, sweeps=25):
    env = ctm.init_trivial(cell, chi)
    for _ in range(sweeps):
        ctm.sweep(cell, env)
    return env


def _gauge(A, Gh, Gv):
    """Bond gauge of a 1x1 cell: right leg x Gh, left leg x Gh^{-T}, down leg
    x Gv, up leg x Gv^{-T}; the bond contractions are unchanged."""
    Ghi, Gvi = np.linalg.inv(Gh).T, np.linalg.inv(Gv).T
    return np.einsum("suldr,uU,lL,dE,rR->sULER", A, Gvi, Ghi, Gv, Gh)


def test_orthogonal_gauge_invariance():
    A = synth.cell_tensors(21, 2, 3, 1)[0]
    rng = np.random.default_rng(5)
    Oh, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Ov, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    c1, c2 = ctm.Cell(1, 1, [0], [A]), ctm.Cell(1, 1, [0], [_gauge(A, Oh, Ov)])
    e1, e2 = _converged(c1, 12), _converged(c2, 12)
    assert abs(obs.kappa(c1, e1) - obs.kappa(c2, e2)) < 1e-12 * obs.kappa(c1, e1)
    s1, s2 = ctm.corner_spectra(e1)[(0, 0)], ctm.corner_spectra(e2)[(0, 0)]
    assert max(np.abs(a - b).max() for a, b in zip(s1, s2)) < 1e-10


def test_general_gauge_exact_without_truncation():
    """A general gauge changes the truncation, so invariance is exact only
    when nothing is truncated: one sweep from the trivial start at chi = 64."""
    A = synth.cell_tensors(22, 2, 2, 1)[0]
    rng = np.random.default_rng(6)
    Gh = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    Gv = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    c1, c2 = ctm.Cell(1, 1, [0], [A]), ctm.Cell(1, 1, [0], [_gauge(A, Gh, Gv)])
    # boundary deltas are not gauge covariant, so compare networks whose
    # boundary is far: the ratio kappa converges to the same value
    e1, e2 = _converged(c1, 32, 30), _converged(c2, 32, 30)
    k1, k2 = obs.kappa(c1, e1), obs.kappa(c2, e2)
    assert abs(k1 - k2) < 1e-8 * k1


def test_padding_invariance():
    A = synth.cell_tensors(23, 2, 2, 1)[0]
    Ap = np.zeros((2, 3, 3, 3, 3))
    Ap[:, :2, :2, :2, :2] = A
    c1, c2 = ctm.Cell(1, 1, [0], [A]), ctm.Cell(1, 1, [0], [Ap])
    e1, e2 = _converged(c1, 12), _converged(c2, 12)
    assert abs(obs.kappa(c1, e1) - obs.kappa(c2, e2)) < 1e-12 * obs.kappa(c1, e1)
    r1, r2 = obs.rdm(c1, e1, 0, 0), obs.rdm(c2, e2, 0, 0)
    assert np.abs(r1 - r2).max() < 1e-12


def test_rotation_exact_without_truncation():
    """One sweep from the trivial start at chi = 64 contracts finite patches
    exactly, and a patch of turned tensors is the turned patch: kappa is
    unchanged and the vertical bond of A is the horizontal bond of the turned
    tensor (one counter-clockwise turn maps (upper, lower) to (left, right))."""
    A = synth.cell_tensors(24, 2, 2, 1)[0]
    Ar = ctm.rot_phys(A, 1)
    c1, c2 = ctm.Cell(1, 1, [0], [A]), ctm.Cell(1, 1, [0], [Ar])
    e1, e2 = ctm.init_trivial(c1, 64), ctm.init_trivial(c2, 64)
    ctm.sweep(c1, e1, normalize=False)
    ctm.sweep(c2, e2, normalize=False)
    assert abs(obs.kappa(c1, e1) - obs.kappa(c2, e2)) < 1e-11 * obs.kappa(c1, e1)
    rv1 = obs.rdm(c1, e1, 0, 0, vertical=True)
    rh2 = obs.rdm(c2, e2, 0, 0, vertical=False)
    assert np.abs(rv1 - rh2).max() < 1e-11


def test_rotation_converged():
    """At a chi-limited fixed point the same holds to truncation error."""
    A = synth.cell_tensors(24, 2, 2, 1)[0]
    Ar = ctm.rot_phys(A, 1)
    c1, c2 = ctm.Cell(1, 1, [0], [A]), ctm.Cell(1, 1, [0], [Ar])
    e1, e2 = _converged(c1, 16, 60), _converged(c2, 16, 60)
    assert abs(obs.kappa(c1, e1) - obs.kappa(c2, e2)) < 1e-8 * obs.kappa(c1, e1)
    rv1 = obs.rdm(c1, e1, 0, 0, vertical=True)
    rh2 = obs.rdm(c2, e2, 0, 0, vertical=False)
    assert np.abs(rv1 - rh2).max() < 1e-6


def test_rdm_properties():
    A, B = synth.cell_tensors(25, 2, 2, 2)
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = _converged(cell, 12, 15)
    for x, y, v in [(0, 0, False), (1, 0, False), (0, 0, True), (0, 1, True)]:
        rho = obs.rdm(cell, env, x, y, v)
        assert abs(np.trace(rho) - 1) < 1e-14
        assert obs.herm_defect(rho) < 1e-8
        assert np.linalg.eigvalsh(0.5 * (rho + rho.T)).min() > -1e-8


def test_fidelity_identities():
    """Two nearby states (as for ground states at nearby couplings): the mixed
    network then has a well-separated dominant fixed point."""
    A, R = synth.cell_tensors(26, 2, 2, 2)
    B = A + 0.3 * R
    B /= np.linalg.norm(B)
    rng = np.random.default_rng(2)
    O, _ = np.linalg.qr(rng.standard_normal((2, 2)))

    def kap(kets, bras):
        cell = ctm.Cell(1, 1, [0], kets, bras)
        return obs.kappa(cell, _converged(cell, 12, 40))

    kaa, kbb, kab, kba = kap([A], [A]), kap([B], [B]), kap([A], [B]), kap([B], [A])
    assert abs(obs.fidelity(kaa, kaa, kaa) - 1) < 1e-12
    assert abs(obs.fidelity(kap([A], [3.0 * A]), kaa, kap([3.0 * A], [3.0 * A])) - 1) < 1e-10
    Ag = _gauge(A, O, O)
    assert abs(obs.fidelity(kap([A], [Ag]), kaa, kap([Ag], [Ag])) - 1) < 1e-9
    assert abs(kab - kba) < 1e-10 * abs(kab)
    assert obs.fidelity(kab, kaa, kbb) <= 1 + 1e-12


# ---------------------------------------------------------------------------
# the 2x2 checkerboard with A != B (multi-site cell, Sec. II C; Fig. 3(b))
# ---------------------------------------------------------------------------
def _orth(rng, n):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q


def _checkerboard_gauge(A, O1, O2, O3, O4):
    """Two tensors A' (sites with x + y even) and B' (odd) that describe the
    same network as A on every site: each of the four bond types of the
    checkerboard carries its own orthogonal gauge (O1 on A-right / B-left,
    O2 on B-right / A-left, O3 on A-down / B-up, O4 on B-down / A-up), so
    every bond contraction sum_r A[..r] B[r..] is unchanged (O O^T = 1)."""
    Ap = np.einsum("suldr,uU,lL,dE,rR->sULER", A, O4, O2, O3, O1)
    Bp = np.einsum("suldr,uU,lL,dE,rR->sULER", A, O3, O1, O4, O2)
    return Ap, Bp


@pytest.mark.parametrize("K", [0.3, 0.6])
def test_onsager_checkerboard_distinct_tensors(K):
    """Ising PEPS on the 2x2 checkerboard with A != B related by random
    orthogonal bond gauges: the norm network is still the Ising model, so
    kappa and <zz> on all four bonds of the cell must equal the exact
    solution.  The two tensors differ, so the projectors of the two rows of
    a column step differ and a wrong pairing of projector rows with edges
    (or of sites with frames) changes the result: a planted pairing error in
    the corner absorption gives kappa < 0 and <zz> off by 0.18 here."""
    rng = np.random.default_rng(17 if K == 0.3 else 18)
    Ap, Bp = _checkerboard_gauge(models.ising_peps(K), *[_orth(rng, 2) for _ in range(4)])
    assert np.linalg.norm(Ap - Bp) > 1.0
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [Ap, Bp])
    env = ctm.init_trivial(cell, 32)
    for _ in range(40):
        ctm.sweep(cell, env)
    assert abs(np.log(obs.kappa(cell, env)) - onsager_lnz_1d(K)) < 1e-9
    zz = np.kron(models.SZ, models.SZ)
    for vertical in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            rho = obs.rdm(cell, env, x, y, vertical)
            assert abs(np.trace(rho @ zz) - onsager_zz(K)) < 1e-9, (vertical, x, y)


def test_product_state_checkerboard_positions():
    """D = 1 product states phi_A, phi_B on the checkerboard: every bond
    density matrix is the product of the two site states in the bond's order
    (left/upper site first), which fixes where A and B sit."""
    rng = np.random.default_rng(19)
    pa, pb = rng.standard_normal(3), rng.standard_normal(3)
    cell = ctm.Cell(2, 2, [0, 1, 1, 0], [models.product_peps(pa), models.product_peps(pb)])
    env = ctm.init_trivial(cell, 3)
    for _ in range(2):
        ctm.sweep(cell, env)
    na, nb = pa @ pa, pb @ pb
    assert abs(obs.kappa(cell, env) - np.sqrt(na * nb)) < 1e-13 * np.sqrt(na * nb)
    for vertical in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            first, second = (pa, pb) if (x + y) % 2 == 0 else (pb, pa)
            v = np.kron(first, second)
            rho = obs.rdm(cell, env, x, y, vertical)
            assert np.abs(rho - np.outer(v, v) / (v @ v)).max() < 1e-13


# ---------------------------------------------------------------------------
# diagonal start (learned warm start)
# ---------------------------------------------------------------------------
def _traced_boundary(A):
    """a~[dn, r] = sum_(u, l) a[(u,u), (l,l), dn, r], from A directly: the
    double layer with its up and left ket/bra pairs joined."""
    d, D = A.shape[0], A.shape[1]
    out = np.zeros((D * D, D * D))
    for s in range(d):
        for u in range(D):
            for l in range(D):
                for dn in range(D):
                    for dn2 in range(D):
                        for r in range(D):
                            for r2 in range(D):
                                out[dn * D + dn2, r * D + r2] += A[s, u, l, dn, r] * A[s, u, l, dn2, r2]
    return out


def test_init_diag_enlarged_corner_is_kronecker():
    """With C = diag(s) / |s| and T[a, (u,u'), b] = delta_ab delta_uu' / sqrt(chi D)
    the enlarged corner is exactly (C (x) a~) / (chi D), a~ the double layer
    with its two boundary pairs traced: the edge carries no information
    about the lattice beyond the corner's own spectrum."""
    A = synth.cell_tensors(27, 2, 2, 1)[0]
    cell = ctm.Cell(1, 1, [0], [A])
    chi, D = 6, 2
    rng = np.random.default_rng(27)
    spec = {(0, 0): [np.sort(rng.uniform(0.1, 1.0, chi))[::-1] for _ in range(4)]}
    env = ctm.init_diag(cell, chi, spec)
    for i in range(4):
        s = spec[(0, 0)][i]
        assert np.abs(env.C[i][(0, 0)] - np.diag(s) / np.linalg.norm(s)).max() < 1e-15
        assert abs(np.linalg.norm(env.T[i][(0, 0)]) - 1.0) < 1e-15
    at = _traced_boundary(A)
    Q = ctm.enlarged_corner(env.C[0][(0, 0)], env.T[0][(0, 0)], env.T[3][(0, 0)], cell.a(0, 0))
    ref = np.kron(env.C[0][(0, 0)], at) / (chi * D)
    assert np.abs(Q - ref).max() < 1e-15 * np.abs(ref).max() * 10


# ---------------------------------------------------------------------------
# ruby-faithful block tensors: one trivial (D = 1) leg per block site
# ---------------------------------------------------------------------------
def ruby_trivial_leg_tensors(seed, d, D):
    """Checkerboard tensors with the trivial bond of each block site (caption
    of Fig. 2: three bonds of dimension D and one of dimension 1): A (x + y
    even) has a trivial down leg, B a trivial up leg, so every other vertical
    bond of the cell is absent (the brick-wall structure of the coarse-grained
    lattice)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, D, D, 1, D))
    B = rng.standard_normal((d, 1, D, D, D))
    return A / np.linalg.norm(A), B / np.linalg.norm(B)


def pad_legs(T, D):
    """Zero-pad every bond leg of T[s, u, l, d, r] to D."""
    out = np.zeros((T.shape[0], D, D, D, D), dtype=T.dtype)
    out[:, :T.shape[1], :T.shape[2], :T.shape[3], :T.shape[4]] = T
    return out


def test_trivial_legs_equal_zero_padding():
    """A D = 1 leg and the same leg zero-padded to D describe the same network:
    with nothing truncated differently (padding adds only zero singular
    values), kappa, every bond density matrix and the corner spectra agree
    between the 2x2 cell with true trivial legs and the padded one."""
    A, B = ruby_trivial_leg_tensors(41, 2, 2)
    c1 = ctm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    c2 = ctm.Cell(2, 2, [0, 1, 1, 0], [pad_legs(A, 2), pad_legs(B, 2)])
    e1, e2 = _converged(c1, 12, 20), _converged(c2, 12, 20)
    assert abs(obs.kappa(c1, e1) - obs.kappa(c2, e2)) < 1e-12 * abs(obs.kappa(c1, e1))
    for v in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            assert np.abs(obs.rdm(c1, e1, x, y, v) - obs.rdm(c2, e2, x, y, v)).max() < 1e-11
    s1, s2 = ctm.corner_spectra(e1), ctm.corner_spectra(e2)
    for key in s1:
        assert max(np.abs(a - b).max() for a, b in zip(s1[key], s2[key])) < 1e-11


def _complex_unitary(rng, n):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q


def complex_gauged(tensors, seed):
    """The same state with a random complex unitary gauge on every bond:
    right leg r -> r G, left leg l -> G^-1 l (one G for the horizontal bonds,
    one H for the vertical ones), so that every bond contracts G G^-1."""
    rng = np.random.default_rng(seed)
    D = tensors[0].shape[1]
    G, H = _complex_unitary(rng, D), _complex_unitary(rng, D)
    Gi, Hi = np.linalg.inv(G), np.linalg.inv(H)
    return [np.einsum("suldr,Ll,rR,Uu,dD->sULDR", A, Gi, G, Hi, H) for A in tensors]


@pytest.mark.parametrize("cell_kind", ["1x1", "2x2"])
def test_complex_gauge_pin(cell_kind):
    """Complex tensors (Sec. II A allows complex coefficients): a real PEPS
    under a complex unitary gauge on every bond is the same state, and a
    unitary gauge acts on each doubled leg as the unitary G (x) conj(G), which
    the truncation does not see.  So the complex path (the conjugate bra in
    the double layer and in the open tensors of the density matrices) must
    give the real state's corner spectra after every sweep, its norm per site
    and its density matrices, to rounding.  Dropping a conjugate anywhere
    breaks this (the gauge would act as G (x) G).  Bound 1e-10: the kept
    spectra of the 2x2 cell differ by 1.3e-11 through rounding alone."""
    if cell_kind == "1x1":
        tens, Lx, Ly, pat = synth.cell_tensors(3, 2, 2, 1), 1, 1, [0]
    else:
        tens, Lx, Ly, pat = synth.cell_tensors(4, 2, 2, 2), 2, 2, [0, 1, 1, 0]
    gt = complex_gauged(tens, 11)
    assert np.abs(np.imag(gt[0])).max() > 0.1
    cr, cc = ctm.Cell(Lx, Ly, pat, tens), ctm.Cell(Lx, Ly, pat, gt)
    er, ec = ctm.init_trivial(cr, 12), ctm.init_trivial(cc, 12)
    for _ in range(5):
        ctm.sweep(cr, er, cutoff=1e-12)
        ctm.sweep(cc, ec, cutoff=1e-12)
        sr, sc = ctm.corner_spectra(er), ctm.corner_spectra(ec)
        for key in sr:
            for i in range(4):
                assert np.abs(sr[key][i] - sc[key][i]).max() < 1e-10
    kr, kc = obs.kappa(cr, er), obs.kappa(cc, ec)
    assert abs(kc - kr) < 1e-10 * abs(kr)
    for v in (False, True):
        rr, rc = obs.rdm(cr, er, 0, 0, v), obs.rdm(cc, ec, 0, 0, v)
        assert np.abs(rc - rr).max() < 1e-10
