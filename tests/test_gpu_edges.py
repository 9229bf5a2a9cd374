"""Edge cases of the GPU path against the oracle on the same seeded inputs:
the smallest environment (chi = 1), bond dimension one (product states,
whose norm and density matrices have closed forms), a physical dimension of
one, rectangular and larger cells (2x1, 1x2, 3x2, 3x3, 4x4 with several
tensors, their norm by row transfer), and the largest chi the configuration
admits (chi + oversampling = 176).

Tolerances as in the parity tests: lock-step spectra 1e-8, kappa and
density matrices 1e-10 relative.
"""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs
from oracle import models

pytestmark = pytest.mark.gpu

ORDER = ["L", "R", "U", "D"]


def _spec_oracle(env, Lx, Ly):
    sp = octm.corner_spectra(env)
    return np.array([[sp[(x, y)][c] for c in range(4)] for y in range(Ly) for x in range(Lx)])


def _lockstep(tens, Lx, Ly, pattern, chi, sweeps, **kw):
    from paper_1711_04798_amd import CTM
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pattern, chi=chi, **kw)
    cell = octm.Cell(Lx, Ly, pattern, tens)
    env = octm.init_trivial(cell, chi)
    worst = 0.0
    for _ in range(sweeps):
        for dn in ORDER:
            k = octm.DIRS[dn]
            lx, _ = octm.frame_dims(k, Lx, Ly)
            for xp in range(lx):
                octm.column_step(cell, env, k, xp)
                g.move(dn, 1)
                err = np.abs(_spec_oracle(env, Lx, Ly) - g.spectra()).max()
                worst = max(worst, err)
                assert err < 1e-8, (dn, xp, err)
    return g, cell, env, worst


def test_chi_one(gpu):
    """chi = 1: every corner and edge is a single index (a rank-one boundary)."""
    A, = synth.cell_tensors(2, 2, 3, 1)
    print("case chi=1", flush=True)
    g, cell, env, worst = _lockstep([A], 1, 1, [0], 1, 4)
    ko, kg = oobs.kappa(cell, env), g.norm()
    print("chi=1: kappa oracle %.15f gpu %.15f" % (ko, kg))
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    g.close()


def test_product_states_closed_form(gpu):
    """D = 1 product states on the 2x2 checkerboard with different site states:
    kappa per site = geometric mean of |phi|^2 and every bond density matrix
    the product of the two site projectors (closed forms)."""
    from paper_1711_04798_amd import CTM
    rng = np.random.default_rng(8)
    phis = [rng.standard_normal(3) for _ in range(2)]
    tens = [models.product_peps(p) for p in phis]
    print("case product states", flush=True)
    g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=4)
    g.converge(tol=1e-12, max_sweeps=20)
    want_k = np.sqrt(np.dot(phis[0], phis[0]) * np.dot(phis[1], phis[1]))
    kg = g.norm()
    print("product: kappa %.15f closed form %.15f" % (kg, want_k))
    assert abs(kg - want_k) <= 1e-12 * want_k
    proj = [np.outer(p, p) / np.dot(p, p) for p in phis]
    for (x, y, v) in [(0, 0, False), (1, 0, False), (0, 0, True), (1, 1, True)]:
        first = proj[(x + y) % 2]
        second = proj[(x + y + 1) % 2]
        rg, _ = g.rdm(x, y, v)
        assert np.abs(rg - np.kron(first, second)).max() < 1e-12
    g.close()


def test_physical_dimension_one(gpu):
    """d = 1: the double layer is a single outer product per site."""
    A, B = synth.cell_tensors(9, 1, 2, 2)
    print("case d=1", flush=True)
    g, cell, env, worst = _lockstep([A, B], 2, 2, [0, 1, 1, 0], 6, 4)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    g.close()


@pytest.mark.parametrize("Lx,Ly,pattern,nt", [(2, 1, [0, 1], 2), (1, 2, [0, 1], 2), (3, 2, [0, 1, 2, 1, 2, 0], 3),
                                              (3, 3, [0, 1, 2, 1, 2, 0, 2, 0, 1], 3),
                                              (4, 4, [0, 1, 0, 1, 1, 0, 1, 0, 0, 1, 0, 1, 1, 0, 1, 0], 2)])
def test_cells(gpu, Lx, Ly, pattern, nt):
    """Rectangular and larger cells, several tensors: spectra lock-step over
    two sweeps (every column of every direction), then the norm per site
    (row transfer for cells other than 1x1 and 2x2) and one horizontal and
    one vertical density matrix."""
    tens = synth.cell_tensors(20 + Lx * 10 + Ly, 2, 2, nt)
    print("case cell", Lx, Ly, flush=True)
    g, cell, env, worst = _lockstep(tens, Lx, Ly, pattern, 6, 2)
    ko, kg = oobs.kappa(cell, env), g.norm()
    print("cell %dx%d: worst spectra %.2e, kappa oracle %.15f gpu %.15f" % (Lx, Ly, worst, ko, kg))
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    for v in (False, True):
        ro = oobs.rdm(cell, env, Lx - 1, Ly - 1, v)
        rg, _ = g.rdm(Lx - 1, Ly - 1, v)
        assert np.linalg.norm(rg - ro) <= 1e-10 * np.linalg.norm(ro)
    g.close()


def test_largest_chi(gpu):
    """chi = 160 with 16 oversampling columns (the 176-column subspace limit),
    1x1 cell, d = 2, D = 2 (cut dimension 640): two sweeps lock-step."""
    A, = synth.cell_tensors(4, 2, 2, 1)
    print("case chi=160", flush=True)
    g, cell, env, worst = _lockstep([A], 1, 1, [0], 160, 2)
    ko, kg = oobs.kappa(cell, env), g.norm()
    print("chi=160: worst spectra %.2e kappa rel %.2e" % (worst, abs(kg - ko) / abs(ko)))
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    g.close()
