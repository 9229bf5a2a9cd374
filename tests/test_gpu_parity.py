"""Parity of the HIP path (through the C ABI) with the CPU float64 oracle on
the same seeded inputs: move-by-move corner spectra, then the norm per site
and the nearest-neighbour density matrices.

Environment tensors are defined only up to gauge, so the comparison is on
gauge-invariant quantities: normalised corner spectra, kappa, rho.

Tolerances: kappa and rho to 1e-10 relative.  Lock-step corner spectra to
1e-8 absolute: when the smallest kept singular value of the half-system
product is ~1e-8 of the largest (c0, seed 0), float64 fixes that singular
direction only to ~u / (sigma_chi / sigma_1), in the oracle's dense SVD as in
the GPU solver, and the corners inherit it.
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


def _lockstep(A_list, Lx, Ly, pattern, chi, sweeps, tol_spec, **kw):
    from paper_1711_04798_amd import CTM
    g = CTM([A_list], Lx=Lx, Ly=Ly, pattern=pattern, chi=chi, **kw)
    cell = octm.Cell(Lx, Ly, pattern, A_list)
    env = octm.init_trivial(cell, chi)
    worst = 0.0
    for sw in range(sweeps):
        for dn in ORDER:
            k = octm.DIRS[dn]
            lx, _ = octm.frame_dims(k, Lx, Ly)
            for xp in range(lx):
                octm.column_step(cell, env, k, xp)
                g.move(dn, 1)
                so = _spec_oracle(env, Lx, Ly)
                sg = g.spectra()
                err = np.abs(so - sg).max()
                worst = max(worst, err)
                assert err < tol_spec, "sweep %d dir %s col %d: spectra differ by %.3e" % (sw, dn, xp, err)
    return g, cell, env, worst


@pytest.mark.parametrize("seed", [0, 1])
def test_c0_lockstep(gpu, seed):
    """1x1 cell, d=2, D=2, chi=16: spectra after every column step, then kappa
    and both nearest-neighbour density matrices after 10 sweeps."""
    A, = synth.cell_tensors(seed, 2, 2, 1)
    print("case c0 seed", seed, flush=True)
    g, cell, env, worst = _lockstep([A], 1, 1, [0], 16, 10, 1e-8)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    for vert in (False, True):
        ro = oobs.rdm(cell, env, 0, 0, vert)
        rg, herm = g.rdm(0, 0, vert)
        assert np.linalg.norm(rg - ro) <= 1e-10 * np.linalg.norm(ro)
        assert abs(np.trace(rg) - 1.0) < 1e-13
    g.close()
    print("c0 seed %d: worst spectra diff %.2e, kappa rel %.2e" % (seed, worst, abs(kg - ko) / ko))


def test_checkerboard_small_lockstep(gpu):
    """2x2 checkerboard, d=2, D=2, chi=8 (several positions, both projector rows)."""
    A, B = synth.cell_tensors(3, 2, 2, 2)
    print("case 2x2 small", flush=True)
    g, cell, env, worst = _lockstep([A, B], 2, 2, [0, 1, 1, 0], 8, 6, 1e-8)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    for (x, y, v) in [(0, 0, False), (1, 0, False), (0, 1, True), (1, 1, True)]:
        ro = oobs.rdm(cell, env, x, y, v)
        rg, _ = g.rdm(x, y, v)
        assert np.linalg.norm(rg - ro) <= 1e-10 * np.linalg.norm(ro)
    g.close()


def test_ising_kappa(gpu):
    """Ising PEPS at K=0.3: kappa and <zz> match the oracle after 30 sweeps."""
    A = models.ising_peps(0.3)
    print("case ising", flush=True)
    from paper_1711_04798_amd import CTM
    g = CTM([[A]], chi=16)
    g.sweep(30)
    cell = octm.Cell(1, 1, [0], [A])
    env = octm.init_trivial(cell, 16)
    for _ in range(30):
        octm.sweep(cell, env)
    ko, kg = oobs.kappa(cell, env), g.norm()
    zz = np.kron(models.SZ, models.SZ)
    zo = np.trace(oobs.rdm(cell, env, 0, 0) @ zz)
    zg = g.expect(0, 0, False, zz)
    g.close()
    assert abs(kg - ko) <= 1e-10 * ko
    assert abs(zg - zo) <= 1e-10
