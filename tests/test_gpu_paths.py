"""GPU paths checked element by element or move by move against the CPU
float64 oracle on the same seeded inputs, through the C ABI:

* the diagonal start (warm start) in lock-step;
* the batched form at the benchmark's per-instance shapes (d = 8,
  D in {3, 4, 5} x chi in {32, 64, 100}) in lock-step, float64;
* the 2x2 checkerboard with A != B related by orthogonal bond gauges (Ising
  model) in lock-step, then against the exact solution;
* the fidelity per site on the 2x2 checkerboard;
* the two-site density matrix at d = 8, element by element;
* reduced-precision enlarged corners, element by element against a bound
  from the rounding of each stage.

Spectra are compared to 1e-8 absolute after every column step (directions
near the relative cutoff 1e-8 are fixed by float64 only to that level);
kappa, fidelity and density matrices to 1e-10 relative.
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


def _orth(rng, n):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q


def _checkerboard_gauge(A, O1, O2, O3, O4):
    Ap = np.einsum("suldr,uU,lL,dE,rR->sULER", A, O4, O2, O3, O1)
    Bp = np.einsum("suldr,uU,lL,dE,rR->sULER", A, O3, O1, O4, O2)
    return Ap, Bp


def _lockstep(g, cell, env, Lx, Ly, sweeps, cutoff, tol=1e-8, inst=0):
    worst = 0.0
    for sw in range(sweeps):
        for dn in ORDER:
            k = octm.DIRS[dn]
            lx, _ = octm.frame_dims(k, Lx, Ly)
            for xp in range(lx):
                octm.column_step(cell, env, k, xp, cutoff=cutoff)
                g.move(dn, 1)
                err = np.abs(_spec_oracle(env, Lx, Ly) - g.spectra(inst)).max()
                worst = max(worst, err)
                assert err < tol, (sw, dn, xp, err)
    return worst


@pytest.mark.parametrize("cell_kind", ["1x1", "2x2"])
def test_diag_start_lockstep(gpu, cell_kind):
    """CTM_INIT_DIAG: C_i = diag(s_i), T = delta_ab delta_uu' (normalised) from
    the same spectra on both sides; spectra after every column step of two
    sweeps, then kappa."""
    from paper_1711_04798_amd import CTM
    if cell_kind == "1x1":
        tens, Lx, Ly, pat, chi = synth.cell_tensors(8, 2, 2, 1), 1, 1, [0], 12
    else:
        tens, Lx, Ly, pat, chi = synth.cell_tensors(9, 2, 2, 2), 2, 2, [0, 1, 1, 0], 8
    rng = np.random.default_rng(10)
    spec = np.sort(rng.uniform(0.05, 1.0, (Lx * Ly, 4, chi)), axis=2)[:, :, ::-1].copy()
    print("case diag start", cell_kind, flush=True)
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pat, chi=chi, cutoff=1e-8, init="diag", spectrum=spec[None])
    cell = octm.Cell(Lx, Ly, pat, tens)
    env = octm.init_diag(cell, chi, {(x, y): list(spec[y * Lx + x]) for y in range(Ly) for x in range(Lx)})
    # the starting spectra themselves
    assert np.abs(_spec_oracle(env, Lx, Ly) - g.spectra()).max() < 1e-14
    worst = _lockstep(g, cell, env, Lx, Ly, 2, 1e-8)
    ko, kg = oobs.kappa(cell, env), g.norm()
    g.close()
    print("diag start %s: worst spectra %.2e, kappa rel %.2e" % (cell_kind, worst, abs(kg - ko) / abs(ko)))
    assert abs(kg - ko) <= 1e-10 * abs(ko)


def test_batched_benchmark_shapes_lockstep(gpu):
    """One instance for each (D, chi) of the batched benchmark, d = 8, float64,
    all in one batched context: each instance against its own oracle run,
    spectra after every column step of two sweeps, then kappa."""
    from paper_1711_04798_amd import CTM
    rng = np.random.default_rng(11)
    inst = [(D, chi, synth.peps_tensor(rng, 8, D)) for D in (3, 4, 5) for chi in (32, 64, 100)]
    print("case batched shapes", [(D, c) for D, c, _ in inst], flush=True)
    g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst], cutoff=1e-8)
    cells = [octm.Cell(1, 1, [0], [A]) for _, _, A in inst]
    envs = [octm.init_trivial(cell, c) for cell, (_, c, _) in zip(cells, inst)]
    for sw in range(2):
        for dn in ORDER:
            g.move(dn, 1)
            for i, (cell, env) in enumerate(zip(cells, envs)):
                octm.column_step(cell, env, octm.DIRS[dn], 0, cutoff=1e-8)
                err = np.abs(_spec_oracle(env, 1, 1) - g.spectra(i)).max()
                assert err < 1e-8, (sw, dn, inst[i][:2], err)
        print("sweep %d done" % sw, flush=True)
    for i, (cell, env) in enumerate(zip(cells, envs)):
        ko, kg = oobs.kappa(cell, env), g.norm(i)
        assert abs(kg - ko) <= 1e-10 * abs(ko), (inst[i][:2], kg, ko)
    g.close()


def test_gauged_checkerboard_lockstep(gpu):
    """Ising PEPS at K = 0.3 on the 2x2 checkerboard with A != B (orthogonal
    bond gauges): spectra after every column step of three sweeps against
    the oracle, then kappa and <zz> on all four bonds after 40 sweeps
    against the oracle and the exact solution."""
    from paper_1711_04798_amd import CTM
    from test_oracle_pins import onsager_lnz_1d, onsager_zz
    K = 0.3
    rng = np.random.default_rng(17)
    Ap, Bp = _checkerboard_gauge(models.ising_peps(K), *[_orth(rng, 2) for _ in range(4)])
    print("case gauged checkerboard", flush=True)
    g = CTM([[Ap, Bp]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=32)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [Ap, Bp])
    env = octm.init_trivial(cell, 32)
    _lockstep(g, cell, env, 2, 2, 3, 1e-12)
    g.sweep(37)
    for _ in range(37):
        octm.sweep(cell, env)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    assert abs(np.log(kg) - onsager_lnz_1d(K)) < 1e-9
    zz = np.kron(models.SZ, models.SZ)
    for v in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            zg = g.expect(x, y, v, zz)
            zo = np.trace(oobs.rdm(cell, env, x, y, v) @ zz)
            assert abs(zg - zo) < 1e-10 and abs(zg - onsager_zz(K)) < 1e-9, (v, x, y, zg, zo)
    g.close()


def test_fidelity_checkerboard(gpu):
    """Fidelity per site of two nearby 2x2 checkerboard states (d = 2, D = 2,
    chi = 16) against the oracle's three converged runs, float64."""
    from paper_1711_04798_amd import binding
    rng = np.random.default_rng(12)
    A = synth.cell_tensors(13, 2, 2, 2)
    B = [a + 0.2 * synth.peps_tensor(rng, 2, 2) for a in A]
    B = [b / np.linalg.norm(b) for b in B]
    print("case fidelity checkerboard", flush=True)
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=16)
    dg, lg, sw, conv = binding.fidelity(A, B, tol=1e-11, max_sweeps=300, cutoff=1e-8, **kw)
    assert conv and max(sw) < 300, sw
    kap = {}
    for name, kets, bras in (("ab", A, B), ("aa", A, None), ("bb", B, None)):
        cell = octm.Cell(2, 2, [0, 1, 1, 0], kets, bras)
        env = octm.init_trivial(cell, 16)
        octm.converge(cell, env, tol=1e-11, max_sweeps=300, cutoff=1e-8)
        kap[name] = oobs.kappa(cell, env)
    do = oobs.fidelity(kap["ab"], kap["aa"], kap["bb"])
    print("checkerboard fidelity gpu %.15f oracle %.15f sweeps %s" % (dg, do, sw))
    assert 0 < dg <= 1 + 1e-12
    assert abs(dg - do) <= 1e-10 * abs(do)


def test_rdm_d8_elementwise(gpu):
    """Two-site density matrices of the ruby-size checkerboard (d = 8, D = 4,
    chi = 64, 64 x 64) after one lock-step sweep, element by element, on all
    four horizontal and vertical bonds of the cell."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(0, 8, 4, 2)
    print("case rdm d8", flush=True)
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=64, cutoff=1e-8)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, 64)
    for dn in ORDER:
        for xp in range(2):
            octm.column_step(cell, env, octm.DIRS[dn], xp, cutoff=1e-8)
        g.move(dn, 2)
    for v in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            ro = oobs.rdm(cell, env, x, y, v)
            rg, herm = g.rdm(x, y, v)
            err = np.abs(rg - ro).max() / np.abs(ro).max()
            print("rho bond (%d,%d,%d): max elementwise rel err %.2e, herm defect %.1e" % (x, y, v, err, herm))
            assert err <= 1e-10
            assert abs(herm - oobs.herm_defect(ro)) <= 1e-9
    g.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
@pytest.mark.parametrize("D,chi", [(2, 16), (4, 12)])
def test_reduced_precision_corners_elementwise(gpu, prec, D, chi):
    """Enlarged corners of the reduced-precision paths from an imported oracle
    environment, element by element.  Each stage rounds its operands or its
    output once to the working type (C, the edges and the double layer; the
    stage outputs X and Y), and accumulates in fp32; every rounding error of an
    element is at most u times the same contraction taken over absolute
    values.  Bound per element: (8 u + K u_fp32) (|C| |T| |T| |a|)_ij with K
    the total contraction length of the three stages."""
    from paper_1711_04798_amd import CTM
    from test_gpu_stages import _dump, env_to_flat
    tens = synth.cell_tensors(7, 2, D, 2)
    Lx = Ly = 2
    pat = [0, 1, 1, 0]
    cell = octm.Cell(Lx, Ly, pat, tens)
    env = octm.init_trivial(cell, chi)
    for _ in range(3):
        octm.sweep(cell, env)
    print("case elementwise corners", prec, D, chi, flush=True)
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pat, chi=chi, prec=prec, max_iters=2, resid_tol=0.0, cutoff=1e-6)
    g.import_env(env_to_flat(env, Lx, Ly))
    g.move("L", 1)
    n = chi * D * D
    u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -24
    K = 2 * chi + D ** 4
    fr = octm._Frame(cell, env, 0)
    for yp in range(2):
        Qo = octm.plaquette_corners(fr, 0, yp)
        cx, cy = [0, 1, 1, 0], [yp, yp, yp + 1, yp + 1]
        for q in range(4):
            a = octm.rot_a(fr.a(cx[q], cy[q]), q)
            Qabs = octm.enlarged_corner(np.abs(fr.C(q, cx[q], cy[q])), np.abs(fr.T(q, cx[q], cy[q])),
                                        np.abs(fr.T((q + 3) % 4, cx[q], cy[q])), np.abs(a))
            Qg = _dump(g, 0, 4 * yp + q, (n, n), np.float32).astype(np.float64)
            bound = (8 * u + K * 2.0 ** -24) * Qabs
            ratio = np.max(np.abs(Qg - Qo[q]) / (bound + 1e-300))
            print("%s Q%d row %d: max |dQ| / bound %.3f" % (prec, q + 1, yp, ratio))
            assert np.all(np.abs(Qg - Qo[q]) <= bound)
    g.close()


def test_set_corner_spectra_lockstep(gpu):
    """ctm_set_corner_spectra (the corners of a running environment get new
    singular values, vectors kept) against the same operation in the oracle:
    two sweeps from the trivial start, the injection, then two lock-step
    sweeps.  The new values are zero wherever a corner's own singular value
    is below 1e-10 of its largest (there the singular vectors are not
    determined, by either side)."""
    from paper_1711_04798_amd import CTM
    A = synth.cell_tensors(14, 2, 2, 1)[0]
    chi = 8
    print("case set corner spectra", flush=True)
    g = CTM([[A]], chi=chi, cutoff=1e-8)
    cell = octm.Cell(1, 1, [0], [A])
    env = octm.init_trivial(cell, chi)
    g.sweep(2)
    for _ in range(2):
        octm.sweep(cell, env, cutoff=1e-8)
    rng = np.random.default_rng(15)
    new = np.zeros((1, 4, chi))
    for i in range(4):
        U, s, Vh = np.linalg.svd(env.C[i][(0, 0)])
        r = int(np.sum(s > 1e-10 * s[0]))
        new[0, i, :r] = np.sort(rng.uniform(0.1, 1.0, r))[::-1]
        C = U @ np.diag(new[0, i]) @ Vh
        env.C[i][(0, 0)] = C / np.linalg.norm(C)
    g.set_corner_spectra(new)
    so = _spec_oracle(env, 1, 1)
    assert np.abs(so - g.spectra()).max() < 1e-12
    assert np.abs(so[0] - new[0] / new[0].sum(axis=1, keepdims=True)).max() < 1e-14
    _lockstep(g, cell, env, 1, 1, 2, 1e-8)
    ko, kg = oobs.kappa(cell, env), g.norm()
    g.close()
    assert abs(kg - ko) <= 1e-10 * abs(ko)


def test_ruby_trivial_legs_by_padding(gpu):
    """Ruby-faithful block tensors (d = 8: A with a trivial down leg, B with a
    trivial up leg, the other legs D = 3) run on the GPU zero-padded to D = 3
    on every leg, against the oracle with the true D = 1 legs: corner spectra
    after every column step of two sweeps, then kappa and the eight bond
    energies of the ruby model.  (On this brick wall every corner matrix
    stays rank 1 -- each corner absorbs its edges through a missing bond --
    so the environment lives in the edges, and kappa and the energies are
    the informative checks.)"""
    from paper_1711_04798_amd import CTM
    from test_oracle_pins import ruby_trivial_leg_tensors, pad_legs
    A, B = ruby_trivial_leg_tensors(42, 8, 3)
    print("case ruby trivial legs", flush=True)
    g = CTM([[pad_legs(A, 3), pad_legs(B, 3)]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24, cutoff=1e-8)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, 24)
    worst = _lockstep(g, cell, env, 2, 2, 2, 1e-8)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    bh = models.ruby_bond_h()
    for v in (False, True):
        for x, y in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            h = bh(x, y, v)
            eo = float(np.real(np.trace(oobs.rdm(cell, env, x, y, v) @ h)))
            eg = g.expect(x, y, v, h)
            assert abs(eg - eo) <= 1e-10 * max(1.0, abs(eo)), (x, y, v, eg, eo)
    g.close()
    print("ruby trivial legs: worst spectra %.2e, kappa rel %.2e" % (worst, abs(kg - ko) / abs(ko)))
