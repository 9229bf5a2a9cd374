"""Single-layer contractions (the ket tensor and the bra tensor absorbed one at
a time, Sec. II D) against the oracle, which forms the double layer: the
enlarged corners element by element, the projectors, the moved environment,
converged observables, mixed (fidelity) networks with a bra different from
the ket, the batched form in graph mode, and a bond dimension D = 8.

Tolerances: float64 as in the double-layer parity tests (corners 1e-13 of
the largest element, truncated half-system operator 1e-11, norm per site
1e-10, lock-step spectra 1e-8); float32 and bf16 element by element
against the rounding bound of the contraction chain.
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


@pytest.mark.parametrize("direction", ["L", "U", "R", "D"])
@pytest.mark.parametrize("d,D,chi,bra", [(2, 2, 8, False), (3, 3, 10, True)])
def test_single_layer_one_step(gpu, direction, d, D, chi, bra):
    """From the oracle's environment after three sweeps, one column step in
    single-layer float64: the eight enlarged corners, the truncated
    half-system operator Uh^T P1 P2 Lh^T and the norm per site of the moved
    environment; with bra, the bra tensors differ from the kets (the mixed
    network of the fidelity)."""
    from paper_1711_04798_amd import CTM
    from test_gpu_stages import _dump, env_to_flat
    kets = synth.cell_tensors(11, d, D, 2)
    bras = synth.cell_tensors(12, d, D, 2) if bra else None
    Lx = Ly = 2
    pat = [0, 1, 1, 0]
    cell = octm.Cell(Lx, Ly, pat, kets, bras)
    env = octm.init_trivial(cell, chi)
    for _ in range(3):
        octm.sweep(cell, env)
    print("case single layer", direction, d, D, chi, bra, flush=True)
    g = CTM([kets], Lx=Lx, Ly=Ly, pattern=pat, chi=chi, bras=[bras] if bra else None, single_layer=True)
    g.import_env(env_to_flat(env, Lx, Ly))
    k = octm.DIRS[direction]
    g.move(direction, 1)
    n = chi * D * D
    fr = octm._Frame(cell, env, k)
    for yp in range(fr.Ly):
        Qo = octm.plaquette_corners(fr, 0, yp)
        for q in range(4):
            Qg = _dump(g, 0, 4 * yp + q, (n, n))
            err = np.abs(Qg - Qo[q]).max() / np.abs(Qo[q]).max()
            print("Q%d row %d rel err %.2e" % (q + 1, yp, err))
            assert err < 1e-13
        P1o, P2o, info = octm.projectors(*Qo, chi, 1e-12, return_info=True)
        P1g = _dump(g, 1, yp, (n, chi))
        P2g = _dump(g, 2, yp, (n, chi)).T
        Uh, Lh = Qo[0] @ Qo[1], Qo[2] @ Qo[3]
        No, Ng = Uh.T @ P1o @ P2o @ Lh.T, Uh.T @ P1g @ P2g @ Lh.T
        err = np.abs(No - Ng).max() / np.abs(No).max()
        print("row %d N_chi rel err %.2e" % (yp, err))
        assert err < 1e-11
    ref = env.copy()
    octm.column_step(cell, ref, k, 0)
    # the norm per site of the moved environment, each side from its own
    ko, kg = oobs.kappa(cell, ref), g.norm()
    print("kappa after step: oracle %.15f gpu %.15f" % (ko, kg))
    assert abs(ko - kg) < 1e-10 * abs(ko)
    g.close()


@pytest.mark.parametrize("prec,d", [("fp32", 2), ("bf16", 2), ("bf16", 4)])
@pytest.mark.parametrize("D,chi", [(2, 16), (4, 12)])
def test_single_layer_reduced_corners_elementwise(gpu, prec, d, D, chi):
    """Reduced-precision single-layer corners from an imported oracle
    environment, element by element.  Each stage rounds its output once
    after accumulating in float32 (X in float32; Y and the ket-layer
    intermediate Z in the working type: float32, or bf16 in the bf16 form),
    and the tensors are rounded once; every rounding error of an element is
    at most u times the same contraction over absolute values, the double
    layer replaced by sum_s |A| |B|.  Bound: (8 u + K u_fp32)
    (|C| |T| |T| |a|)_ij with u the unit roundoff of the working type and
    K = 2 chi + D^2 + d D^2 the total contraction length.  bf16 with d = 4 runs
    the products on the bf16 corner kernel (Y gathered, the first product
    transposed), d = 2 on the generic GEMM."""
    from paper_1711_04798_amd import CTM
    from test_gpu_stages import _dump, env_to_flat
    tens = synth.cell_tensors(7, d, D, 2)
    Lx = Ly = 2
    pat = [0, 1, 1, 0]
    cell = octm.Cell(Lx, Ly, pat, tens)
    env = octm.init_trivial(cell, chi)
    for _ in range(3):
        octm.sweep(cell, env)
    print("case single layer reduced corners", prec, d, D, chi, flush=True)
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pat, chi=chi, prec=prec, max_iters=2, resid_tol=0.0, cutoff=1e-6,
            single_layer=True)
    g.import_env(env_to_flat(env, Lx, Ly))
    g.move("L", 1)
    n = chi * D * D
    u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -24
    K = 2 * chi + D * D + d * D * D
    fr = octm._Frame(cell, env, 0)
    abs_cell = octm.Cell(Lx, Ly, pat, [np.abs(t) for t in tens])
    fa = octm._Frame(abs_cell, env, 0)
    for yp in range(2):
        Qo = octm.plaquette_corners(fr, 0, yp)
        cx, cy = [0, 1, 1, 0], [yp, yp, yp + 1, yp + 1]
        for q in range(4):
            a_abs = octm.rot_a(fa.a(cx[q], cy[q]), q)
            Qabs = octm.enlarged_corner(np.abs(fr.C(q, cx[q], cy[q])), np.abs(fr.T(q, cx[q], cy[q])),
                                        np.abs(fr.T((q + 3) % 4, cx[q], cy[q])), a_abs)
            Qg = _dump(g, 0, 4 * yp + q, (n, n), np.float32).astype(np.float64)
            bound = (8 * u + K * 2.0 ** -24) * Qabs
            ratio = np.max(np.abs(Qg - Qo[q]) / (bound + 1e-300))
            print("Q%d row %d: max |dQ| / bound %.3f" % (q + 1, yp, ratio))
            assert np.all(np.abs(Qg - Qo[q]) <= bound)
    g.close()


def test_single_layer_c1_converged(gpu):
    """float64 single-layer CTM of the 2x2 ruby-size cell (d=8, D=4, chi=64)
    from the trivial start to convergence, against the oracle's converged
    environment (tests/golden/c1.json): norm per site, energy per spin of
    the ruby model and corner spectra."""
    from paper_1711_04798_amd import CTM
    from test_gpu_observables import _golden, _gpu_energy
    gold = _golden("c1")
    w = gold["workload"]
    A, B = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    print("case single layer c1 converged", flush=True)
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=w["chi"], cutoff=w["cutoff"], single_layer=True)
    sw, dl, ok = g.converge(tol=w["tol"], max_sweeps=w["max_sweeps"])
    assert ok, (sw, dl)
    kg = g.norm()
    eg, _ = _gpu_energy(g, models.ruby_bond_h())
    sg = g.spectra()
    g.close()
    so = np.array(gold["spectra"])
    print("single layer c1: sweeps %d (oracle %d); kappa rel %.2e; E/spin %.15f vs %.15f; spectra %.2e"
          % (sw[0], gold["sweeps"], abs(kg - gold["kappa"]) / gold["kappa"], eg / 12, gold["energy_per_spin"],
             np.abs(sg - so).max()))
    assert abs(kg - gold["kappa"]) <= 1e-10 * abs(gold["kappa"])
    assert abs(eg / 12 - gold["energy_per_spin"]) <= 1e-10 * max(abs(gold["energy_per_spin"]), 1e-3)
    assert np.abs(sg - so).max() < 1e-8


def test_single_layer_fidelity(gpu):
    """Fidelity per site through the single-layer route (its mixed network has
    a bra different from the ket) against the oracle's three CTM runs."""
    from paper_1711_04798_amd import binding
    A = synth.cell_tensors(21, 2, 2, 2)
    B = [a + 0.2 * b for a, b in zip(A, synth.cell_tensors(22, 2, 2, 2))]
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=12)
    print("case single layer fidelity", flush=True)
    dg, lg, sw, ok = binding.fidelity(A, B, tol=1e-11, max_sweeps=300, single_layer=True, **kw)
    assert ok, sw
    kap = []
    for kets, bras in ((A, B), (A, A), (B, B)):
        cell = octm.Cell(2, 2, [0, 1, 1, 0], kets, bras)
        env = octm.init_trivial(cell, 12)
        octm.converge(cell, env, tol=1e-11, max_sweeps=300)
        kap.append(oobs.kappa(cell, env))
    do = oobs.fidelity(*kap)
    print("single layer fidelity gpu %.15f oracle %.15f sweeps %s" % (dg, do, sw))
    assert abs(dg - do) <= 1e-9 * do


def test_single_layer_batched_graph(gpu):
    """Batched instances of mixed (D, chi) in graph mode (one captured sweep,
    the shape classes as concurrent branches) through the single-layer route:
    each converged environment against the same instance run alone through
    the double layer."""
    from paper_1711_04798_amd import CTM
    shapes = [(3, 16), (4, 12), (3, 16), (4, 12)]
    tens = [synth.cell_tensors(30 + i, 2, D, 1) for i, (D, _) in enumerate(shapes)]
    chis = [c for _, c in shapes]
    print("case single layer batched graph", flush=True)
    g = CTM(tens, chi=chis, prec="fp64", resid_tol=0.0, max_iters=6, use_graph=True, single_layer=True)
    sw, dl, ok = g.converge(tol=1e-9, max_sweeps=200)
    assert ok, (sw, dl)
    for i in range(len(shapes)):
        h = CTM([tens[i]], chi=chis[i], prec="fp64", resid_tol=0.0, max_iters=6)
        sw1, dl1, ok1 = h.converge(tol=1e-9, max_sweeps=200)
        assert ok1
        ds = np.abs(g.spectra(i) - h.spectra()).max()
        dk = abs(g.norm(i) - h.norm()) / abs(h.norm())
        print("instance %d: sweeps %d vs %d, spectra %.2e, kappa rel %.2e" % (i, sw[i], sw1[0], ds, dk))
        assert ds < 1e-6 and dk < 1e-9
        h.close()
    g.close()


def test_single_layer_large_D_lockstep(gpu):
    """Bond dimension D = 8 (the double layer has D^8 = 1.7e7 entries per
    rotation): one sweep of the 1x1 cell from the trivial start in
    single-layer float64, corner spectra after every move against the
    oracle's."""
    from paper_1711_04798_amd import CTM
    (A,) = synth.cell_tensors(5, 2, 8, 1)
    chi = 16
    print("case single layer D=8", flush=True)
    g = CTM([[A]], chi=chi, cutoff=1e-8, single_layer=True)
    cell = octm.Cell(1, 1, [0], [A])
    env = octm.init_trivial(cell, chi)
    for dn in ORDER:
        octm.column_step(cell, env, octm.DIRS[dn], 0, cutoff=1e-8)
        g.move(dn, 1)
        err = np.abs(_spec_oracle(env, 1, 1) - g.spectra()).max()
        print("after %s: spectra max diff %.2e" % (dn, err))
        assert err < 1e-8
    ko, kg = oobs.kappa(cell, env), g.norm()
    print("kappa oracle %.15f gpu %.15f" % (ko, kg))
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    g.close()
