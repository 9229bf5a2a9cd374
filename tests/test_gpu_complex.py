"""Complex kets on the GPU (Sec. II A: d D^4 complex coefficients per tensor),
run on the real form of the double layer (a unitary pair basis on every
doubled leg), against the oracle's complex CTM on the same tensors:

* random complex tensors, 2x2 checkerboard, d = 2, D = 2 and 3: corner
  spectra after every column step of the first sweep (1e-8), then each side
  converges on its own (spectrum change 1e-11 per sweep): spectra 1e-9, the
  norm per site 1e-10 relative, both bond density matrices element by
  element (complex, 1e-9 of their norm) and tr(rho h) for a real h.  Past
  the first sweep these workloads amplify rounding (near-degenerate values
  at the truncation): the oracle's own complex run and the same run on the
  real form of the double layer drift to 2e-8 apart in the second sweep,
  while their converged environments agree to 5e-13;
* a real PEPS under a complex unitary gauge on every bond (the same state):
  spectra, norm and density matrices equal to the GPU's real run (1e-10);
* bf16 contractions of complex tensors run and stay within the precision
  form's level of the float64 result;
* the boundary operator, the real density-matrix call and the fidelity
  refuse complex tensors.
"""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs

from test_oracle_pins import complex_gauged

pytestmark = pytest.mark.gpu

ORDER = ["L", "R", "U", "D"]


def _complex_tensors(seed, d, D, n):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        A = rng.standard_normal((d, D, D, D, D)) + 1j * rng.standard_normal((d, D, D, D, D))
        out.append(A / np.linalg.norm(A))
    return out


def _spec_oracle(env, Lx, Ly):
    sp = octm.corner_spectra(env)
    return np.array([[sp[(x, y)][c] for c in range(4)] for y in range(Ly) for x in range(Lx)])


@pytest.mark.parametrize("D,chi", [(2, 16), (3, 24)])
def test_complex_lockstep_vs_oracle(gpu, D, chi):
    from paper_1711_04798_amd import CTM
    tens = _complex_tensors(30 + D, 2, D, 2)
    print("case complex lock-step D", D, flush=True)
    g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi)
    assert g.complex
    cell = octm.Cell(2, 2, [0, 1, 1, 0], tens)
    env = octm.init_trivial(cell, chi)
    worst = 0.0
    for dn in ORDER:
        k = octm.DIRS[dn]
        lx, _ = octm.frame_dims(k, 2, 2)
        for xp in range(lx):
            octm.column_step(cell, env, k, xp)
            g.move(dn, 1)
            err = np.abs(_spec_oracle(env, 2, 2) - g.spectra()).max()
            worst = max(worst, err)
            assert err < 1e-8, (dn, xp, err)
    sw, dl, ok = g.converge(tol=1e-11, max_sweeps=300)
    so, do, oko = octm.converge(cell, env, tol=1e-11, max_sweeps=300, cutoff=1e-12)
    assert ok and oko, (sw, so)
    dconv = np.abs(_spec_oracle(env, 2, 2) - g.spectra()).max()
    ko, kg = oobs.kappa(cell, env), g.norm()
    print("complex D=%d: worst first-sweep spectra %.2e, converged (gpu %d, oracle %d sweeps) spectra %.2e, "
          "kappa oracle %s gpu %.15f" % (D, worst, sw[0], so, dconv, ko, kg))
    assert dconv < 1e-9
    assert abs(np.imag(ko)) < 1e-12 * abs(ko) and abs(kg - np.real(ko)) <= 1e-10 * abs(ko)
    h = np.random.default_rng(1).standard_normal((4, 4))
    h = h + h.T
    for v in (False, True):
        ro = oobs.rdm(cell, env, 1, 1, v)
        rg, herm = g.rdm(1, 1, v)
        assert np.iscomplexobj(rg)
        err = np.linalg.norm(rg - ro) / np.linalg.norm(ro)
        print("  rdm vertical=%s: rel err %.2e, max |Im| %.2e, herm defect %.2e" % (v, err, np.abs(ro.imag).max(), herm))
        assert err <= 1e-9
        eo = np.real(np.trace(ro @ h))
        eg = g.expect(1, 1, v, h)
        assert abs(eg - eo) <= 1e-9 * max(1.0, abs(eo))
    g.close()


def test_complex_gauge_of_real_state(gpu):
    from paper_1711_04798_amd import CTM
    tens = synth.cell_tensors(4, 2, 3, 2)
    gt = complex_gauged(tens, 12)
    print("case complex gauge of a real state", flush=True)
    gr = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24)
    gc = CTM([gt], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24)
    gr.sweep(4)
    gc.sweep(4)
    ds = np.abs(gr.spectra() - gc.spectra()).max()
    kr, kc = gr.norm(), gc.norm()
    print("gauge: spectra %.2e, kappa real %.15f complex %.15f" % (ds, kr, kc))
    assert ds < 1e-10 and abs(kr - kc) <= 1e-10 * kr
    for v in (False, True):
        rr, _ = gr.rdm(0, 0, v)
        rc, _ = gc.rdm(0, 0, v)
        assert np.abs(rc - rr).max() <= 1e-10 * np.abs(rr).max()
    gr.close()
    gc.close()


def test_complex_bf16(gpu):
    """bf16 contractions (the real form of the double layer packed for the
    bf16 corner kernel) against float64 on the same complex tensors after
    eight sweeps: norm per site and density matrix at the precision form's
    level (the real tensors of this shape agree to about 1e-5)."""
    from paper_1711_04798_amd import CTM
    tens = _complex_tensors(40, 8, 4, 2)
    print("case complex bf16", flush=True)
    runs = {}
    for prec in ("fp64", "bf16"):
        opts = dict(cutoff=1e-12) if prec == "fp64" else dict(max_iters=2, resid_tol=0.0, cutoff=1e-7)
        g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=64, prec=prec, **opts)
        g.sweep(8)
        runs[prec] = (g.norm(), g.rdm(0, 0, False)[0])
        g.close()
    k64, r64 = runs["fp64"]
    k16, r16 = runs["bf16"]
    print("bf16 vs fp64: kappa rel %.2e, rdm rel %.2e" % (abs(k16 - k64) / k64,
                                                         np.linalg.norm(r16 - r64) / np.linalg.norm(r64)))
    assert abs(k16 - k64) <= 1e-4 * k64
    assert np.linalg.norm(r16 - r64) <= 1e-3 * np.linalg.norm(r64)


def test_complex_refusals(gpu):
    from paper_1711_04798_amd import CTM, binding
    tens = _complex_tensors(50, 2, 2, 1)
    g = CTM([tens], chi=8)
    with pytest.raises(binding.CtmError) as e:
        g.boundary_spectrum(2)
    assert e.value.status == binding.CTM_E_INVALID
    import ctypes
    rho = np.zeros((4, 4))
    st = binding.load().ctm_rdm(g.ctx, 0, 0, 0, 0, rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert st == binding.CTM_E_INVALID
    with pytest.raises(ValueError):
        CTM([tens], chi=8, bras=[tens])
    g.close()


def test_complex_batched_graph(gpu):
    """Several complex instances of different shapes in one context, swept by
    the captured graph with concurrent class branches, against each instance
    run alone in eager mode: spectra, norms and density matrices to 1e-12."""
    from paper_1711_04798_amd import CTM
    shapes = [(2, 2, 8), (2, 3, 12), (2, 2, 8)]
    tens = [_complex_tensors(60 + i, d, D, 1) for i, (d, D, chi) in enumerate(shapes)]
    chis = [chi for _, _, chi in shapes]
    print("case complex batched graph", flush=True)
    gb = CTM(tens, chi=chis, max_iters=3, resid_tol=0.0, cutoff=1e-10, use_graph=True)
    assert gb.complex
    sw, dl, ok = gb.converge(tol=0.0, max_sweeps=6)
    for i, (d, D, chi) in enumerate(shapes):
        g1 = CTM([tens[i]], chi=chi, max_iters=3, resid_tol=0.0, cutoff=1e-10)
        g1.converge(tol=0.0, max_sweeps=6)
        ds = np.abs(gb.spectra(inst=i) - g1.spectra()).max()
        dk = abs(gb.norm(inst=i) - g1.norm()) / g1.norm()
        rb, _ = gb.rdm(0, 0, False, inst=i)
        r1, _ = g1.rdm(0, 0, False)
        print("instance %d: spectra %.2e kappa %.2e rdm %.2e" % (i, ds, dk, np.abs(rb - r1).max()))
        assert ds < 1e-12 and dk < 1e-12 and np.abs(rb - r1).max() < 1e-12
        g1.close()
    gb.close()
