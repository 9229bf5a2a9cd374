"""GPU observables, fidelity, checkpointing and error paths, through the C ABI,
against the CPU float64 oracle on the same seeded inputs.

Tolerances: kappa, energies and fidelities to 1e-10 relative in float64 after
the same number of sweeps; lock-step corner spectra to 1e-8 (see the
parity-test module for why spectra are looser).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs
from oracle import models

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ORDER = ["L", "R", "U", "D"]
BONDS = [(x, y, v) for v in (False, True) for y in range(2) for x in range(2)]


def _spec_oracle(env, Lx, Ly):
    sp = octm.corner_spectra(env)
    return np.array([[sp[(x, y)][c] for c in range(4)] for y in range(Ly) for x in range(Lx)])


def _gpu_energy(g, bond_h):
    vals = []
    for (x, y, v) in BONDS:
        h = bond_h(x, y, v)
        vals.append(g.expect(x, y, v, h))
    return float(np.sum(vals)), vals


def test_c1_one_sweep_lockstep(gpu):
    """2x2 checkerboard at ruby size (d=8, D=4, chi=64), float64: spectra after
    every column step of one sweep, then kappa and the eight bond energies of
    the ruby model."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(0, 8, 4, 2)
    print("case c1 lockstep", flush=True)
    # relative cutoff 1e-8: kept directions are fixed well above float64 noise
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=64, cutoff=1e-8)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, 64)
    for dn in ORDER:
        k = octm.DIRS[dn]
        for xp in range(2):
            octm.column_step(cell, env, k, xp, cutoff=1e-8)
            g.move(dn, 1)
            err = np.abs(_spec_oracle(env, 2, 2) - g.spectra()).max()
            assert err < 1e-8, (dn, xp, err)
    ko, kg = oobs.kappa(cell, env), g.norm()
    assert abs(kg - ko) <= 1e-10 * abs(ko)
    bh = models.ruby_bond_h()
    eo, vo = oobs.energy(cell, env, bh)
    eg, vg = _gpu_energy(g, bh)
    g.close()
    scale = max(abs(eo), 1e-3)
    assert abs(eg - eo) <= 1e-10 * scale, (eg, eo)
    assert np.abs(np.array(vg) - np.array(vo)).max() <= 1e-10 * scale


def _golden(name):
    p = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(p):
        pytest.skip("golden file %s not generated" % p)
    return json.load(open(p))


def test_c1_converged(gpu):
    """float64 GPU CTM from the trivial start, converged, against the oracle's
    converged environment (stored by tests/golden/make_golden.py): kappa, the
    energy per spin and the corner spectra."""
    from paper_1711_04798_amd import CTM
    gold = _golden("c1")
    w = gold["workload"]
    A, B = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    print("case c1 converged", flush=True)
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=w["chi"], cutoff=w["cutoff"])
    sw, dl, ok = g.converge(tol=w["tol"], max_sweeps=w["max_sweeps"])
    assert ok == gold["converged"], (sw, dl)
    kg = g.norm()
    eg, _ = _gpu_energy(g, models.ruby_bond_h())
    sg = g.spectra()
    g.close()
    so = np.array(gold["spectra"])
    print("c1: gpu sweeps %d delta %.2e (oracle %d); kappa rel %.2e; E/spin %.15f vs %.15f; spectra %.2e"
          % (sw[0], dl[0], gold["sweeps"], abs(kg - gold["kappa"]) / gold["kappa"], eg / 12,
             gold["energy_per_spin"], np.abs(sg - so).max()))
    assert abs(kg - gold["kappa"]) <= 1e-10 * abs(gold["kappa"])
    assert abs(eg / 12 - gold["energy_per_spin"]) <= 1e-10 * max(abs(gold["energy_per_spin"]), 1e-3)
    assert np.abs(sg - so).max() < 1e-8


def test_c2_converged(gpu):
    """The benchmark workload (2x2, d=8, D=6, chi=144) in float64 on the GPU,
    converged from the trivial start, against the oracle's converged
    environment (tests/golden/make_golden.py, cutoff 1e-8, Delta < 1e-8):
    kappa, the energy per spin and the corner spectra.  The bounds allow for
    the 1e-8 convergence threshold of both runs."""
    import time
    from paper_1711_04798_amd import CTM
    gold = _golden("c2")
    w = gold["workload"]
    A, B = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    print("case c2 converged", flush=True)
    t0 = time.time()
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=w["chi"], cutoff=w["cutoff"])
    sw, dl, ok = g.converge(tol=w["tol"], max_sweeps=w["max_sweeps"])
    assert ok == gold["converged"], (sw, dl)
    kg = g.norm()
    eg, _ = _gpu_energy(g, models.ruby_bond_h())
    sg = g.spectra()
    g.close()
    so = np.array(gold["spectra"])
    print("c2: gpu sweeps %d delta %.2e (oracle %d) in %.1f s; kappa rel %.2e; E/spin %.15f vs %.15f; spectra %.2e"
          % (sw[0], dl[0], gold["sweeps"], time.time() - t0, abs(kg - gold["kappa"]) / gold["kappa"], eg / 12,
             gold["energy_per_spin"], np.abs(sg - so).max()))
    assert abs(kg - gold["kappa"]) <= 1e-9 * abs(gold["kappa"])
    assert abs(eg / 12 - gold["energy_per_spin"]) <= 1e-9 * max(abs(gold["energy_per_spin"]), 1e-3)
    assert np.abs(sg - so).max() < 1e-7


def test_fidelity_gpu(gpu):
    """Fidelity per site of two nearby 1x1 states (d=2, D=2, chi=16) against
    the oracle's three converged runs; d(A, A) = 1."""
    from paper_1711_04798_amd import binding
    rng = np.random.default_rng(5)
    A, = synth.cell_tensors(11, 2, 2, 1)
    B = A + 0.3 * synth.peps_tensor(rng, 2, 2)
    B /= np.linalg.norm(B)
    print("case fidelity", flush=True)
    dg, lg, sw, conv = binding.fidelity([A], [B], chi=16, tol=1e-12, max_sweeps=300)
    assert conv and max(sw) < 300, sw
    kap = {}
    for name, kets, bras in (("ab", [A], [B]), ("aa", [A], None), ("bb", [B], None)):
        cell = octm.Cell(1, 1, [0], kets, bras)
        env = octm.init_trivial(cell, 16)
        octm.converge(cell, env, tol=1e-12, max_sweeps=300)
        kap[name] = oobs.kappa(cell, env)
    do = oobs.fidelity(kap["ab"], kap["aa"], kap["bb"])
    print("fidelity gpu %.15f oracle %.15f sweeps %s" % (dg, do, sw))
    assert 0 < dg <= 1 + 1e-12
    assert abs(dg - do) <= 1e-10 * abs(do)
    assert abs(lg - np.log(dg)) < 1e-12
    d1, l1, sw1, conv1 = binding.fidelity([A], [A], chi=16, tol=1e-12, max_sweeps=300)
    assert conv1 and max(sw1) < 300, sw1
    assert abs(d1 - 1.0) < 1e-10 and abs(l1) < 1e-10
    # a budget too small to converge: the value is still returned, with the status
    d2, _, sw2, conv2 = binding.fidelity([A], [B], chi=16, tol=1e-12, max_sweeps=2)
    assert not conv2 and sw2 == [2, 2, 2] and np.isfinite(d2)


def test_checkpoint_roundtrip(gpu):
    """Export after three sweeps, import into a fresh context: the exported
    bytes round-trip exactly and two more sweeps agree with the uninterrupted
    run (the solver's random start differs, so to rounding, not bitwise)."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(2, 2, 3, 2)
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=12)
    print("case checkpoint", flush=True)
    g1 = CTM([[A, B]], **kw)
    g1.sweep(3)
    buf = g1.export_env()
    g2 = CTM([[A, B]], **kw)
    g2.import_env(buf)
    assert np.array_equal(g2.export_env(), buf)
    g1.sweep(2)
    g2.sweep(2)
    s1, s2 = g1.spectra(), g2.spectra()
    k1, k2 = g1.norm(), g2.norm()
    g1.close()
    g2.close()
    assert np.abs(s1 - s2).max() < 1e-9
    assert abs(k1 - k2) <= 1e-10 * abs(k1)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_checkpoint_resume_bitwise(gpu, prec):
    """A run converged in two pieces, with a checkpoint saved after the first
    and loaded into a fresh context, ends bitwise equal to the run done in
    one piece: environment, spectra, kappa, sweep count and Delta."""
    from paper_1711_04798_amd import CTM
    if prec == "fp64":
        A, B = synth.cell_tensors(2, 2, 3, 2)
        kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24, cutoff=1e-8)
    else:
        A, B = synth.cell_tensors(3, 8, 3, 2)
        kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=32, prec="bf16", max_iters=2, resid_tol=0.0,
                  cutoff=1e-6)
    print("case checkpoint bitwise", prec, flush=True)
    g1 = CTM([[A, B]], **kw)
    g1.converge(tol=0.0, max_sweeps=3)
    s_a, d_a, _ = g1.converge(tol=0.0, max_sweeps=3)
    ref = (g1.export_env(), g1.spectra(), g1.norm(), d_a)
    g2 = CTM([[A, B]], **kw)
    g2.converge(tol=0.0, max_sweeps=3)
    ck = g2.save_checkpoint()
    g2.close()
    g3 = CTM([[A, B]], **kw)
    g3.load_checkpoint(ck)
    s_b, d_b, _ = g3.converge(tol=0.0, max_sweeps=3)
    got = (g3.export_env(), g3.spectra(), g3.norm(), d_b)
    g1.close()
    g3.close()
    assert np.array_equal(ref[0], got[0])
    assert np.array_equal(ref[1], got[1])
    assert ref[2] == got[2] and ref[3] == got[3] and s_a == s_b


def test_width_grows_when_filled(gpu):
    """With two oversampling columns the subspace width (chi_eff + 2) is often
    filled by the kept count; a converged run may then not stop at a check
    where that happened, and moves after it grow the width: the converged
    environment matches the oracle's (no width limit) and so do further
    lock-step moves."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(6, 2, 3, 2)
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=24, cutoff=1e-8, oversample=2)
    print("case width growth", flush=True)
    g = CTM([[A, B]], **kw)
    sw, dl, ok = g.converge(tol=1e-10, max_sweeps=200)
    assert ok, (sw, dl)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, 24)
    octm.converge(cell, env, tol=1e-10, max_sweeps=200, cutoff=1e-8)
    so = _spec_oracle(env, 2, 2)
    assert np.abs(g.spectra() - so).max() < 1e-7
    assert abs(g.norm() - oobs.kappa(cell, env)) <= 1e-9 * abs(oobs.kappa(cell, env))
    g.close()


def test_metrics_lines(gpu, tmp_path):
    """Per-check metrics of a float64 run to convergence (2x2, d=8, D=4,
    chi=64): one JSON line per sweep, whose last change and norm per site are
    the ones the run returns, with kept counts within the width and
    discarded weights in [0, 1)."""
    from paper_1711_04798_amd import CTM
    gold = _golden("c1")
    w = gold["workload"]
    A, B = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    print("case metrics", flush=True)
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=w["chi"], cutoff=w["cutoff"])
    path = tmp_path / "m.jsonl"
    g.set_metrics(path, kappa=True)
    sw, dl, ok = g.converge(tol=w["tol"], max_sweeps=w["max_sweeps"])
    g.set_metrics(None)
    kg = g.norm()
    g.close()
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    assert ok and len(lines) == sw[0]
    assert [m["sweep"] for m in lines] == list(range(1, sw[0] + 1))
    last = lines[-1]
    print("metrics: %d lines, last delta %.3e kappa %.12f width %d live %d chi_eff %s discarded %s"
          % (len(lines), last["delta"], last["kappa"], last["width"], last["live_chi"], last["chi_eff"]["L"],
             last["discarded"]["L"]))
    assert abs(last["delta"] - dl[0]) <= 1e-6 * dl[0]
    assert abs(last["kappa"] - kg) <= 1e-6 * kg
    for m in lines:
        assert m["width"] <= w["chi"] + 16 and m["live_chi"] <= w["chi"]
        for dn in "LRUD":
            assert len(m["chi_eff"][dn]) == 4
            assert all(0 < c <= m["width"] for c in m["chi_eff"][dn])
            assert all(0 <= v < 1 for v in m["discarded"][dn])
            assert all(0 <= v < 1e-6 for v in m["max_resid"][dn])


def test_deterministic(gpu):
    """Two contexts on the same input give bit-identical spectra and kappa."""
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(4, 2, 3, 2)
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=12)
    print("case determinism", flush=True)
    out = []
    for _ in range(2):
        g = CTM([[A, B]], **kw)
        g.sweep(3)
        out.append((g.spectra(), g.norm()))
        g.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_nonfinite_input_rejected(gpu):
    from paper_1711_04798_amd import CTM, binding
    A, = synth.cell_tensors(0, 2, 2, 1)
    A = A.copy()
    A[1, 0, 1, 0, 1] = np.nan
    print("case nonfinite", flush=True)
    with pytest.raises(binding.CtmError) as e:
        CTM([[A]], chi=8)
    assert e.value.status == binding.CTM_E_NONFINITE


def test_not_converged_keeps_valid_state(gpu):
    """max_sweeps reached: CTM_E_NOCONV is reported, the state stays usable."""
    from paper_1711_04798_amd import CTM
    A, = synth.cell_tensors(0, 2, 2, 1)
    print("case noconv", flush=True)
    g = CTM([[A]], chi=16)
    sw, dl, ok = g.converge(tol=1e-300, max_sweeps=2)
    assert not ok and sw[0] == 2 and np.isfinite(dl[0])
    k = g.norm()
    g.close()
    cell = octm.Cell(1, 1, [0], [A])
    env = octm.init_trivial(cell, 16)
    for _ in range(2):
        octm.sweep(cell, env)
    assert abs(k - oobs.kappa(cell, env)) <= 1e-10 * abs(k)
