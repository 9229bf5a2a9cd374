"""Batched form through the C ABI: many independent 1x1 instances with uneven
(D, chi) in one context.  Instances with equal (d, D, chi) are moved in
lock-step with grouped launches; with use_graph a whole sweep of every
instance is one captured HIP graph.

Checks: every instance of a mixed batch matches the float64 oracle run on its
own (spectra after each sweep to 1e-8, kappa to 1e-10); the graph replays
reproduce the eager batched run exactly; the batched run matches one context
per instance (to 1e-8 in the spectra: the solver's random start columns
differ, and the directions near the cutoff are fixed only to that level).
"""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs

pytestmark = pytest.mark.gpu


def _spec_oracle(env):
    sp = octm.corner_spectra(env)
    return np.array([[sp[(0, 0)][c] for c in range(4)]])


def _mixed(seed, n, d, Ds, chis):
    return synth.batched_instances(seed, n, d=d, Ds=Ds, chis=chis)


def test_batched_fp64_matches_oracle(gpu):
    """Seven instances, three shape classes (one of a single instance), float64:
    every instance after each of three sweeps against its own oracle run."""
    from paper_1711_04798_amd import CTM
    inst = _mixed(21, 7, 2, (2, 3), (8, 12))
    print("case batched fp64", [(D, c) for D, c, _ in inst], flush=True)
    g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst])
    cells = [octm.Cell(1, 1, [0], [A]) for _, _, A in inst]
    envs = [octm.init_trivial(cell, c) for cell, (_, c, _) in zip(cells, inst)]
    for sw in range(3):
        g.sweep(1)
        for i, (cell, env) in enumerate(zip(cells, envs)):
            octm.sweep(cell, env)
            err = np.abs(_spec_oracle(env) - g.spectra(i)).max()
            assert err < 1e-8, (sw, i, err)
    for i, (cell, env) in enumerate(zip(cells, envs)):
        ko, kg = oobs.kappa(cell, env), g.norm(i)
        assert abs(kg - ko) <= 1e-10 * abs(ko), (i, kg, ko)
    g.close()


def _run(inst, use_graph, tol, max_sweeps, prec="fp32"):
    from paper_1711_04798_amd import CTM
    g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst], prec=prec, max_iters=2,
            resid_tol=0.0, cutoff=1e-6, use_graph=use_graph)
    sw, dl, ok = g.converge(tol=tol, max_sweeps=max_sweeps)
    spec = [g.spectra(i) for i in range(len(inst))]
    kap = [g.norm(i) for i in range(len(inst))]
    g.close()
    return sw, dl, ok, spec, kap


def test_graph_replays_match_eager(gpu):
    """d=8 instances of three classes in float32: the captured-graph sweeps
    (replayed until every instance converged, with host reads in between) give
    the same environments as the eager batched sweeps."""
    inst = _mixed(3, 9, 8, (2, 3), (16, 24))
    print("case graph vs eager", [(D, c) for D, c, _ in inst], flush=True)
    # same number of sweeps for both (tol 0 never converges)
    sw_e, _, _, spec_e, kap_e = _run(inst, False, 0.0, 6)
    sw_g, _, _, spec_g, kap_g = _run(inst, True, 0.0, 6)
    assert sw_e == sw_g == [6] * len(inst)
    for i in range(len(inst)):
        assert np.abs(spec_e[i] - spec_g[i]).max() < 1e-12, i
        assert abs(kap_e[i] - kap_g[i]) <= 1e-12 * abs(kap_e[i]), i


def test_batched_matches_separate_contexts(gpu):
    """The grouped launches compute what one context per instance computes
    (float64, converged solver, so the solver's random start does not matter)."""
    from paper_1711_04798_amd import CTM
    inst = _mixed(5, 6, 8, (2, 3), (16, 24))
    print("case batched vs plain", flush=True)
    g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst])
    g.sweep(3)
    spec_b = [g.spectra(i) for i in range(len(inst))]
    kap_b = [g.norm(i) for i in range(len(inst))]
    g.close()
    for i, (D, c, A) in enumerate(inst):
        p = CTM([[A]], chi=c)
        p.sweep(3)
        assert np.abs(spec_b[i] - p.spectra()).max() < 1e-8, i
        assert abs(kap_b[i] - p.norm()) <= 1e-10 * abs(kap_b[i]), i
        p.close()


def test_batched_converges_per_instance(gpu):
    """Every instance reports the sweep at which its own change fell below tol."""
    inst = _mixed(8, 5, 8, (2, 3), (16, 24))
    print("case batched converge", flush=True)
    sw, dl, ok, _, _ = _run(inst, True, 1e-4, 60)
    assert ok, (sw, dl)
    assert all(d < 1e-4 for d in dl) and all(1 <= s <= 60 for s in sw)
