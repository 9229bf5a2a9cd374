"""Precision form: the double-layer stage of the enlarged corners in bf16
(fp32 accumulation), or every contraction in fp32, on MFMA; projector
solver, normalisations and master copies in float64.  The error of the
energy per spin of the ruby model (all couplings 1), of the norm per site
kappa and of the leading corner-spectrum ratios sigma_i / sigma_1 (i < 8)
is measured against the float64 result and bounded here.

Reduced precision keeps singular values above 1e-7 sigma_1 (below that the
float32 half-system product is rounding noise) and runs a fixed number of
sweeps: its corner spectra keep changing at the rounding level (~1e-4 per
sweep in fp32, ~1e-3 in bf16), so a 1e-10 convergence test never ends.

References: the oracle's converged environment stored by
tests/golden/make_golden.py (relative cutoff 1e-8) where present, else the
float64 GPU path with the same cutoff (itself checked against the oracle by
the parity tests).

Bounds: energy per spin 1e-4 relative (fp32 and bf16); kappa 1e-7 relative;
spectrum ratios 1e-3 absolute in fp32, 5e-3 in bf16 (where the normalised
spectra fluctuate by ~2e-3 from one sweep to the next).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import models

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BONDS = [(x, y, v) for v in (False, True) for y in range(2) for x in range(2)]
BOUNDS = {"fp32": (1e-4, 1e-7, 1e-3), "bf16": (1e-4, 1e-7, 5e-3)}


def _energy(g):
    bh = models.ruby_bond_h()
    return sum(g.expect(x, y, v, bh(x, y, v)) for (x, y, v) in BONDS) / 12.0


def _converged(D, chi, prec, sweeps, single_layer=False):
    from paper_1711_04798_amd import CTM
    A, B = synth.cell_tensors(0, 8, D, 2)
    if prec == "fp64":
        kw, tol = dict(cutoff=1e-8), 1e-10
    else:
        kw, tol = dict(max_iters=2, resid_tol=0.0, cutoff=1e-7), 0.0
    g = CTM([[A, B]], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi, prec=prec, single_layer=single_layer, **kw)
    sw, dl, ok = g.converge(tol=tol, max_sweeps=sweeps)
    out = dict(sweeps=sw[0], delta=dl[0], E=_energy(g), kappa=g.norm(), spec=g.spectra())
    g.close()
    return out


_REF = {}


def _reference(name, D, chi, max_sweeps):
    if name in _REF:
        return _REF[name]
    p = os.path.join(HERE, "golden", name + ".json")
    if os.path.exists(p):
        gold = json.load(open(p))
        _REF[name] = dict(E=gold["energy_per_spin"], kappa=gold["kappa"], spec=np.array(gold["spectra"]),
                    src="oracle")
        return _REF[name]
    r = _converged(D, chi, "fp64", max_sweeps)
    r["src"] = "gpu-fp64"
    _REF[name] = r
    return r


def _check(name, D, chi, prec, max_sweeps):
    # "fp32-single", "bf16-single": through the single-layer route
    single = prec.endswith("-single")
    prec = prec.split("-")[0]
    ref = _reference(name, D, chi, max_sweeps)
    got = _converged(D, chi, prec, max_sweeps, single)
    e_rel = abs(got["E"] - ref["E"]) / abs(ref["E"])
    k_rel = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    ratio = lambda sp: sp[:, :, :8] / sp[:, :, :1]
    s_err = np.abs(ratio(got["spec"]) - ratio(ref["spec"])).max()
    print("precision %s%s D=%d chi=%d vs %s: sweeps %d delta %.1e  E/spin %.12f (ref %.12f) rel %.2e  "
          "kappa rel %.2e  spectrum ratios %.2e" % (prec, " single-layer" if single else "", D, chi, ref["src"], got["sweeps"], got["delta"], got["E"],
                                           ref["E"], e_rel, k_rel, s_err), flush=True)
    be, bk, bs = BOUNDS[prec]
    assert e_rel < be and k_rel < bk and s_err < bs


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp32-single", "bf16-single"])
def test_precision_ruby_size(gpu, prec):
    """2x2 checkerboard, d=8, D=4, chi=64."""
    print("case precision c1", prec, flush=True)
    _check("c1", 4, 64, prec, 20)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp32-single", "bf16-single"])
def test_precision_benchmark_size(gpu, prec):
    """2x2 checkerboard, d=8, D=6, chi=144 (the benchmark workload)."""
    print("case precision c2", prec, flush=True)
    _check("c2", 6, 144, prec, 12)


FID_BOUND = {"fp32": 1e-6, "bf16": 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_precision_fidelity(gpu, prec):
    """Fidelity per site of two nearby ruby-size checkerboard states (d=8,
    D=4, chi=64; the second set is the first plus 0.1 times seeded noise):
    the reduced-precision runs (fixed sweep count, their spectra fluctuate at
    the rounding level) against the converged float64 run."""
    from paper_1711_04798_amd import binding
    A = synth.cell_tensors(0, 8, 4, 2)
    rng = np.random.default_rng(50)
    B = [a + 0.1 * synth.peps_tensor(rng, 8, 4) for a in A]
    B = [b / np.linalg.norm(b) for b in B]
    kw = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=64)
    print("case precision fidelity", prec, flush=True)
    d64, _, sw64, ok64 = binding.fidelity(A, B, tol=1e-10, max_sweeps=60, cutoff=1e-8, **kw)
    assert ok64, sw64
    dr, _, swr, _ = binding.fidelity(A, B, prec=prec, tol=0.0, max_sweeps=20, max_iters=2, resid_tol=0.0,
                                     cutoff=1e-7, **kw)
    rel = abs(dr - d64) / d64
    print("fidelity per site: float64 %.12f (sweeps %s), %s %.12f, rel err %.2e" % (d64, sw64, prec, dr, rel))
    assert rel < FID_BOUND[prec]
