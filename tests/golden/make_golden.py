"""Writes the stored expected values of the converged-environment tests.

Calls only the float64 CPU oracle and the seeded input generators.  For each
workload it runs the oracle's CTM from the trivial start until the corner
spectra change by less than `tol` per sweep (or `max_sweeps`), then records the
sweep history, the corner spectra, the norm per site and the ruby-model bond
energies (all couplings 1, block-site terms of App. A) into <name>.json.

    python tests/golden/make_golden.py c1        # 2x2, d=8, D=4, chi=64
    python tests/golden/make_golden.py c2        # 2x2, d=8, D=6, chi=144 (hours)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ctm as octm, obs as oobs, models  # noqa: E402

# The relative cutoff of the kept singular values is 1e-8: with 1e-12 the
# kept set reaches directions whose singular vectors float64 fixes only to
# ~1e-4, and the corner spectra then keep changing by ~2e-8 per sweep forever.
WORKLOADS = {
    "c1": dict(d=8, D=4, chi=64, seed=0, tol=1e-10, max_sweeps=40, cutoff=1e-8),
    "c2": dict(d=8, D=6, chi=144, seed=0, tol=1e-8, max_sweeps=14, cutoff=1e-8),
}


def run(name):
    w = WORKLOADS[name]
    A, B = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], [A, B])
    env = octm.init_trivial(cell, w["chi"])
    s_old = octm.corner_spectra(env)
    hist = []
    t0 = time.time()
    converged = False
    for it in range(1, w["max_sweeps"] + 1):
        octm.sweep(cell, env, w["cutoff"])
        s_new = octm.corner_spectra(env)
        delta = octm.spectra_delta(s_new, s_old)
        s_old = s_new
        hist.append(float(delta))
        print("%s sweep %d delta %.3e (%.0f s)" % (name, it, delta, time.time() - t0), flush=True)
        if delta < w["tol"]:
            converged = True
            break
    kap = oobs.kappa(cell, env)
    e_cell, e_bonds = oobs.energy(cell, env, models.ruby_bond_h())
    spec = np.array([[np.asarray(v) for v in s_old[(x, y)]] for y in range(2) for x in range(2)])
    out = dict(workload=dict(w, Lx=2, Ly=2, pattern=[0, 1, 1, 0], init="trivial"),
               sweeps=len(hist), converged=converged, delta_history=hist,
               kappa=float(np.real(kap)), energy_cell=e_cell, energy_bonds=e_bonds,
               energy_per_spin=e_cell / 12.0,
               spectra_layout="[position y*Lx+x][corner C1..C4][chi]",
               spectra=spec.tolist())
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", name, "kappa", out["kappa"], "E/spin", out["energy_per_spin"], flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c1"]:
        run(n)
