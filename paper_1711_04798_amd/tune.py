"""Launch-variant tuner: runs the benchmark workloads once with tile-table
tuning on (every new shape of the split products times its variants on its
own operands; the generic GEMM times its tiles) and writes the table, which
the binding loads with the library.

    python -m paper_1711_04798_amd.tune [--out PATH]

Run it on the MI355X the table is for; commit the file it writes next to
this module (tiles.json).
"""
import argparse
import ctypes
import os
import sys
import time

import numpy as np


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(here, "tiles.json"))
    args = ap.parse_args()
    import torch
    import synth
    from paper_1711_04798_amd import binding
    from paper_1711_04798_amd.binding import CTM
    lib = binding.load(tile_table=False)
    lib.ctm_tile_table_clear()
    lib.ctm_tile_table_tune(1)
    t0 = time.time()
    # the benchmark workload: the first sweeps run at the full extent, the
    # later ones at the live extent the convergence check sets
    tens = synth.cell_tensors(0, 8, 6, 2)
    for prec in ("bf16", "fp32"):
        g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=144, prec=prec, max_iters=2, resid_tol=0.0,
                cutoff=1e-7)
        for _ in range(4):
            g.converge(tol=0.0, max_sweeps=1)
        g.close()
        _log("tune: benchmark workload %s done (%.0f s)" % (prec, time.time() - t0))
    # float64 ruby-size and benchmark-size convergence
    for D, chi in ((4, 64), (6, 144)):
        g = CTM([synth.cell_tensors(0, 8, D, 2)], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi, cutoff=1e-8)
        g.converge(tol=1e-10, max_sweeps=3)
        g.close()
        _log("tune: float64 D=%d chi=%d done (%.0f s)" % (D, chi, time.time() - t0))
    # batched forms (grouped launches of every class) and the warm-start runs
    inst = synth.batched_instances(0, 256, d=8)
    for prec, it, cut in (("fp64", 3, 1e-8), ("fp32", 2, 1e-6)):
        g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst], prec=prec, max_iters=it, resid_tol=0.0,
                cutoff=cut, use_graph=True)
        g.converge(tol=0.0, max_sweeps=3)
        g.close()
        _log("tune: batched %s done (%.0f s)" % (prec, time.time() - t0))
    torch.cuda.synchronize()
    n = ctypes.c_int32()
    binding._check(lib.ctm_tile_table_save(args.out.encode(), ctypes.byref(n)))
    lib.ctm_tile_table_tune(0)
    print("tile table: %d entries -> %s (%.0f s)" % (n.value, args.out, time.time() - t0))


if __name__ == "__main__":
    main()
