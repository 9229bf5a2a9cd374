#!/usr/bin/env python3
"""Benchmark of the CTM hot path on one MI355X.

Workload: 2x2 checkerboard iPEPS (tensors A, B with d = 8, D = 6, i.i.d. N(0,1)
from seed 0, unit Frobenius norm), environment dimension chi = 144; bulk
contractions in bf16 (fp32 accumulation) on MFMA, projector SVD in float64.

One step = one CTM sweep (L, R, U, D moves = 8 column steps for a 2x2 cell)
followed by the convergence check (float64 SVD of all 16 corners and the
spectrum change).  The metric is column steps ("moves") per second.

Roofline: the enlarged-corner double-layer contraction (2 chi^2 D^8 flop per
corner, eight corners per launch), timed live with HIP events on the
library's stream over the timed region.  The CPU baseline times the float64
oracle on one plaquette row of one column step of the same workload (half of
a column step for the 2x2 cell) on the host cores.

    python bench.py [--steps K] [--warmup W] [--prec bf16|fp32|fp64] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
WORKLOAD = dict(Lx=2, Ly=2, pattern=[0, 1, 1, 0], d=8, D=6, chi=144, seed=0)


# committed counter summaries, one per live extent of the corner kernel
COUNTERS = os.path.join(ROOT, "profiles", "corner_bf16_2x2_d8_D6_chi144_live%d_hbm_counters.md")
CORNER_SRC = os.path.join(ROOT, "paper_1711_04798_amd", "csrc", "corner_bf16.hip")


def measured_traffic(live_chi):
    """HBM bytes per launch of the bf16 corner kernel from the committed
    counter summary, or None when the kernel source changed since or the
    counters were taken at another live extent."""
    import hashlib
    try:
        sha = hashlib.sha1(open(CORNER_SRC, "rb").read()).hexdigest()
        fields = dict(l.split(":", 1) for l in open(COUNTERS % int(live_chi)).read().splitlines()
                      if l.startswith(("source_sha1:", "hbm_bytes_per_launch:", "live_chi:")))
        if fields.get("source_sha1", "").strip() != sha:
            return None
        if int(fields.get("live_chi", "-1").strip()) != int(live_chi):
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solver_opts(prec):
    if prec == "fp64":
        return dict(oversample=16, max_iters=30, resid_tol=1e-13, cutoff=1e-12)
    # float32 half-system products: singular values below ~1e-7 sigma_1 are
    # rounding noise; warm-started subspace iteration, one plain iteration
    # then one Rayleigh-Ritz step per projector
    return dict(oversample=16, max_iters=2, resid_tol=0.0, cutoff=1e-7)


def solver_status(g):
    """Diagnostic: solver statuses of the last column step's rows."""
    import ctypes
    import numpy as np
    from paper_1711_04798_amd import binding
    lib = binding.load()
    lib.ctm_debug_dump.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_size_t]
    out = []
    for r in range(max(g.Lx, g.Ly)):
        buf = np.zeros(14, dtype=np.int32)
        if lib.ctm_debug_dump(g.ctx, 3, r, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes) == 0:
            f = buf.view(np.float64)
            out.append({"chi_eff": int(buf[0]), "iters": int(buf[2]), "jacobi_sweeps": int(buf[8]),
                        "max_resid": float(f[3]), "discarded": float(f[6])})
    return out


def cpu_baseline(tensors):
    """Oracle (float64, NumPy) on one row of one column step: four enlarged
    corners, dense half-system SVD projectors, absorption of that row."""
    import numpy as np
    from oracle import ctm as octm
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 0) for i in threadpool_info()] or [0])
    except Exception:
        threads = 0
    cores = len(os.sched_getaffinity(0))
    w = WORKLOAD
    cell = octm.Cell(w["Lx"], w["Ly"], w["pattern"], tensors)
    env = octm.init_diag(cell, w["chi"], {(x, y): [np.linspace(1.0, 0.01, w["chi"])] * 4
                                          for y in range(2) for x in range(2)})
    fr = octm._Frame(cell, env, 0)
    t0 = time.perf_counter()
    Qs = octm.plaquette_corners(fr, 0, 0)
    P1, P2 = octm.projectors(*Qs, w["chi"], 1e-12)
    octm.absorb_corner_up(fr.C(0, 0, 0), fr.T(0, 0, 0), P1)
    octm.absorb_edge(fr.T(3, 0, 0), fr.a(0, 0), P1, P2)
    octm.absorb_corner_down(fr.C(3, 0, 0), fr.T(2, 0, 0), P2)
    dt = time.perf_counter() - t0
    # a column step of the 2x2 cell has two rows
    su_rates = su_oracle_rates()
    bd = boundary_oracle_rate()
    return {"value": 1.0 / (2.0 * dt), "unit": "moves/s", "cores": threads or cores,
            "simple_update_steps_per_s_by_D": su_rates,
            "boundary_full_spectrum": bd,
            "kind": "oracle",
            "sample": "one plaquette row (4 enlarged corners, dense float64 half-system "
                      "SVD of n=5184, absorption) of one column step, %.1f s; value = 1/(2 t)"
                      % dt}


def dense_extent_leg(tensors, prec, warm=1, steps=3):
    """The enlarged-corner kernel at the full extent chi = 144 (M = chi^2 =
    20736 rows per corner): the subspace width is pinned at chi + 16 so that
    every contraction runs at the configured chi, as it would for a state
    whose kept rank reaches chi.  Timed like the main leg (HIP events around
    each launch of the kernel)."""
    import ctypes
    import torch
    from paper_1711_04798_amd import CTM, binding
    w = WORKLOAD
    lib = binding.load()
    lib.ctm_debug_set_width.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ctm_debug_set_width.restype = ctypes.c_int
    g = CTM([tensors], Lx=w["Lx"], Ly=w["Ly"], pattern=w["pattern"], chi=w["chi"], prec=prec,
            **solver_opts(prec))
    g.converge(tol=0.0, max_sweeps=2)
    live = ctypes.c_int32()
    assert lib.ctm_debug_set_width(g.ctx, w["chi"] + 16, ctypes.byref(live)) == 0
    for _ in range(warm):
        g.converge(tol=0.0, max_sweeps=1)
    torch.cuda.synchronize()
    g.set_timing(2)
    for _ in range(steps):
        g.converge(tol=0.0, max_sweeps=1)
    torch.cuda.synchronize()
    tm = g.timing()
    g.set_timing(0)
    g.close()
    launches = max(tm["stage3_launches"], 1)
    flop = tm["stage3_flop"] / launches
    avg = tm["stage3_s"] / launches
    ach = flop / avg / 1e12 if avg > 0 else 0.0
    return {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": ach / PEAK_TFLOPS[prec], "live_chi": int(tm["live_chi"]), "flop_per_launch": flop,
            "avg_launch_s": avg, "launches": int(launches),
            "traffic": measured_traffic(int(tm["live_chi"])) if prec == "bf16" else None,
            "note": "enlarged-corner kernel at the full extent (subspace width pinned at chi + 16; "
                    "8 corners of M = chi^2 = 20736 rows, N = K = D^4 = 1296 per launch)"}


SINGLE_LAYER_SHAPES = [(6, 144), (8, 64), (10, 64)]


def single_layer_leg(warm=2, steps=3, precs=("fp32", "bf16")):
    """Double-layer against single-layer contractions of the moves (float32
    contractions, or the bf16 form; float64 solver), 2x2 checkerboard, d = 8,
    at growing D:
    column steps per second over `steps` sweeps after `warm`, and the
    enlarged-corner and absorption phases of one more, instrumented sweep.
    The double layer costs 2 chi^2 D^8 flop per corner, the single-layer
    route 4 chi^2 d D^6 plus its d chi^2 D^4 intermediate through HBM."""
    import torch
    import synth
    from paper_1711_04798_amd import CTM
    out = []
    for prec, (D, chi) in [(p, sh) for p in precs for sh in SINGLE_LAYER_SHAPES]:
        tens = synth.cell_tensors(0, 8, D, 2)
        row = {"D": D, "chi": chi, "prec": prec}
        for route in ("double", "single"):
            log("bench: single-layer leg %s D=%d chi=%d %s" % (prec, D, chi, route))
            g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi, prec=prec,
                    single_layer=(route == "single"), **solver_opts(prec))
            for _ in range(warm):
                g.converge(tol=0.0, max_sweeps=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.converge(tol=0.0, max_sweeps=1)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            g.set_timing(1)
            g.converge(tol=0.0, max_sweeps=1)
            tp = g.timing()
            g.set_timing(0)
            g.close()
            row[route] = {"moves_per_s": 8 * steps / el, "ms_per_sweep": 1e3 * el / steps,
                          "corner_ms_per_sweep": 1e3 * tp["corner_s"], "absorb_ms_per_sweep": 1e3 * tp["absorb_s"],
                          "solver_ms_per_sweep": 1e3 * tp["solver_s"], "live_chi": int(tp["live_chi"])}
        row["speedup_moves"] = row["single"]["moves_per_s"] / row["double"]["moves_per_s"]
        row["speedup_corner"] = row["double"]["corner_ms_per_sweep"] / max(row["single"]["corner_ms_per_sweep"], 1e-9)
        out.append(row)
    return {"rows": out,
            "note": "2x2 checkerboard, d=8, random tensors (seed 0), cutoff 1e-7; contractions at the live extent; "
                    "bf16: the double layer on the bf16 corner kernel, the single-layer products on bf16 MFMA "
                    "(the absorption in float32 on both routes' own paths)"}


SU_FORMS = [dict(n=64, D=2), dict(n=64, D=3), dict(n=1, D=3)]


def su_leg(steps=40):
    """Simple update of ruby-model states (d = 8; couplings J = (s, s, 2 - s)
    over a scan of n points) in lock-step on the GPU: instance Trotter steps
    per second.  The oracle's single-instance rate is measured in the CPU
    baseline leg."""
    import torch
    import synth
    from paper_1711_04798_amd import SimpleUpdate
    from paper_1711_04798_amd.models import ruby_bond_hamiltonians
    rows = []
    for f in SU_FORMS:
        n, D = f["n"], f["D"]
        rng = np.random.default_rng(7)
        tens = [[synth.peps_tensor(rng, 8, D) for _ in range(2)] for _ in range(n)]
        lam = np.full((n, 4, D), 1.0 / np.sqrt(D))
        hs = np.array([ruby_bond_hamiltonians((0.5 + i / n, 0.5 + i / n, 1.5 - i / n)) for i in range(n)])
        log("bench: simple update n=%d D=%d" % (n, D))
        g = SimpleUpdate(tens, lam)
        g.set_gates(hs, 0.01)
        g.evolve(3, 0.0, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.evolve(steps, 0.0, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.close()
        rows.append({"n_inst": n, "d": 8, "D": D, "steps": steps, "ms_per_step": 1e3 * el / steps,
                     "instance_steps_per_s": n * steps / el})
    return {"rows": rows, "note": "ruby model (d = 8), dtau = 0.01, random start; one step = 4 bond updates"}


def su_oracle_rates(steps=5):
    """The oracle's simple update (float64 NumPy, one instance) in steps per
    second, for the bond dimensions of the simple-update leg."""
    import synth
    from oracle import models, su as osu
    out = {}
    for D in sorted({f["D"] for f in SU_FORMS}):
        rng = np.random.default_rng(7)
        T = [synth.peps_tensor(rng, 8, D) for _ in range(2)]
        lam = {b: np.full(D, 1.0 / np.sqrt(D)) for b in osu.BONDS}
        gates = osu.gates_from(models.ruby_bond_h((0.5, 0.5, 1.5)), 0.01)
        t0 = time.perf_counter()
        for _ in range(steps):
            osu.step(T, lam, gates, D)
        out[str(D)] = steps / (time.perf_counter() - t0)
    return out


# boundary density operator: the cylinder of the paper's entropies (D = 8,
# chi = 80, N_v = 6) and a small full-spectrum form the oracle also times
BOUNDARY_FORMS = [dict(D=4, chi=32, nv=4, krylov=256), dict(D=8, chi=80, nv=4, krylov=32),
                  dict(D=8, chi=80, nv=6, krylov=16)]


def boundary_flop(chi, D, Ly, nv, krylov):
    """Float64 flop of one spectrum: 2 krylov ring applications (sigma_R and
    sigma_L^T per basis vector, below the full dimension; the full basis
    adds its block's start vectors, at most 4 more) of nv sites each
    (2 chi^3 D^(nv+1) per site), plus the trace (Ly double transfer matrices,
    2 chi^4 D^2 each, and nv - 1 products of chi^2 x chi^2 matrices)."""
    ring = nv * 2.0 * chi ** 3 * D ** (nv + 1)
    trace = Ly * 2.0 * chi ** 4 * D ** 2 + (nv - 1) * 2.0 * chi ** 6
    return ring, trace


def boundary_leg():
    """Boundary density operator on the cylinder (ctm_boundary_spectrum):
    seconds per spectrum for the leading `krylov` Ritz values (block 4) on a
    CTM environment of the 2x2 cell (d = 8, random tensors, bf16
    single-layer moves, 10 sweeps), and the float64 rate of its ring GEMMs."""
    import torch
    import synth
    from paper_1711_04798_amd import CTM, binding
    rows = []
    env_of = {}
    for f in BOUNDARY_FORMS:
        D, chi, nv, m = f["D"], f["chi"], f["nv"], f["krylov"]
        key = (D, chi)
        if key not in env_of:
            for k in list(env_of):
                env_of.pop(k).close()
            log("bench: boundary leg environment D=%d chi=%d" % (D, chi))
            tens = synth.cell_tensors(3, 8, D, 2)
            g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi, prec="bf16", single_layer=True,
                    **solver_opts("bf16"))
            g.converge(tol=0.0, max_sweeps=10)
            env_of[key] = g
        g = env_of[key]
        log("bench: boundary leg D=%d chi=%d nv=%d krylov=%d" % (D, chi, nv, m))
        row = {"D": D, "chi": chi, "nv": nv, "dim": D ** nv, "krylov": m, "block": 4}
        try:
            g.boundary_spectrum(nv, krylov=1, block=1, nev=1)  # shapes tuned, buffers touched
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, res, S, wt = g.boundary_spectrum(nv, krylov=m, block=4, nev=min(m, 8))
            el = time.perf_counter() - t0
        except binding.CtmError as e:
            row["error"] = str(e)
            rows.append(row)
            continue
        rings = 2 * m if m < D ** nv else 2 * m + 4
        ring, trace = boundary_flop(chi, D, 2, nv, m)
        tf = (rings * ring + trace) / el / 1e12
        row.update({"s_per_spectrum": el, "ring_applications": rings, "ms_per_ring": 1e3 * el / rings,
                    "flop": rings * ring + trace, "tflops": tf, "frac_fp64_peak": tf / PEAK_TFLOPS["fp64"],
                    "leading_p": [float(v) for v in ev[:4]], "max_resid_leading": float(np.max(res[:4])),
                    "captured_weight": wt})
        rows.append(row)
    for g in env_of.values():
        g.close()
    return {"rows": rows,
            "note": "2x2 checkerboard, d = 8, random tensors (seed 3), environment from 10 bf16 single-layer "
                    "sweeps; all boundary arithmetic float64; the rate counts the ring GEMMs and the trace "
                    "over the whole call (syncs and Gram-Schmidt included)"}


def boundary_oracle_rate():
    """The oracle's boundary spectrum (dense sigma_L, sigma_R and eigenvalues,
    float64 NumPy) for the small full-spectrum form, on its own trivially
    initialised environment of that shape (the cost does not depend on the
    values)."""
    import synth
    from oracle import ctm as octm, boundary as obd
    f = BOUNDARY_FORMS[0]
    tens = synth.cell_tensors(3, 8, f["D"], 2)
    cell = octm.Cell(2, 2, [0, 1, 1, 0], tens)
    env = octm.init_trivial(cell, f["chi"])
    t0 = time.perf_counter()
    obd.boundary_spectrum(cell, env, 0, f["nv"])
    return {"D": f["D"], "chi": f["chi"], "nv": f["nv"], "s_per_spectrum": time.perf_counter() - t0}


def complex_leg(steps=5, warm=2):
    """Complex kets (i.i.d. complex normal tensors, the benchmark's shapes)
    against real ones: column steps per second of the benchmark workload in
    bf16.  The complex state runs on the real form of the double layer, so
    the two should cost the same."""
    import torch
    from paper_1711_04798_amd import CTM
    w = WORKLOAD
    rng = np.random.default_rng(5)
    out = {}
    for kind in ("real", "complex"):
        tens = []
        for _ in range(2):
            A = rng.standard_normal((w["d"], w["D"], w["D"], w["D"], w["D"]))
            if kind == "complex":
                A = A + 1j * rng.standard_normal(A.shape)
            tens.append(A / np.linalg.norm(A))
        log("bench: complex leg %s" % kind)
        g = CTM([tens], Lx=w["Lx"], Ly=w["Ly"], pattern=w["pattern"], chi=w["chi"], prec="bf16",
                **solver_opts("bf16"))
        for _ in range(warm):
            g.converge(tol=0.0, max_sweeps=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.converge(tol=0.0, max_sweeps=1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[kind] = {"moves_per_s": 8 * steps / el, "ms_per_sweep": 1e3 * el / steps}
        g.close()
    out["ratio"] = out["complex"]["moves_per_s"] / out["real"]["moves_per_s"]
    out["note"] = "2x2 d=8 D=6 chi=144 bf16, random tensors (seed 5), complex kets on the real form of the double layer"
    return out


BATCHED = dict(n_inst=256, d=8, Ds=(3, 4, 5), chis=(32, 64, 100), seed=0, max_sweeps=60)
# float64 contractions reach Delta < 1e-6; float32 contractions do not (their
# corner spectra keep changing by ~1e-5 .. 1e-4 per sweep), so the float32
# form is run to 1e-4
BATCHED_FORMS = [dict(prec="fp64", max_iters=3, tol=1e-6, plain_per_class=2, concurrent=True),
                 dict(prec="fp64", max_iters=3, tol=1e-6, plain_per_class=0, concurrent=False),
                 dict(prec="fp32", max_iters=2, tol=1e-4, plain_per_class=1, concurrent=True)]


def batched_leg(form):
    """Batched form: 256 independent 1x1 instances, (D, chi) drawn per instance,
    float32 contractions, one captured HIP graph per sweep, converged to tol;
    against plain runs (one context per instance, eager) of a stratified
    sample: the first `plain_per_class` instances of every (D, chi) class.
    Rates count converged instances only; the plain rate is the sample's
    converged count over its time, weighted to the batch's class mix."""
    import torch
    import synth
    from paper_1711_04798_amd import CTM
    b = dict(BATCHED)
    b.update(form)
    inst = synth.batched_instances(b["seed"], b["n_inst"], d=b["d"], Ds=b["Ds"], chis=b["chis"])
    kw = dict(prec=b["prec"], max_iters=b["max_iters"], resid_tol=0.0,
              cutoff=1e-8 if b["prec"] == "fp64" else 1e-6)
    log("bench: batched leg, %d instances, %s, tol %g, concurrent class branches %s"
        % (len(inst), b["prec"], b["tol"], b["concurrent"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = CTM([[A] for _, _, A in inst], chi=[c for _, c, _ in inst], use_graph=True,
            concurrent_classes=b["concurrent"], **kw)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    sw, dl, ok = g.converge(tol=b["tol"], max_sweeps=b["max_sweeps"])
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    g.close()
    del g
    torch.cuda.empty_cache()
    conv = [d < b["tol"] for d in dl]
    n_conv = sum(conv)
    log("bench: batched converge %.2f s (init %.2f s), %d/%d converged, sweeps max %d"
        % (t_b, t_init, n_conv, len(inst), max(sw)))
    if not b["plain_per_class"]:
        return {"envs_per_s": n_conv / t_b, "converged": n_conv, "n_inst": len(inst), "tol": b["tol"],
                "time_s": t_b, "sweeps_mean": float(np.mean(sw)), "dtype": b["prec"],
                "concurrent_class_branches": b["concurrent"],
                "unit": "converged environments/s (converged instances only)"}
    # plain: stratified sample, per class time per instance
    classes = sorted({(D, c) for D, c, _ in inst})
    per_class = {}
    for cls in classes:
        members = [A for D, c, A in inst if (D, c) == cls][:b["plain_per_class"]]
        t_c, n_c, sws = 0.0, 0, []
        for A in members:
            p = CTM([[A]], chi=cls[1], **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1, d1, _ = p.converge(tol=b["tol"], max_sweeps=b["max_sweeps"])
            torch.cuda.synchronize()
            t_c += time.perf_counter() - t0
            n_c += int(d1[0] < b["tol"])
            sws.append(s1[0])
            p.close()
        per_class[cls] = (t_c / len(members), n_c / len(members), float(np.mean(sws)))
    # the plain method on the batch's instance mix: expected time and
    # converged count from the per-class sample
    mix = {cls: sum(1 for D, c, _ in inst if (D, c) == cls) for cls in classes}
    t_plain = sum(mix[c] * per_class[c][0] for c in classes)
    n_plain = sum(mix[c] * per_class[c][1] for c in classes)
    env_b = n_conv / t_b
    env_p = n_plain / t_plain if t_plain > 0 else 0.0
    log("bench: plain sample (%d per class) extrapolated to the batch: %.2f s, %.1f converged"
        % (b["plain_per_class"], t_plain, n_plain))
    return {"envs_per_s": env_b, "plain_envs_per_s": env_p, "speedup": env_b / env_p if env_p > 0 else None,
            "unit": "converged environments/s (converged instances only)", "n_inst": len(inst),
            "converged": n_conv, "tol": b["tol"], "max_sweeps": b["max_sweeps"],
            "delta_median": float(np.median(dl)), "time_s": t_b,
            "sweeps_mean": float(np.mean(sw)), "sweeps_max": int(max(sw)),
            "plain_sample": "%d per (D, chi) class, %d instances" % (b["plain_per_class"],
                                                                     b["plain_per_class"] * len(classes)),
            "plain_sweeps_mean_by_class": {"D%d_chi%d" % c: per_class[c][2] for c in classes},
            "plain_converged_frac_by_class": {"D%d_chi%d" % c: per_class[c][1] for c in classes},
            "dtype": b["prec"], "concurrent_class_branches": b["concurrent"],
            "workload": "256 1x1 iPEPS, d=8, D in {3,4,5}, chi in {32,64,100} per instance (seed 0), "
                        "%s contractions, one HIP graph per sweep of every live instance; plain = one "
                        % b["prec"] +
                        "context per instance, eager, time per class from a stratified sample applied "
                        "to the batch's class counts"}


WARM = dict(d=8, D=4, chi=64, family_seed=0, train_seed=1, test_seed=2, n_train=2000, n_test=200, tol=1e-10,
            max_sweeps=60, hidden=128, steps=4000, lr=2e-3)


def warm_leg():
    """Learned warm start: plain runs from the trivial start converge the
    training members of the family A(theta) (their spectra are the targets);
    the network trains on the device; held-out members then start from the
    predicted spectra, in two readings: (a) diagonal corners (CTM_INIT_DIAG),
    falling back to the trivial start after a budget of twice the plain
    sweeps; (b) a trivial run whose corners get the spectra after its first
    sweep (ctm_set_corner_spectra).  The exact converged spectra in place of
    the prediction bound what any predictor could gain."""
    import torch
    import synth
    from paper_1711_04798_amd import warmstart as ws
    w = WARM
    base = synth.warm_family(w["family_seed"], d=w["d"], D=w["D"])
    th_tr, th_te = synth.warm_thetas(w["train_seed"], w["n_train"]), synth.warm_thetas(w["test_seed"], w["n_test"])
    T_tr = [synth.warm_member(base, t) for t in th_tr]
    T_te = [synth.warm_member(base, t) for t in th_te]
    log("bench: warm-start leg, %d training runs" % len(T_tr))
    t0 = time.perf_counter()
    s_tr, sw_tr, d_tr, _ = ws.converge_batch(T_tr, w["chi"], w["tol"], w["max_sweeps"])
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, hist = ws.train(th_tr, s_tr, hidden=w["hidden"], steps=w["steps"], lr=w["lr"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pred = ws.predict(net, th_te)
    t0 = time.perf_counter()
    s_tv, sw_tv, d_tv, k_tv = ws.converge_batch(T_te, w["chi"], w["tol"], w["max_sweeps"])
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    s_w, sw_w, ok_w, k_w = ws.converge_with_fallback(T_te, w["chi"], w["tol"], w["max_sweeps"], pred,
                                                      warm_budget=2 * int(sw_tv.max()))
    t_warm = time.perf_counter() - t0
    log("bench: warm-start leg, injected spectra")
    t0 = time.perf_counter()
    s_i, sw_i, d_i, k_i = ws.converge_injected(T_te, w["chi"], w["tol"], w["max_sweeps"], pred)
    t_inj = time.perf_counter() - t0
    s_x, sw_x, d_x, k_x = ws.converge_injected(T_te, w["chi"], w["tol"], w["max_sweeps"], s_tv)
    _, sw_xd, d_xd, _ = ws.converge_batch(T_te, w["chi"], w["tol"], 2 * int(sw_tv.max()), spectra=s_tv)
    lg = lambda a: np.log10(np.maximum(a, ws.TARGET_FLOOR))
    mean_pred = lg(s_tr).mean(axis=0)[None]
    conv = lambda d: int(np.sum(np.asarray(d) < w["tol"]))
    return {"plain_sweeps_mean": float(sw_tv.mean()),
            "mlp_diag_sweeps_mean_with_fallback": float(sw_w.mean()), "mlp_diag_converged": int(ok_w.sum()),
            "mlp_injected_sweeps_mean": float(sw_i.mean()), "mlp_injected_converged": conv(d_i),
            "exact_injected_sweeps_mean": float(sw_x.mean()), "exact_injected_converged": conv(d_x),
            "exact_diag_converged": conv(d_xd), "exact_diag_budget": 2 * int(sw_tv.max()),
            "n_test": len(T_te), "plain_envs_per_s": len(T_te) / t_plain,
            "mlp_diag_envs_per_s": len(T_te) / t_warm, "mlp_injected_envs_per_s": conv(d_i) / t_inj,
            "n_train": len(T_tr), "train_data_s": t_data, "train_converged": conv(d_tr),
            "train_s": t_train, "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "pred_log10_err_top8": float(np.abs(lg(pred) - lg(s_tv))[:, :, :8].mean()),
            "mean_predictor_log10_err_top8": float(np.abs(mean_pred - lg(s_tv))[:, :, :8].mean()),
            "kappa_max_rel_diff_mlp_diag": float(np.max(np.abs(k_w - k_tv) / np.abs(k_tv))),
            "kappa_max_rel_diff_mlp_injected": float(np.max(np.abs(k_i - k_tv) / np.abs(k_tv))),
            "tol": w["tol"],
            "workload": "family A(theta) d=8 D=4 chi=64 1x1, float64 contractions, %d training runs, "
                        "%d held-out" % (len(T_tr), len(T_te))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-full", action="store_true", help="skip the full-extent corner-kernel leg")
    ap.add_argument("--full-extent-only", action="store_true",
                    help="only the corner kernel at the full extent (for profiling runs)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-layer comparison leg")
    ap.add_argument("--single-only", action="store_true", help="only the single-layer comparison leg")
    ap.add_argument("--no-su", action="store_true", help="skip the simple-update leg")
    ap.add_argument("--su-only", action="store_true", help="only the simple-update leg")
    ap.add_argument("--no-boundary", action="store_true", help="skip the boundary-operator leg")
    ap.add_argument("--no-complex", action="store_true", help="skip the complex-tensor leg")
    ap.add_argument("--boundary-only", action="store_true", help="only the boundary-operator leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the CTM hot path here is a single-GPU "
              "build (multi-GPU sharding is described in the design notes, not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1711_04798_amd import CTM

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 5}))
        return

    w = WORKLOAD
    tensors = synth.cell_tensors(w["seed"], w["d"], w["D"], 2)
    if args.single_only:
        print(json.dumps({"single_layer": single_layer_leg()}), flush=True)
        return
    if args.su_only:
        print(json.dumps({"simple_update": su_leg()}), flush=True)
        return
    if args.boundary_only:
        print(json.dumps({"boundary": boundary_leg()}), flush=True)
        return
    if args.full_extent_only:
        print(json.dumps({"roofline_full_extent": dense_extent_leg(tensors, args.prec)}), flush=True)
        return
    log("bench: init chi=%d D=%d prec=%s" % (w["chi"], w["D"], args.prec))
    g = CTM([tensors], Lx=w["Lx"], Ly=w["Ly"], pattern=w["pattern"], chi=w["chi"],
            prec=args.prec, **solver_opts(args.prec))
    moves_per_sweep = 2 * w["Lx"] + 2 * w["Ly"]
    for i in range(args.warmup):
        t = time.perf_counter()
        g.converge(tol=0.0, max_sweeps=1)
        torch.cuda.synchronize()
        log("bench: warmup sweep %d %.2f s" % (i, time.perf_counter() - t))
    torch.cuda.synchronize()
    # the timed region records only the events around the enlarged-corner
    # kernel (for the roofline); the phase breakdown comes from two more,
    # fully instrumented steps afterwards
    g.set_timing(2)
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, delta, _ = g.converge(tol=0.0, max_sweeps=1)
        log("bench: step %d delta %.3e elapsed %.2f s" % (i, delta[0], time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = g.timing()
    g.set_timing(1)
    phase_steps = 2
    for i in range(phase_steps):
        g.converge(tol=0.0, max_sweeps=1)
    tp = g.timing()
    g.set_timing(0)
    status = solver_status(g)
    log("bench: solver status of the last column step: %s" % status)
    g.close()

    moves = moves_per_sweep * args.steps
    value = moves / elapsed
    launches = max(tm["stage3_launches"], 1)
    flop_per_launch = tm["stage3_flop"] / launches
    flop_nominal = tm["stage3_flop_nominal"] / launches
    avg = tm["stage3_s"] / launches
    achieved = flop_per_launch / avg / 1e12 if avg > 0 else 0.0
    peak = PEAK_TFLOPS[args.prec]
    live_chi = int(tm["live_chi"])
    out = {
        "metric": "CTM moves/s + MFMA util at D=6 χ=144; converged envs/s batched vs plain",
        "value": value,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "2x2 checkerboard iPEPS d=8 D=6 chi=144, %s contractions, "
                               "float64 projector SVD; step = 1 sweep (8 moves) + convergence check; "
                               "contractions at the live extent (chi_live = %d: every index beyond "
                               "is an exact zero)" % (args.prec, live_chi),
                   "Lx": 2, "Ly": 2, "d": 8, "D": 6, "chi": 144, "seed": 0,
                   "chi_eff": max([r["chi_eff"] for r in status] or [0]),
                   "cutoff": solver_opts(args.prec)["cutoff"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(live_chi) if args.prec == "bf16" else None,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "enlarged-corner double-layer contraction (%s, 8 corners "
                               "per launch, 2 chi_live^2 D^8 flop each)"
                               % ("corner_bf16_dma_kernel" if args.prec == "bf16" else "gemm_kernel"),
                     "live_chi": live_chi,
                     "flop_per_launch": flop_per_launch, "avg_launch_s": avg,
                     "launches": int(launches),
                     "nominal": {"note": "the same launches counted at chi = %d (2 chi^2 D^8 per corner): "
                                         "work on indices that are exact zeros and are not computed"
                                         % w["chi"],
                                 "flop_per_launch": flop_nominal,
                                 "achieved": flop_nominal / avg / 1e12 if avg > 0 else 0.0,
                                 "frac": (flop_nominal / avg / 1e12 if avg > 0 else 0.0) / peak}},
        "phase_ms_per_step": {"corner": 1e3 * tp["corner_s"] / phase_steps,
                              "solver": 1e3 * tp["solver_s"] / phase_steps,
                              "absorb": 1e3 * tp["absorb_s"] / phase_steps,
                              "note": "from %d instrumented steps after the timed region" % phase_steps},
    }
    if not args.no_full:
        log("bench: enlarged-corner kernel at the full extent")
        out["roofline_full_extent"] = dense_extent_leg(tensors, args.prec)
    if not args.no_single:
        out["single_layer"] = single_layer_leg()
    if not args.no_su:
        out["simple_update"] = su_leg()
    if not args.no_boundary:
        out["boundary"] = boundary_leg()
    if not args.no_complex:
        out["complex"] = complex_leg()
    if not args.no_batched:
        out["batched"] = batched_leg(BATCHED_FORMS[0])
        out["batched"]["sequential_class_branches"] = batched_leg(BATCHED_FORMS[1])
        out["batched_fp32"] = batched_leg(BATCHED_FORMS[2])
    if not args.no_warm:
        out["warm_start"] = warm_leg()
    if not args.no_cpu:
        log("bench: cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(tensors)
        if "simple_update" in out:
            rates = out["cpu_baseline"]["simple_update_steps_per_s_by_D"]
            for r in out["simple_update"]["rows"]:
                r["speedup_vs_oracle"] = r["instance_steps_per_s"] / rates[str(r["D"])]
        if "boundary" in out:
            bd = out["cpu_baseline"]["boundary_full_spectrum"]
            for r in out["boundary"]["rows"]:
                if (r["D"], r["chi"], r["nv"]) == (bd["D"], bd["chi"], bd["nv"]) and "s_per_spectrum" in r:
                    r["speedup_vs_oracle"] = bd["s_per_spectrum"] / r["s_per_spectrum"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
