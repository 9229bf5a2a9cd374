"""CPU checks of the C ABI library: it loads, exports every function declared
in include/*.h, calls the HIP runtime from its wrappers, and its whole host
orchestration passes the host-side bounds checks in dry-run mode (no GPU:
every launch and copy is checked against the workspace allocations and then
skipped)."""
import ctypes
import json
import glob
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1711_04798_amd", "libctm.so")


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_1711_04798_amd import build
        build.build()
    return LIB


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ctm_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol(lib_path):
    names = declared()
    assert {"ctm_init", "ctm_move", "ctm_converge", "ctm_rdm", "ctm_fidelity"} <= names
    assert {"ctm_checkpoint_save", "ctm_checkpoint_load", "ctm_checkpoint_bytes"} <= names
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_wrappers_call_the_runtime(lib_path):
    """The copy / memset / synchronise wrappers must reach the HIP runtime
    (a wrapper that called itself once spun forever on the host)."""
    out = subprocess.run(["nm", "-D", lib_path], capture_output=True, text=True).stdout
    undef = {l.split()[-1].split("@")[0] for l in out.splitlines() if " U " in l}
    for sym in ("hipMemcpyAsync", "hipMemsetAsync", "hipStreamSynchronize", "hipLaunchKernel"):
        assert sym in undef, sym


DRY = r'''
import ctypes, json, os, sys, tempfile
sys.path.insert(0, %(root)r)
from paper_1711_04798_amd import binding as b
lib = b.load(%(lib)r)
out = {}
for case in %(cases)r:
    name, Lx, Ly, pat, nt, d, D, chi, prec = case[:9]
    extra = dict(case[9]) if len(case) > 9 else {}
    bnv = extra.pop("boundary_nv", None)
    cfg, keep = b.make_config(Lx, Ly, pat, nt, d, D, chi, prec, max_iters=2, **extra)
    n = b.workspace_size(cfg)
    ptrs = (ctypes.c_void_p * (nt * len(d)))(*[(1 << 30) + 4096 * i for i in range(nt * len(d))])
    ctx = ctypes.c_void_p()
    st = [lib.ctm_init(ctypes.byref(cfg), ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), None,
                       ctypes.c_void_p(1 << 40), n, None, 0, None, ctypes.byref(ctx))]
    st.append(lib.ctm_move(ctx, 4, 1))
    for dr in range(4):
        st.append(lib.ctm_move(ctx, dr, 3))
    sw = (ctypes.c_int32 * len(d))(); dl = (ctypes.c_double * len(d))()
    mf = tempfile.mktemp(suffix=".jsonl")
    st.append(lib.ctm_set_metrics(ctx, mf.encode(), 1))
    st.append(lib.ctm_converge(ctx, 1e-10, 2, 1, sw, dl))
    st.append(lib.ctm_set_metrics(ctx, None, 0))
    # the dry run reads back zeros: every instance stops at the first check
    ml = [json.loads(l) for l in open(mf)]
    os.remove(mf)
    st.append(0 if len(ml) == len(d) and all(set(m["chi_eff"]) == set("LRUD") for m in ml) else 99)
    k = ctypes.c_double()
    # narrowed subspace: every stage at the live extent, under the bounds checks
    live = ctypes.c_int32()
    st.append(lib.ctm_debug_set_width(ctx, 9, ctypes.byref(live)))
    st.append(lib.ctm_move(ctx, 4, 1))
    for dr in range(4):
        st.append(lib.ctm_move(ctx, dr, 1))
    nb = lib.ctm_checkpoint_bytes(ctx, 0)
    ck = (ctypes.c_char * nb)()
    st.append(lib.ctm_checkpoint_save(ctx, 0, ck, nb))
    st.append(lib.ctm_checkpoint_load(ctx, 0, ck, nb))
    eb = lib.ctm_env_bytes(ctx, 0)
    eh = (ctypes.c_char * eb)()
    st.append(lib.ctm_env_export(ctx, 0, eh, eb))
    st.append(lib.ctm_env_import(ctx, 0, eh, eb))
    cx = extra.get("complex_tensors", False)
    if not cx and (bnv or (Ly in (1, 2) and D[0] <= 4)):
        nv = bnv or 2 * Ly
        kry = min(D[0] ** nv, 12)
        wsb = ctypes.c_size_t()
        st.append(lib.ctm_boundary_workspace_size(ctx, 0, nv, kry, ctypes.byref(wsb)))
        ev = (ctypes.c_double * kry)(); rs = (ctypes.c_double * kry)()
        ent = ctypes.c_double(); wt = ctypes.c_double()
        st.append(lib.ctm_boundary_spectrum(ctx, 0, 0, nv, kry, min(2, kry), 3, ctypes.c_void_p(1 << 44), wsb.value,
                                            kry, ev, rs, ctypes.byref(ent), ctypes.byref(wt)))
    if True:
        st.append(lib.ctm_norm(ctx, 0, ctypes.byref(k)))
        rho = (ctypes.c_double * (2 * d[0] ** 4))(); h = ctypes.c_double()
        for v in (0, 1):
            st.append((lib.ctm_rdm_complex if cx else lib.ctm_rdm)(ctx, 0, 1, 0, v, rho, ctypes.byref(h)))
    spec = (ctypes.c_double * (Lx * Ly * 4 * chi[0]))()
    st.append(lib.ctm_spectra(ctx, 0, spec))
    out[name] = [st, lib.ctm_last_error().decode(), n]
    lib.ctm_destroy(ctx)
print(json.dumps(out))
'''

CASES = [
    ("c0", 1, 1, [0], 1, [2], [2], [16], "fp64"),
    ("c1", 2, 2, [0, 1, 1, 0], 2, [8], [4], [64], "fp64"),
    ("c2_bf16", 2, 2, [0, 1, 1, 0], 2, [8], [6], [144], "bf16"),
    ("c2_fp32", 2, 2, [0, 1, 1, 0], 2, [8], [6], [144], "fp32"),
    ("mixed_1x1", 1, 1, [0], 1, [8, 8, 8], [3, 5, 4], [32, 100, 64], "fp32"),
    ("tiny_chi", 1, 1, [0], 1, [2], [3], [1], "fp64"),
    ("rect_2x1", 2, 1, [0, 1], 2, [2], [2], [8], "fp64"),
    # batched form: classes of equal (d, D, chi) moved in lock-step
    ("batched", 1, 1, [0], 1, [8] * 40, [3, 4, 5, 3] * 10, [32, 64, 100, 32] * 10, "fp32"),
    # single-layer contractions (no double layer in the moves)
    ("c1_single", 2, 2, [0, 1, 1, 0], 2, [8], [4], [64], "fp64", {"single_layer": True}),
    ("c2_single", 2, 2, [0, 1, 1, 0], 2, [8], [6], [144], "fp32", {"single_layer": True}),
    ("c2_single_bf16", 2, 2, [0, 1, 1, 0], 2, [8], [6], [144], "bf16", {"single_layer": True}),
    ("large_D_single", 2, 2, [0, 1, 1, 0], 2, [8], [12], [100], "fp32", {"single_layer": True}),
    ("batched_single", 1, 1, [0], 1, [8] * 6, [3, 4, 5] * 2, [32, 64, 100] * 2, "fp32",
     {"single_layer": True, "use_graph": True}),
    # the cylinder of Sec. V's entropies: D = 8, chi = 80, N_v = 6 (ring
    # state of 1.7e9 doubles, its GEMMs in several launches)
    ("boundary_D8", 2, 2, [0, 1, 1, 0], 2, [8], [8], [80], "bf16", {"single_layer": True, "boundary_nv": 6}),
    # complex kets on the real form of the double layer
    ("complex_fp64", 2, 2, [0, 1, 1, 0], 2, [2], [3], [24], "fp64", {"complex_tensors": True}),
    ("complex_bf16", 2, 2, [0, 1, 1, 0], 2, [8], [6], [144], "bf16", {"complex_tensors": True}),
]


def test_dry_run_orchestration(lib_path):
    import json
    code = DRY % {"root": ROOT, "cases": CASES, "lib": lib_path}
    env = dict(os.environ, CTM_DRY_RUN="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr
    res = json.loads(r.stdout.strip().splitlines()[-1])
    for name, (st, err, nbytes) in res.items():
        assert all(s == 0 for s in st), (name, st, err)
    # the c2 workspace fits comfortably in one MI355X's HBM
    assert res["c2_bf16"][2] < 16e9


def test_complex_rejections(lib_path):
    """Complex kets: not with the single-layer route, not for the fidelity
    (the mixed network has no real form), not for the boundary operator."""
    from paper_1711_04798_amd import binding as b
    lib = b.load()
    cfg, keep = b.make_config(1, 1, [0], 1, [2], [2], [8], complex_tensors=True, single_layer=True)
    with pytest.raises(b.CtmError) as e:
        b.workspace_size(cfg)
    assert e.value.status == b.CTM_E_INVALID
    cfg, keep = b.make_config(1, 1, [0], 1, [2], [2], [8], complex_tensors=True)
    assert b.workspace_size(cfg) > 0
    dv, lv = ctypes.c_double(), ctypes.c_double()
    sw = (ctypes.c_int32 * 3)()
    ptrs = (ctypes.c_void_p * 1)(1 << 30)
    pp = ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p))
    st = lib.ctm_fidelity(ctypes.byref(cfg), pp, pp, None, 0, None, 1e-8, 10, ctypes.byref(dv), ctypes.byref(lv), sw)
    assert st == b.CTM_E_INVALID and b"real tensors" in lib.ctm_last_error()
    with pytest.raises(ValueError):
        b.fidelity([np.zeros((2, 2, 2, 2, 2), dtype=complex)], [np.zeros((2, 2, 2, 2, 2))])


def test_invalid_configs_rejected(lib_path):
    from paper_1711_04798_amd import binding as b
    b.load()
    for bad in [dict(chi=[0]), dict(D=[0]), dict(chi=[200])]:
        kw = dict(d=[2], D=[2], chi=[4])
        kw.update(bad)
        cfg, keep = b.make_config(1, 1, [0], 1, kw["d"], kw["D"], kw["chi"])
        with pytest.raises(b.CtmError) as e:
            b.workspace_size(cfg)
        assert e.value.status == b.CTM_E_INVALID


def test_tile_table_roundtrip(lib_path, tmp_path):
    """The launch-variant table written by save reads back entry for entry;
    a malformed entry is rejected."""
    code = r'''
import ctypes, json, sys
sys.path.insert(0, %(root)r)
from paper_1711_04798_amd import binding as b
lib = b.load(tile_table=False)
lib.ctm_tile_table_clear()
src, dst, bad = sys.argv[1], sys.argv[2], sys.argv[3]
n = ctypes.c_int32()
assert lib.ctm_tile_table_load(src.encode(), ctypes.byref(n)) == 0 and n.value == 4
assert lib.ctm_tile_table_save(dst.encode(), ctypes.byref(n)) == 0 and n.value == 4
print(lib.ctm_tile_table_load(bad.encode(), ctypes.byref(n)))
''' % {"root": ROOT}
    entries = [
        {"kernel": "ts", "ta": 1, "tc": 0, "ak": 1, "bk": 1, "groups": 2, "M": 1728, "N": 48, "K": 1728, "variant": 1},
        {"kernel": "gemm", "ta": 0, "tc": 0, "ak": 1, "bk": 0, "groups": 0, "M": 48, "N": 1728, "K": 48, "variant": 3},
        {"kernel": "splitk", "ta": 0, "tc": 0, "ak": 0, "bk": 1, "groups": 2, "M": 48, "N": 48, "K": 1728,
         "variant": 0},
        {"kernel": "corner", "ta": 2, "tc": 1, "ak": 1, "bk": 1, "groups": 8, "M": 2304, "N": 1296, "K": 1296,
         "variant": 2},
    ]
    src, dst, bad = tmp_path / "a.json", tmp_path / "b.json", tmp_path / "c.json"
    src.write_text("[\n" + ",\n".join(json.dumps(e) for e in entries) + "\n]\n")
    bad.write_text('[\n{"kernel": "ts", "ta": 1, "variant": 9}\n]\n')
    r = subprocess.run([sys.executable, "-c", code, str(src), str(dst), str(bad)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"  # CTM_E_INVALID
    key = lambda e: (e["kernel"], e["ta"], e["tc"], e["ak"], e["bk"], e["groups"], e["M"], e["N"], e["K"])
    got = json.loads(dst.read_text())
    assert sorted((key(e), e["variant"]) for e in got) == sorted((key(e), e["variant"]) for e in entries)


DRY_SU = r'''
import ctypes, json, sys
sys.path.insert(0, %(root)r)
from paper_1711_04798_amd import binding as b
lib = b.load(%(lib)r, tile_table=False)
out = []
for n, d, D in ((1, 2, 3), (3, 8, 2), (40, 2, 4), (2, 8, 3), (2, 8, 5)):
    nb = ctypes.c_size_t()
    st = [lib.ctm_su_workspace_size(n, d, D, ctypes.byref(nb))]
    ctx = ctypes.c_void_p()
    st.append(lib.ctm_su_init(n, d, D, ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31), ctypes.c_void_p(1 << 40),
                              nb.value, None, ctypes.byref(ctx)))
    st.append(lib.ctm_su_set_gates(ctx, ctypes.c_void_p(1 << 32), 0.05))
    steps = ctypes.c_int32()
    ch = (ctypes.c_double * n)()
    st.append(lib.ctm_su_evolve(ctx, 3, 0.0, 1, ctypes.byref(steps), ch))
    st.append(lib.ctm_su_state(ctx, ctypes.c_void_p(1 << 33), ctypes.c_void_p(1 << 34)))
    st.append(lib.ctm_su_peps(ctx, ctypes.c_void_p(1 << 35)))
    out.append([n, d, D, st, steps.value, lib.ctm_last_error().decode()])
    lib.ctm_su_destroy(ctx)
nb = ctypes.c_size_t()
out.append(["too big", lib.ctm_su_workspace_size(1, 64, 4, ctypes.byref(nb))])
print(json.dumps(out))
'''


def run_su_dry(lib, extra_env=None):
    import json
    env = dict(os.environ, CTM_DRY_RUN="1", **(extra_env or {}))
    r = subprocess.run([sys.executable, "-c", DRY_SU % {"root": ROOT, "lib": lib}], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1]), r


def test_su_dry_run(lib_path):
    """The simple update's orchestration (gate construction, Trotter steps,
    state and iPEPS export, the full Jacobi and the subspace-iteration
    truncation) passes the host-side bounds checks; d D above the factor
    size limit is rejected."""
    res, _ = run_su_dry(lib_path)
    for row in res[:-1]:
        n, d, D, st, steps, err = row
        assert all(v == 0 for v in st), row
        assert steps == 3
    assert res[-1][1] == 1  # CTM_E_INVALID: d D = 256 > 192
