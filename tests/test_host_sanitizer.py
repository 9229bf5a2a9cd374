"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host side (planning, orchestration, the boundary operator's
Lanczos and Jacobi, checkpoint and environment (de)serialisation, the
launch-variant table's JSON reader and writer) is built with ASan and UBSan
on the host pass only, and driven in dry-run mode: every launch and copy is
checked against the workspace allocations and then skipped, so no device is
needed and no device code runs.  Any host out-of-bounds access, use after
free or undefined behaviour aborts the run.
"""
import glob
import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))
from paper_1711_04798_amd import build as pkg_build  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "--offload-arch=gfx950", "-std=c++17", "-fPIC"]


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def san_lib(tmp_path_factory):
    try:
        hipcc = pkg_build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    if asan_runtime() is None:
        pytest.skip("clang ASan runtime not found")
    out = tmp_path_factory.mktemp("san")

    def comp(src):
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        extra = [f for f in pkg_build.HIPFLAGS if f != "-O3" and f not in FLAGS]
        cmd = [hipcc, *FLAGS, *extra, *SAN, "-I", pkg_build.INC, "-c", os.path.join(pkg_build.SRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with ThreadPoolExecutor(max_workers=min(7, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, pkg_build.SOURCES))
    lib = str(out / "libctm_san.so")
    r = subprocess.run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *SAN, *objs, "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    # the instrumentation is really there
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms
    return lib


def run_sanitized(code, *args):
    env = dict(os.environ, CTM_DRY_RUN="1", LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", code, *args], capture_output=True, text=True, env=env, timeout=900)
    report = r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr, report
    assert "runtime error:" not in r.stderr, report
    assert r.returncode == 0, report
    return r.stdout


def test_orchestration_under_sanitizers(san_lib):
    import test_abi
    code = test_abi.DRY % {"root": ROOT, "cases": test_abi.CASES, "lib": san_lib}
    res = json.loads(run_sanitized(code).strip().splitlines()[-1])
    assert set(res) == {c[0] for c in test_abi.CASES}
    for name, (st, err, nbytes) in res.items():
        assert all(s == 0 for s in st), (name, st, err)


FID = r'''
import ctypes, sys
sys.path.insert(0, %(root)r)
from paper_1711_04798_amd import binding as b
lib = b.load(%(lib)r, tile_table=False)
for prec in ("fp64", "bf16"):
    cfg, keep = b.make_config(2, 2, [0, 1, 1, 0], 2, [8], [4], [32], prec, max_iters=2)
    n = b.workspace_size(cfg)
    A = (ctypes.c_void_p * 2)(1 << 30, (1 << 30) + 4096)
    B = (ctypes.c_void_p * 2)(1 << 31, (1 << 31) + 4096)
    d, ld = ctypes.c_double(), ctypes.c_double()
    sw = (ctypes.c_int32 * 3)()
    st = lib.ctm_fidelity(ctypes.byref(cfg), ctypes.cast(A, ctypes.POINTER(ctypes.c_void_p)),
                          ctypes.cast(B, ctypes.POINTER(ctypes.c_void_p)), ctypes.c_void_p(1 << 40), n, None,
                          1e-10, 3, ctypes.byref(d), ctypes.byref(ld), sw)
    # the dry run reads back zeros: spectra never change, so the runs stop at once
    print(prec, st, lib.ctm_last_error().decode())
src, dst, bad = sys.argv[1], sys.argv[2], sys.argv[3]
n = ctypes.c_int32()
print("load", lib.ctm_tile_table_load(src.encode(), ctypes.byref(n)), n.value)
print("save", lib.ctm_tile_table_save(dst.encode(), ctypes.byref(n)), n.value)
print("bad", lib.ctm_tile_table_load(bad.encode(), ctypes.byref(n)))
'''


def test_fidelity_and_tile_table_under_sanitizers(san_lib, tmp_path):
    table = os.path.join(ROOT, "paper_1711_04798_amd", "tiles.json")
    bad = tmp_path / "bad.json"
    # truncated and malformed entries
    bad.write_text('[\n{"kernel": "gemm", "ta": 0, "tc": 0, "ak": 1, "bk": 0, "groups": 0, "M": 4\n'
                   '{"kernel": "zz", "variant": -3}\n')
    out = run_sanitized(FID % {"root": ROOT, "lib": san_lib}, table, str(tmp_path / "out.json"), str(bad))
    lines = dict((l.split()[0], l.split()[1:]) for l in out.strip().splitlines())
    n_entries = len(json.load(open(table)))
    assert lines["load"] == ["0", str(n_entries)]
    assert lines["save"] == ["0", str(n_entries)]
    assert lines["bad"][0] != "0"
    for prec in ("fp64", "bf16"):
        assert lines[prec][0] in ("0", "4"), lines[prec]  # CTM_OK or CTM_E_NOCONV


def test_simple_update_under_sanitizers(san_lib):
    import test_abi
    env = dict(LD_PRELOAD=asan_runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res, r = test_abi.run_su_dry(san_lib, env)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-3000:]
    for row in res[:-1]:
        assert all(v == 0 for v in row[3]), row
