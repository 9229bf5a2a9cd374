"""Stage-by-stage parity from an identical environment: the oracle's
environment is imported into the GPU context, one column step is taken on
both sides, and the enlarged corners (elementwise), the projector product
P1 P2 (gauge invariant) and the norm per site of the updated environment are
compared."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs

pytestmark = pytest.mark.gpu


def _dump(g, what, index, shape, dtype=np.float64):
    from paper_1711_04798_amd import binding
    lib = binding.load()
    lib.ctm_debug_dump.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]
    lib.ctm_debug_dump.restype = ctypes.c_int
    buf = np.zeros(shape, dtype=dtype)
    st = lib.ctm_debug_dump(g.ctx, what, index, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes)
    assert st == 0, lib.ctm_last_error()
    return buf


def env_to_flat(env, Lx, Ly):
    parts = [env.C[c][(x, y)].ravel() for c in range(4) for y in range(Ly) for x in range(Lx)]
    parts += [env.T[c][(x, y)].ravel() for c in range(4) for y in range(Ly) for x in range(Lx)]
    return np.concatenate(parts)


def flat_to_env(buf, Lx, Ly, chi, D2):
    env = octm.Env(Lx, Ly, chi)
    o = 0
    for c in range(4):
        for y in range(Ly):
            for x in range(Lx):
                env.C[c][(x, y)] = buf[o:o + chi * chi].reshape(chi, chi); o += chi * chi
    for c in range(4):
        for y in range(Ly):
            for x in range(Lx):
                env.T[c][(x, y)] = buf[o:o + chi * chi * D2].reshape(chi, D2, chi); o += chi * chi * D2
    return env


@pytest.mark.parametrize("direction", ["L", "U", "R", "D"])
@pytest.mark.parametrize("case", ["c0", "2x2"])
def test_one_step_from_same_env(gpu, direction, case):
    from paper_1711_04798_amd import CTM
    if case == "c0":
        tens = synth.cell_tensors(0, 2, 2, 1); Lx = Ly = 1; pat = [0]; chi = 16
    else:
        tens = synth.cell_tensors(3, 2, 2, 2); Lx = Ly = 2; pat = [0, 1, 1, 0]; chi = 8
    cell = octm.Cell(Lx, Ly, pat, tens)
    env = octm.init_trivial(cell, chi)
    for _ in range(3):
        octm.sweep(cell, env)
    print("case", case, direction, flush=True)
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pat, chi=chi)
    g.import_env(env_to_flat(env, Lx, Ly))
    k = octm.DIRS[direction]
    g.move(direction, 1)
    n = chi * 4
    fr = octm._Frame(cell, env, k)
    lx, ly = fr.Lx, fr.Ly
    for yp in range(ly):
        Qo = octm.plaquette_corners(fr, 0, yp)
        for q in range(4):
            Qg = _dump(g, 0, 4 * yp + q, (n, n))
            err = np.abs(Qg - Qo[q]).max() / np.abs(Qo[q]).max()
            print("Q%d row %d rel err %.2e" % (q + 1, yp, err))
            assert err < 1e-13
        P1o, P2o, info = octm.projectors(*Qo, chi, 1e-12, return_info=True)
        P1g = _dump(g, 1, yp, (n, chi))
        P2g = _dump(g, 2, yp, (n, chi)).T
        stt = _dump(g, 3, yp, (14,), np.int32)
        keep = info["keep"]
        # compare the truncated half-system operator Uh^T P1 P2 Lh^T (well
        # conditioned); P1 P2 alone amplifies the smallest kept direction by
        # 1 / sigma_chi
        Uh, Lh = Qo[0] @ Qo[1], Qo[2] @ Qo[3]
        No, Ng = Uh.T @ P1o @ P2o @ Lh.T, Uh.T @ P1g @ P2g @ Lh.T
        err = np.abs(No - Ng).max() / np.abs(No).max()
        res = _dump(g, 3, yp, (7,), np.float64)
        print("row %d keep oracle %d gpu %d iters %d jacobi sweeps %d max_resid %.2e, N_chi rel err %.2e"
              % (yp, keep, stt[0], stt[2], stt[8], res[3], err))
        assert stt[0] == keep
        assert err < 1e-11
        # discarded weight over the subspace's k values (k = stt[10] columns):
        # the oracle's over its top k singular values
        So = np.asarray(info["S"], dtype=np.float64)[:stt[10]]
        do = float((So[keep:] ** 2).sum() / (So ** 2).sum())
        print("row %d discarded weight oracle %.3e gpu %.3e" % (yp, do, res[6]))
        assert abs(res[6] - do) <= 1e-3 * do + 1e-15
    ref = env.copy()
    octm.column_step(cell, ref, k, 0)
    # the norm per site of the moved environment, each side from its own
    ko, kg = oobs.kappa(cell, ref), g.norm()
    print("kappa after step: oracle %.15f gpu %.15f" % (ko, kg))
    assert abs(ko - kg) < 1e-10 * abs(ko)
    g.close()


@pytest.mark.parametrize("prec,tol", [("bf16", 2e-2), ("fp32", 1e-5)])
@pytest.mark.parametrize("D,chi", [(2, 16), (4, 12)])
def test_reduced_precision_corners(gpu, prec, tol, D, chi):
    """Enlarged corners of the bf16 / fp32 paths against the float64 oracle
    from the same environment.  The operands are rounded to the working type
    (unit roundoff 2^-8 for bf16, 2^-24 for fp32) and accumulated in fp32, so
    the relative Frobenius error is a few unit roundoffs."""
    from paper_1711_04798_amd import CTM
    tens = synth.cell_tensors(7, 2, D, 2)
    Lx = Ly = 2
    pat = [0, 1, 1, 0]
    cell = octm.Cell(Lx, Ly, pat, tens)
    env = octm.init_trivial(cell, chi)
    for _ in range(3):
        octm.sweep(cell, env)
    print("case", prec, D, chi, flush=True)
    g = CTM([tens], Lx=Lx, Ly=Ly, pattern=pat, chi=chi, prec=prec, max_iters=2, resid_tol=0.0, cutoff=1e-6)
    g.import_env(env_to_flat(env, Lx, Ly))
    g.move("L", 1)
    n = chi * D * D
    fr = octm._Frame(cell, env, 0)
    for yp in range(2):
        Qo = octm.plaquette_corners(fr, 0, yp)
        for q in range(4):
            Qg = _dump(g, 0, 4 * yp + q, (n, n), np.float32).astype(np.float64)
            err = np.linalg.norm(Qg - Qo[q]) / np.linalg.norm(Qo[q])
            print("%s Q%d row %d rel err %.2e" % (prec, q + 1, yp, err))
            assert err < tol
    g.close()
