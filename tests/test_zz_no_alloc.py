"""The allocation-free fidelity entry point (ctm_fidelity_noalloc) against the
workspace entry point (ctm_fidelity) through the C ABI: two calls in a row,
the second on a smaller configuration, each bitwise equal to the workspace
call (same kernels, same tiles) and within 1e-10 of the CPU oracle."""
import numpy as np
import pytest

import synth
from oracle import ctm as octm
from oracle import obs as oobs

pytestmark = pytest.mark.gpu


def _oracle_fidelity(A, B, chi, tol, max_sweeps):
    kap = {}
    for name, kets, bras in (("ab", [A], [B]), ("aa", [A], None), ("bb", [B], None)):
        cell = octm.Cell(1, 1, [0], kets, bras)
        env = octm.init_trivial(cell, chi)
        octm.converge(cell, env, tol=tol, max_sweeps=max_sweeps)
        kap[name] = oobs.kappa(cell, env)
    return oobs.fidelity(kap["ab"], kap["aa"], kap["bb"])


@pytest.mark.parametrize("order", [0, 1])
def test_noalloc_matches_workspace_entry(gpu, order):
    from paper_1711_04798_amd import binding
    rng = np.random.default_rng(7)
    cases = []
    for (D, chi) in ((3, 24), (2, 8)):
        A, = synth.cell_tensors(40 + D, 2, D, 1)
        B = A + 0.25 * synth.peps_tensor(rng, 2, D)
        B /= np.linalg.norm(B)
        cases.append((A, B, chi))
    if order:
        cases = cases[::-1]
    for A, B, chi in cases:
        print("case noalloc fidelity D=%d chi=%d" % (A.shape[1], chi), flush=True)
        kw = dict(chi=chi, tol=1e-12, max_sweeps=300, autotune=False)
        d0, l0, s0, c0 = binding.fidelity([A], [B], **kw)
        d1, l1, s1, c1 = binding.fidelity_noalloc([A], [B], **kw)
        assert c0 and c1 and s0 == s1, (s0, s1)
        assert d0 == d1 and l0 == l1
        do = _oracle_fidelity(A, B, chi, 1e-12, 300)
        assert abs(d1 - do) <= 1e-10 * abs(do), (d1, do)


def test_noalloc_rejects_oversized(gpu):
    from paper_1711_04798_amd import binding
    A, B = synth.cell_tensors(50, 8, 4, 2)
    print("case noalloc oversized", flush=True)
    with pytest.raises(binding.CtmError) as e:
        binding.fidelity_noalloc([A], [B], chi=64, tol=1e-10, max_sweeps=5)
    assert e.value.status == binding.CTM_E_NOMEM
    assert binding.load().ctm_fidelity_noalloc_max_bytes() == 64 << 20
