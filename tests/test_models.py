"""The host-side ruby bond Hamiltonians of the package (built bit by bit)
equal the oracle's (built from Kronecker products), for several couplings."""
import numpy as np

from oracle import models as om
from paper_1711_04798_amd import models as pm


def test_ruby_bond_hamiltonians_match_oracle():
    for J in [(1.0, 1.0, 1.0), (0.8, 0.8, 0.4), (1.3, -0.2, 0.5)]:
        got = pm.ruby_bond_hamiltonians(J)
        bh = om.ruby_bond_h(J)
        want = [bh(0, 0, False), bh(1, 0, False), bh(0, 0, True), bh(1, 0, True)]
        for g, w in zip(got, want):
            assert np.abs(g - w).max() < 1e-14
