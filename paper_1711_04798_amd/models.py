"""Bond Hamiltonians of the ruby model on the 2x2 checkerboard of block
sites (App. A), as host arrays for ctm_su_set_gates and ctm_expect.

Each block site holds the three spins of a triangle, d = 8, basis index
s = 4 b1 + 2 b2 + b3 (b = 0: sigma^z = +1).  Every two-spin product carries
-J_alpha (the model Hamiltonian H = -sum_alpha J_alpha sum sigma^alpha
sigma^alpha); the on-site triangle terms -J_z (z1 z2 + z1 z3 + z2 z3) are
split half and half over the two vertical bonds of a site; the B -> A
horizontal term is the zero operator.  Two-site operators act on
(s_first, s_second), the first site the left or upper one.
"""
import numpy as np

__all__ = ["ruby_bond_hamiltonians"]

_PAULI = {"x": np.array([[0, 1], [1, 0]], dtype=complex),
          "y": np.array([[0, -1j], [1j, 0]], dtype=complex),
          "z": np.array([[1, 0], [0, -1]], dtype=complex)}


def _on_spin(alpha, spin):
    """8 x 8 matrix of sigma^alpha on spin 1, 2 or 3 of a block."""
    sh = 3 - spin  # bit position of the spin in s
    op = _PAULI[alpha]
    m = np.zeros((8, 8), dtype=complex)
    for s in range(8):
        for t in range(8):
            if (s ^ t) & ~(1 << sh) & 7:
                continue  # the other two spins must agree
            m[s, t] = op[(s >> sh) & 1, (t >> sh) & 1]
    return m


def _two(first, second):
    return np.einsum("ab,cd->acbd", first, second).reshape(64, 64)


def ruby_bond_hamiltonians(J=(1.0, 1.0, 1.0)):
    """float64 [4][64][64]: H_r (A left), H_l (B left), H_u (A on top), H_d
    (B on top), the order of the simple update's bond types h0, h1, v0, v1."""
    Jx, Jy, Jz = J
    X = {i: _on_spin("x", i) for i in (1, 2, 3)}
    Y = {i: _on_spin("y", i) for i in (1, 2, 3)}
    Z = {i: _on_spin("z", i) for i in (1, 2, 3)}
    tri = -Jz * (Z[1] @ Z[2] + Z[1] @ Z[3] + Z[2] @ Z[3])
    one = np.eye(8)
    Hr = -Jx * _two(X[1], X[1]) - Jy * _two(Y[3], Y[3])
    Hl = np.zeros((64, 64))
    vert = -Jx * _two(X[3], X[2]) - Jy * _two(Y[2], Y[1])
    Hu = 0.5 * (_two(tri, one) + _two(one, tri)) + vert
    Hd = 0.5 * (_two(tri, one) + _two(one, tri)) + vert
    out = np.array([Hr, Hl, Hu, Hd])
    assert np.abs(out.imag).max() < 1e-14
    return np.ascontiguousarray(out.real)
