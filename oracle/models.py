"""Oracle: model tensors and Hamiltonian terms (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Ruby model (Sec. V, Eq. "eq:H-KR"; block-site form in App. A)
----------------------------------------------------------------
H_R = -sum_alpha J_alpha sum_{alpha-links} sigma^alpha_i sigma^alpha_j.  Each
block site holds the three spins of a triangle, d = 2^3 = 8 (Sec. II B).
Readings where the appendix is silent or garbled:
* The appendix lists the spin products without -J_alpha; each product of two
  sigma^alpha is multiplied here by -J_alpha, as in Eq. "eq:H-KR".
* The B -> A horizontal term is written as the identity operator; it is taken
  as "no interaction" (the zero operator), since the gate it generates is the
  identity.
* Block basis: s = 4 b1 + 2 b2 + b3 for spins 1, 2, 3 of the triangle, with
  b = 0 meaning sigma^z = +1.
* On the checkerboard (A at x + y even) a horizontal bond with A on the left is
  H_r, with B on the left H_l (= 0); a vertical bond with A on top is H_u, with
  B on top H_d.  Two-site operators act on (s_first, s_second) with the left
  (or upper) site first.
* Energy per spin = (energy per 2x2 cell) / 12 (four block sites of three
  spins each).
"""
import numpy as np

__all__ = [
    "PAULI", "spin_op", "ruby_terms", "ruby_bond_h", "ising_peps",
    "product_peps",
]

I2 = np.eye(2)
SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SY = np.array([[0.0, -1.0j], [1.0j, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
PAULI = {"x": SX, "y": SY, "z": SZ}


def spin_op(ops, n=3):
    """Kronecker product over n spins, spin 1 the most significant factor.

    `ops` maps spin number (1-based) to a 2x2 matrix; other spins get identity.
    """
    out = np.eye(1)
    for j in range(1, n + 1):
        out = np.kron(out, ops.get(j, I2))
    return out


def _pair(alpha, i, beta, j):
    """sigma^alpha on spin i of the first block times sigma^beta on spin j of the second."""
    return np.kron(spin_op({i: PAULI[alpha]}), spin_op({j: PAULI[beta]}))


def ruby_terms(J=(1.0, 1.0, 1.0)):
    """Block-site ruby terms of App. A with the -J_alpha factors.

    Returns a dict of real matrices: 'hA', 'hB' (8x8 on-site triangle terms),
    'hx_AB', 'hx_BA', 'hy_AB', 'hy_BA' (64x64, first factor the first block
    named), and the bond Hamiltonians 'Hr', 'Hl', 'Hu', 'Hd' (64x64).
    """
    Jx, Jy, Jz = J
    zz = (spin_op({1: SZ, 2: SZ}) + spin_op({1: SZ, 3: SZ})
          + spin_op({2: SZ, 3: SZ}))
    hA = -Jz * zz
    hB = -Jz * zz
    hx_AB = -Jx * _pair("x", 1, "x", 1) - Jy * _pair("y", 3, "y", 3)
    hx_BA = np.zeros((64, 64))
    hy_AB = -Jx * _pair("x", 3, "x", 2) - Jy * _pair("y", 2, "y", 1)
    # h^y_{iB,jA}: sigma^x_{B3} sigma^x_{A2} + sigma^y_{B2} sigma^y_{A1},
    # with B the first (upper) block
    hy_BA = -Jx * _pair("x", 3, "x", 2) - Jy * _pair("y", 2, "y", 1)
    e8 = np.eye(8)
    Hr = hx_AB
    Hl = hx_BA
    Hu = 0.5 * (np.kron(hA, e8) + np.kron(e8, hB)) + hy_AB
    Hd = 0.5 * (np.kron(hB, e8) + np.kron(e8, hA)) + hy_BA
    out = dict(hA=hA, hB=hB, hx_AB=hx_AB, hx_BA=hx_BA, hy_AB=hy_AB,
               hy_BA=hy_BA, Hr=Hr, Hl=Hl, Hu=Hu, Hd=Hd)
    return {k: np.real_if_close(v) for k, v in out.items()}


def ruby_bond_h(J=(1.0, 1.0, 1.0)):
    """bond_h(x, y, vertical) for the 2x2 checkerboard (A at x + y even)."""
    t = ruby_terms(J)

    def bond_h(x, y, vertical):
        first_is_A = (x + y) % 2 == 0
        if vertical:
            return t["Hu"] if first_is_A else t["Hd"]
        return t["Hr"] if first_is_A else t["Hl"]

    return bond_h


def ising_peps(K):
    """PEPS whose norm network is the classical Ising model at coupling K.

    A[s, u, l, d, r] = W[s, u] W[s, l] W[s, d] W[s, r] with W W^T =
    exp((K/2) s s'), so that ket and bra together give exp(K s s') per bond.
    """
    c, s = np.sqrt(np.cosh(K / 2)), np.sqrt(np.sinh(K / 2))
    W = np.array([[c, s], [c, -s]])
    return np.einsum("su,sl,sd,sr->suldr", W, W, W, W)


def product_peps(phi):
    """D = 1 tensor A[s, 0, 0, 0, 0] = phi_s."""
    phi = np.asarray(phi)
    return phi.reshape(-1, 1, 1, 1, 1)
