"""Oracle: observables from a CTM environment (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Norm per site.  The paper expresses the fidelity per site through dominant
  eigenvectors of transfer matrices (Sec. III, Eqs. for F, the 0D transfer
  matrices E and K, and Eq. "fidelity"), and states that, asymptotically on the
  infinite lattice, all of them are given by the corners and edges of the CTM
  environment (Sec. III, Fig. 5 caption and the paragraph after Eq.
  "fidelity").  With the environment around one unit cell this gives the ratio
      kappa_cell = Z11 * Z00 / (Z10 * Z01)
  where Z11 is the cell surrounded by its environment, Z00 the four corners
  alone, Z10 the top and bottom strips joined directly and Z01 the left and
  right strips joined directly.  Applied to the norm network it is the norm per
  cell; applied to the mixed network A (x) B* it is the fidelity scaling
  variable before normalisation.  Per site: kappa_cell ** (1 / (Lx Ly)).
* Fidelity per site (Sec. III, Eq. "fidelity"): for normalised states,
  d = |kappa_AB| / sqrt(kappa_AA kappa_BB) with every kappa per site.
* Nearest-neighbour reduced density matrices and correlators (Sec. II C; the
  observables of Sec. VI): the two-site window with open physical legs, divided
  by its trace, never symmetrised.
* Energy: sum over the bonds of a cell of tr(rho_b h_b) (Sec. II B, H as a
  sum of nearest-neighbour terms; App. A for the ruby block-site terms).
"""
import numpy as np

from .ctm import _Frame, rot_phys

__all__ = ["cell_Z", "kappa", "rdm", "energy", "fidelity", "herm_defect"]


# --------------------------------------------------------------------------
# Z11, Z00, Z10, Z01 around the unit cell anchored at site (0, 0)
# --------------------------------------------------------------------------
def _top(env, Lx):
    """[a, U_0 .. U_{Lx-1}, b]: C1 T1 .. T1 C2 along the top of the cell."""
    v = env.C[0][(0, 0)]                                    # [a, n]
    for x in range(Lx):
        v = np.tensordot(v, env.T[0][(x, 0)], axes=([v.ndim - 1], [0]))
    return np.tensordot(v, env.C[1][(Lx - 1, 0)], axes=([v.ndim - 1], [0]))


def _bottom(env, Lx, Ly):
    """[g, Dn_0 .. Dn_{Lx-1}, b]: C4 T3 .. T3 C3 along the bottom, legs facing up."""
    y = Ly - 1
    w = env.C[3][(0, y)].T                                  # [g (T4-side), d (T3-side)]
    for x in range(Lx):
        T3 = env.T[2][(x, y)]                               # [z (C3-side), Dn, d (C4-side)]
        w = np.tensordot(w, T3, axes=([w.ndim - 1], [2]))    # [..., z, Dn]
        w = np.moveaxis(w, -2, -1)                          # [..., Dn, z]
    C3 = env.C[2][(Lx - 1, y)]                              # [t (T2-side), z (T3-side)]
    return np.tensordot(w, C3, axes=([w.ndim - 1], [1]))     # [g, Dn.., t]


def _row(v, cell, env, y, with_sites=True):
    """Push the boundary [a, U_0.., b] through row y of the cell."""
    Lx = cell.Lx
    T4 = env.T[3][(0, y)]                                   # [g, L, a]
    v = np.tensordot(T4, v, axes=([2], [0]))                # [g, L, U_0.., b]
    if with_sites:
        for x in range(Lx):
            a = cell.a(x, y)                                # [U, L, Dn, R]
            # current layout [g, Dn_0..Dn_{x-1}, L, U_x, U_{x+1}.., b]
            v = np.tensordot(v, a, axes=([1 + x, 2 + x], [1, 0]))  # [..., Dn, R]
            v = np.moveaxis(v, -2, 1 + x)                   # Dn back in place
            v = np.moveaxis(v, -1, 2 + x)                   # R becomes the next L
    T2 = env.T[1][(Lx - 1, y)]                              # [b, R, b']
    nd = v.ndim
    return np.tensordot(v, T2, axes=([nd - 2, nd - 1], [1, 0]))


def cell_Z(cell, env):
    """(Z11, Z00, Z10, Z01) of the cell window anchored at site (0, 0)."""
    Lx, Ly = cell.Lx, cell.Ly
    top = _top(env, Lx)
    bot = _bottom(env, Lx, Ly)
    # Z10: top strip joined directly to the bottom strip
    Z10 = np.tensordot(top, bot, axes=(list(range(top.ndim)),) * 2)
    # Z11: full window
    v = top
    for y in range(Ly):
        v = _row(v, cell, env, y)
    Z11 = np.tensordot(v, bot, axes=(list(range(v.ndim)),) * 2)
    # Z00: corners only
    Z00 = np.trace(env.C[0][(0, 0)] @ env.C[1][(Lx - 1, 0)]
                   @ env.C[2][(Lx - 1, Ly - 1)] @ env.C[3][(0, Ly - 1)])
    # Z01: left strip joined directly to the right strip
    m = env.C[0][(0, 0)] @ env.C[1][(Lx - 1, 0)]            # [a, b]
    for y in range(Ly):
        T4 = env.T[3][(0, y)]                               # [g, L, a]
        T2 = env.T[1][(Lx - 1, y)]                          # [b, R, b']
        m = np.einsum("gla,ab,blc->gc", T4, m, T2)
    Z01 = np.einsum("gc,dg,cd->", m, env.C[3][(0, Ly - 1)],
                    env.C[2][(Lx - 1, Ly - 1)])
    return Z11, Z00, Z10, Z01


def kappa(cell, env, per_site=True):
    """kappa_cell = Z11 Z00 / (Z10 Z01); per site its (Lx Ly)-th root."""
    Z11, Z00, Z10, Z01 = cell_Z(cell, env)
    k = Z11 * Z00 / (Z10 * Z01)
    if per_site:
        n = cell.Lx * cell.Ly
        if n > 1:
            k = np.sign(k.real) * np.abs(k) ** (1.0 / n) if np.isrealobj(k) else k ** (1.0 / n)
    return k


# --------------------------------------------------------------------------
# Two-site reduced density matrices
# --------------------------------------------------------------------------
def _split(x, axis, dk, db):
    shp = list(x.shape)
    shp[axis:axis + 1] = [dk, db]
    return x.reshape(shp)


def rdm(cell, env, x, y, vertical=False, raw=False):
    """rho[(s1, s2), (s1', s2')] for the bond from site (x, y) to its right
    (vertical=False) or lower (vertical=True) neighbour.

    The vertical bond is the horizontal bond of the picture turned by one
    counter-clockwise quarter turn, whose left site is the upper site.
    Rows carry the ket indices (s1, s2), columns the bra indices.
    """
    k = 1 if vertical else 0
    fr = _Frame(cell, env, k)
    # frame position of (x, y): one turn maps (x, y) to (y, -x)
    if vertical:
        xp, yp = y % fr.Lx, (-x) % fr.Ly
    else:
        xp, yp = x % fr.Lx, y % fr.Ly

    def kb(xq, yq):
        s = fr.site(xq, yq)
        return rot_phys(cell.ket(*s), k), rot_phys(cell.bra(*s), k)

    A1, B1 = kb(xp, yp)
    A2, B2 = kb(xp + 1, yp)
    # left block: C1 T1 / T4 site / C4 T3
    X = np.einsum("pn,nue->pue", fr.C(0, xp, yp), fr.T(0, xp, yp))
    X = np.einsum("glp,pue->glue", fr.T(3, xp, yp), X)
    X = np.einsum("dg,glue->dlue", fr.C(3, xp, yp), X)
    X = np.einsum("zkd,dlue->zklue", fr.T(2, xp, yp), X)     # [z, Dn, L, U, e]
    _, Du, Dl, Dd, Dr = A1.shape
    _, Eu, El, Ed, Er = B1.shape
    X = _split(_split(_split(X, 3, Du, Eu), 2, Dl, El), 1, Dd, Ed)
    # X [z, d, d', l, l', u, u', e]
    L = np.einsum("zdDlLuUe,suldr,SULDR->zesrSR", X, A1, np.conj(B1),
                  optimize=True)
    # right block: T1 C2 / site T2 / T3 C3
    Y = np.einsum("mun,nb->mub", fr.T(0, xp + 1, yp), fr.C(1, xp + 1, yp))
    Y = np.einsum("mub,brt->murt", Y, fr.T(1, xp + 1, yp))
    Y = np.einsum("murt,ts->murs", Y, fr.C(2, xp + 1, yp))
    Y = np.einsum("murs,skz->murkz", Y, fr.T(2, xp + 1, yp))  # [m, U, R, Dn, z]
    _, Du, Dl, Dd, Dr = A2.shape
    _, Eu, El, Ed, Er = B2.shape
    Y = _split(_split(_split(Y, 3, Dd, Ed), 2, Dr, Er), 1, Du, Eu)
    # Y [m, u, u', r, r', d, d', z]
    R = np.einsum("muUrRdDz,suldr,SULDR->mzslSL", Y, A2, np.conj(B2),
                  optimize=True)
    rho = np.einsum("zesrSR,ezqrQR->sqSQ", L, R, optimize=True)
    d1, d2 = A1.shape[0], A2.shape[0]
    rho = rho.reshape(d1 * d2, d1 * d2)
    if raw:
        return rho
    return rho / np.trace(rho)


def herm_defect(rho):
    """||rho - rho^H||_F / ||rho||_F."""
    return np.linalg.norm(rho - rho.conj().T) / np.linalg.norm(rho)


def energy(cell, env, bond_h):
    """Sum over the cell's 2 Lx Ly bonds of Re tr(rho_b h_b).

    `bond_h(x, y, vertical)` returns the two-site operator of the bond from
    (x, y) to its right / lower neighbour, as a matrix on (s1, s2) with the
    same ordering as `rdm`.  Returns (total per cell, list of bond values).
    """
    vals = []
    for vertical in (False, True):
        for y in range(cell.Ly):
            for x in range(cell.Lx):
                h = bond_h(x, y, vertical)
                if h is None:
                    vals.append(0.0)
                    continue
                rho = rdm(cell, env, x, y, vertical)
                vals.append(float(np.real(np.trace(rho @ h))))
    return float(np.sum(vals)), vals


def fidelity(kappa_ab, kappa_aa, kappa_bb):
    """d = |kappa_AB| / sqrt(kappa_AA kappa_BB), all per site."""
    return float(np.abs(kappa_ab) / np.sqrt(np.abs(kappa_aa * kappa_bb)))
