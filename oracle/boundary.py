"""Oracle: boundary density operator and entanglement entropy of half an
infinite cylinder from CTM edge tensors (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (Sec. IV, Eq. "Eq:rho" and the text after it):
* the reduced density matrix of half an infinite cylinder of circumference
  N_v is an isometry applied to sqrt(sigma_L^T) sigma_R sqrt(sigma_L^T), so it
  has the spectrum of sigma_L^T sigma_R;
* sigma_L and sigma_R are the dominant left and right eigenvectors of the
  PEPS transfer matrix around the circumference, approximated by the
  half-row transfer tensors T_l and T_r of the CTM environment wrapped
  around a circle of N_v sites;
* the entanglement entropy follows from those eigenvalues.

Readings (the figure is missing):
* The cut runs between columns x0 - 1 and x0 of the cell.  sigma_L is the
  ring of the left edges T4 of column x0 (they face the left legs of the
  sites of column x0), sigma_R the ring of the right edges T2 of column
  x0 - 1 (they face the right legs of the sites of column x0 - 1): both act
  on the virtual indices of the N_v bonds that cross the cut.
* The ring runs over rows y = 0 .. N_v - 1 (edge of row y mod Ly), each
  edge's up-side chi leg joined to the down-side chi leg of the edge above
  and the last one to the first.  A virtual index of the ring is
  (v_0, .., v_{N_v-1}) with v_0 the most significant.
* sigma[(ket), (bra)] carries the ket layer's bond index in the row and the
  bra layer's in the column (the fused double-layer leg is ket-major).
  sigma_L^T sigma_R contracts the ket indices of the two rings.
* Eigenvalues are divided by their sum (the trace); the entropy is
  S = -sum p log p over the positive p.
"""
import numpy as np

__all__ = ["sigma_left", "sigma_right", "boundary_spectrum", "entropy"]


def _ring(mats):
    """Dense ring operator from edge tensors given as [up, ket, bra, down].

    Returns S[(ket_0..ket_{n-1}), (bra_0..bra_{n-1})] = Tr_chi prod_y E_y."""
    n = len(mats)
    chi = mats[0].shape[0]
    D = mats[0].shape[1]
    out = np.zeros((D ** n, D ** n))
    for a0 in range(chi):
        # X[ket.., bra.., c] for the ring opened at row 0's up leg = a0
        X = mats[0][a0]                                  # [ket, bra, c]
        for y in range(1, n):
            X = np.tensordot(X, mats[y], axes=([X.ndim - 1], [0]))  # [..., ket_y, bra_y, c]
        # close the ring: last down leg = a0
        X = X[..., a0]                                   # [k0, b0, k1, b1, ...]
        perm = list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2))
        out += X.transpose(perm).reshape(D ** n, D ** n)
    return out


def _edges(env, which, x, Ly, nv, Dk, Db):
    mats = []
    for y in range(nv):
        T = env.T[which][(x, y % Ly)]
        chi = T.shape[0]
        T = T.reshape(chi, Dk, Db, chi)
        if which == 3:
            # T4[down, (ket, bra), up] -> [up, ket, bra, down]
            T = T.transpose(3, 1, 2, 0)
        mats.append(T)
    return mats


def sigma_left(cell, env, x0, nv):
    """sigma_L: the left edges T4 of column x0 wrapped around N_v rows."""
    x0 = x0 % cell.Lx
    A, B = cell.ket(x0, 0), cell.bra(x0, 0)
    return _ring(_edges(env, 3, x0, cell.Ly, nv, A.shape[2], B.shape[2]))


def sigma_right(cell, env, x0, nv):
    """sigma_R: the right edges T2 of column x0 - 1 wrapped around N_v rows."""
    xr = (x0 - 1) % cell.Lx
    A, B = cell.ket(xr, 0), cell.bra(xr, 0)
    return _ring(_edges(env, 1, xr, cell.Ly, nv, A.shape[4], B.shape[4]))


def boundary_spectrum(cell, env, x0, nv):
    """Eigenvalues of sigma_L^T sigma_R divided by their sum, descending
    (real parts; the imaginary parts are returned for inspection)."""
    if nv % cell.Ly:
        raise ValueError("the circumference must be a multiple of the cell height")
    sl, sr = sigma_left(cell, env, x0, nv), sigma_right(cell, env, x0, nv)
    w = np.linalg.eigvals(sl.T @ sr)
    tr = np.trace(sl.T @ sr)
    order = np.argsort(-w.real)
    w = w[order] / tr
    return w.real, w.imag


def entropy(p):
    """-sum p log p over the positive entries."""
    p = np.asarray(p)
    p = p[p > 0]
    return float(-np.sum(p * np.log(p)))
