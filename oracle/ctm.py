"""Oracle: directional corner-transfer-matrix (CTM) renormalisation, float64, CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring): never called by the GPU
library.

What the paper fixes
--------------------
* The reduced (double-layer) tensor a is obtained by contracting A with A* over
  the physical index (Sec. II C, caption of Fig. 3(a)); for the fidelity the
  bra layer is the second state's tensor (caption of Fig. 4(a)).
* The environment of the unit cell consists of four chi x chi corner matrices
  C1..C4 and edge tensors of shape chi x chi x D^2 (Sec. II C, caption of
  Fig. 3(b)); it is obtained by the directional CTM method and its refinement
  for multi-site cells (Sec. II C).

Readings where the paper is silent (the full list is in the design notes)
------------------------------------------------------------------------
* Tensor legs: A[s, u, l, d, r]; x points right, y points down; a site (x, y)
  uses tensor ``pattern[y * Lx + x]``.
* Double-layer legs are fused ket-major: U = u * D_bra + u'.
* Every site (x, y) owns a full environment C1..C4, T1..T4.  C1 is up-left,
  T1 up, C2 up-right, T2 right, C3 down-right, T3 down, C4 down-left.  Legs of
  each environment tensor are listed clockwise around the site:
  C1[T4-side, T1-side], T1[C1-side, inner, C2-side], C2[T1-side, T2-side],
  T2[C2-side, inner, C3-side], C3[T2-side, T3-side], T3[C3-side, inner, C4-side],
  C4[T3-side, T4-side], T4[C4-side, inner, C1-side].
* A cut index is (chi leg, D^2 leg), chi-major.
* Projectors come from the SVD of the product of the two half-system
  matrices (the four enlarged corners of a plaquette), N = (Lh Uh)^T, keeping
  the top chi singular values above a relative cutoff; the inverse square root
  of the kept singular values is split symmetrically between the two
  projectors.
* A move in direction L, U, R, D is a left move of the picture turned by
  k = 0, 1, 2, 3 counter-clockwise quarter turns; one sweep is L, R, U, D; a
  left move treats columns x = 0 .. Lx-1 in order, one column step each.  In a
  column step all projectors are computed from the current environment before
  any tensor is replaced.
* New corners and edges are divided by their Frobenius norm.
* Trivial start: C = e0 e0^T and T[a, (u,u'), b] = delta_a0 delta_b0 delta_uu'
  (open boundary with ket and bra boundary bonds traced), zero-padded to chi.
"""
import numpy as np

__all__ = [
    "double_layer", "rot_a", "rot_phys", "Cell", "Env", "frame_dims",
    "frame_site", "enlarged_corner", "projectors", "column_step", "move",
    "sweep", "corner_spectra", "converge", "init_trivial", "init_diag",
]

DIRS = {"L": 0, "U": 1, "R": 2, "D": 3}
SWEEP_ORDER = ("L", "R", "U", "D")


# --------------------------------------------------------------------------
# Double layer (Sec. II C, Fig. 3(a) caption; Fig. 4(a) caption for A != B)
# --------------------------------------------------------------------------
def double_layer(A, B=None):
    """a[U, L, Dn, R] = sum_s A[s,u,l,d,r] * conj(B[s,u',l',d',r']).

    Each double leg is fused ket-major: U = u * Du' + u'.  With B omitted the
    bra layer is A itself (the norm network); with B given it is the mixed
    network used for the fidelity.
    """
    if B is None:
        B = A
    a = np.einsum("suldr,svmeq->uvlmderq", A, np.conj(B))
    _, Du, Dl, Dd, Dr = A.shape
    _, Eu, El, Ed, Er = B.shape
    return a.reshape(Du * Eu, Dl * El, Dd * Ed, Dr * Er)


def rot_a(a, k):
    """Turn a double-layer tensor [U, L, Dn, R] by k counter-clockwise quarter turns.

    After one turn the new up leg is the old right leg, the new left leg the
    old up leg, and so on: rot(a)[U', L', D', R'] = a[L', D', R', U'].
    """
    for _ in range(k % 4):
        a = a.transpose(3, 0, 1, 2)
    return a


def rot_phys(A, k):
    """The same quarter turns applied to the bond legs of A[s, u, l, d, r]."""
    for _ in range(k % 4):
        A = A.transpose(0, 4, 1, 2, 3)
    return A


# --------------------------------------------------------------------------
# Unit cell and environment containers
# --------------------------------------------------------------------------
class Cell:
    """Lx x Ly unit cell: site (x, y) carries ket tensor kets[pattern[y*Lx+x]].

    `bras` (same length as `kets`) gives the bra layer; by default the bra
    layer is the ket layer (norm network).
    """

    def __init__(self, Lx, Ly, pattern, kets, bras=None):
        self.Lx, self.Ly = Lx, Ly
        self.pattern = list(pattern)
        self.kets = [np.asarray(A) for A in kets]
        self.bras = self.kets if bras is None else [np.asarray(B) for B in bras]
        self._a = [double_layer(A, B) for A, B in zip(self.kets, self.bras)]

    def tid(self, x, y):
        return self.pattern[(y % self.Ly) * self.Lx + (x % self.Lx)]

    def a(self, x, y):
        return self._a[self.tid(x, y)]

    def ket(self, x, y):
        return self.kets[self.tid(x, y)]

    def bra(self, x, y):
        return self.bras[self.tid(x, y)]


class Env:
    """C[i][(x, y)], T[i][(x, y)] for i = 0..3 meaning C1..C4 and T1..T4."""

    def __init__(self, Lx, Ly, chi):
        self.Lx, self.Ly, self.chi = Lx, Ly, chi
        self.C = [dict() for _ in range(4)]
        self.T = [dict() for _ in range(4)]

    def copy(self):
        e = Env(self.Lx, self.Ly, self.chi)
        for i in range(4):
            e.C[i] = {k: v.copy() for k, v in self.C[i].items()}
            e.T[i] = {k: v.copy() for k, v in self.T[i].items()}
        return e


def _inner_dims(cell, x, y):
    """(ket D, bra D) of the up, right, down, left legs of site (x, y)."""
    A, B = cell.ket(x, y), cell.bra(x, y)
    # order of T1..T4: up, right, down, left -> A legs u=1, r=4, d=3, l=2
    return [(A.shape[j], B.shape[j]) for j in (1, 4, 3, 2)]


def init_trivial(cell, chi):
    """Open boundary with ket and bra boundary bonds traced, zero-padded to chi."""
    env = Env(cell.Lx, cell.Ly, chi)
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            for i in range(4):
                C = np.zeros((chi, chi))
                C[0, 0] = 1.0
                env.C[i][(x, y)] = C
                Dk, Db = _inner_dims(cell, x, y)[i]
                T = np.zeros((chi, Dk * Db, chi))
                for u in range(min(Dk, Db)):
                    T[0, u * Db + u, 0] = 1.0
                env.T[i][(x, y)] = T
    return env


def init_diag(cell, chi, spectra):
    """Diagonal corners C_i = diag(s_i) and T[a,(u,u'),b] = delta_ab delta_uu'.

    `spectra[(x, y)][i]` is the length-chi vector s_i for corner i at (x, y).
    Every tensor is then divided by its Frobenius norm.
    """
    env = Env(cell.Lx, cell.Ly, chi)
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            for i in range(4):
                C = np.diag(np.asarray(spectra[(x, y)][i], dtype=float))
                env.C[i][(x, y)] = C / np.linalg.norm(C)
                Dk, Db = _inner_dims(cell, x, y)[i]
                T = np.zeros((chi, Dk * Db, chi))
                for u in range(min(Dk, Db)):
                    T[:, u * Db + u, :] = np.eye(chi)
                env.T[i][(x, y)] = T / np.linalg.norm(T)
    return env


# --------------------------------------------------------------------------
# Turned frames: a move in direction k is a left move of the turned picture
# --------------------------------------------------------------------------
def frame_dims(k, Lx, Ly):
    return (Lx, Ly) if k % 2 == 0 else (Ly, Lx)


def frame_site(k, xp, yp, Lx, Ly):
    """Site (x, y) of the cell shown at (xp, yp) after k counter-clockwise turns.

    One turn maps (x, y) to (y, -x); undoing it maps (xp, yp) to (-yp, xp).
    """
    for j in range(k % 4, 0, -1):
        lx, ly = frame_dims(j - 1, Lx, Ly)
        xp, yp = (-yp) % lx, xp % ly
    return xp % Lx, yp % Ly


class _Frame:
    """Role view of cell and environment in the picture turned by k quarter turns."""

    def __init__(self, cell, env, k):
        self.cell, self.env, self.k = cell, env, k % 4
        self.Lx, self.Ly = frame_dims(k, cell.Lx, cell.Ly)

    def site(self, xp, yp):
        return frame_site(self.k, xp % self.Lx, yp % self.Ly,
                          self.cell.Lx, self.cell.Ly)

    def C(self, i, xp, yp):
        return self.env.C[(i + self.k) % 4][self.site(xp, yp)]

    def T(self, i, xp, yp):
        return self.env.T[(i + self.k) % 4][self.site(xp, yp)]

    def setC(self, i, xp, yp, v):
        self.env.C[(i + self.k) % 4][self.site(xp, yp)] = v

    def setT(self, i, xp, yp, v):
        self.env.T[(i + self.k) % 4][self.site(xp, yp)] = v

    def a(self, xp, yp):
        return rot_a(self.cell.a(*self.site(xp, yp)), self.k)


# --------------------------------------------------------------------------
# Enlarged corners and projectors
# --------------------------------------------------------------------------
def enlarged_corner(C, Tn, Tp, a):
    """Q[(g, dn), (b, r)] = sum C[p, n] Tn[n, u, b] Tp[g, l, p] a[u, l, dn, r].

    C is the corner, Tn the edge after it and Tp the edge before it in the
    clockwise order; a is the double-layer tensor in the corner's own frame.
    Rows are the cut shared with the previous corner (chi leg of Tp, then the
    down leg of a); columns the cut shared with the next corner (chi leg of
    Tn, then the right leg of a).
    """
    X = np.einsum("glp,pn->gln", Tp, C)
    Y = np.einsum("gln,nub->glub", X, Tn, optimize=True)
    Q = np.einsum("glub,uldr->gdbr", Y, a, optimize=True)
    g, dn, b, r = Q.shape
    return Q.reshape(g * dn, b * r)


def plaquette_corners(fr, xp, yp):
    """The four enlarged corners Q1..Q4 of the plaquette with top-left site (xp, yp)."""
    Q1 = enlarged_corner(fr.C(0, xp, yp), fr.T(0, xp, yp), fr.T(3, xp, yp),
                         fr.a(xp, yp))
    Q2 = enlarged_corner(fr.C(1, xp + 1, yp), fr.T(1, xp + 1, yp),
                         fr.T(0, xp + 1, yp), rot_a(fr.a(xp + 1, yp), 1))
    Q3 = enlarged_corner(fr.C(2, xp + 1, yp + 1), fr.T(2, xp + 1, yp + 1),
                         fr.T(1, xp + 1, yp + 1), rot_a(fr.a(xp + 1, yp + 1), 2))
    Q4 = enlarged_corner(fr.C(3, xp, yp + 1), fr.T(3, xp, yp + 1),
                         fr.T(2, xp, yp + 1), rot_a(fr.a(xp, yp + 1), 3))
    return Q1, Q2, Q3, Q4


def projectors(Q1, Q2, Q3, Q4, chi, cutoff=1e-12, return_info=False):
    """Projectors on the west cut of a plaquette from its half-system matrices.

    Uh = Q1 Q2 (upper half, west x east) and Lh = Q3 Q4 (lower half, east x
    west); N = (Lh Uh)^T = U S V^H.  With the top chi_eff singular values kept
    (those above cutoff * S[0]):
        P1 = Lh^T V S^(-1/2)      (west x chi, attaches to the upper half)
        P2 = S^(-1/2) U^H Uh^T    (chi x west, attaches to the lower half)
    so that Uh^T P1 P2 Lh^T is the best rank-chi_eff approximation of N.
    Both are zero-padded to chi.
    """
    Uh = Q1 @ Q2
    Lh = Q3 @ Q4
    N = (Lh @ Uh).T
    U, S, Vh = np.linalg.svd(N)
    keep = int(min(chi, np.count_nonzero(S > cutoff * S[0]))) if S[0] > 0 else 0
    w = Q1.shape[0]
    dt = np.result_type(Q1, Q2, Q3, Q4)
    P1 = np.zeros((w, chi), dtype=dt)
    P2 = np.zeros((chi, w), dtype=dt)
    if keep:
        isq = 1.0 / np.sqrt(S[:keep])
        P1[:, :keep] = (Lh.T @ Vh[:keep].conj().T) * isq[None, :]
        P2[:keep, :] = isq[:, None] * (U[:, :keep].conj().T @ Uh.T)
    if return_info:
        return P1, P2, {"S": S, "keep": keep}
    return P1, P2


# --------------------------------------------------------------------------
# Absorption (one column step of a left move)
# --------------------------------------------------------------------------
def absorb_corner_up(C1, T1, P1):
    """C1'[b, r] = sum_(p,u) P1[(p,u), b] (C1 T1)[p, u, r]."""
    CT = np.einsum("pn,nur->pur", C1, T1)
    p, u, r = CT.shape
    return np.einsum("pub,pur->br", P1.reshape(p, u, -1), CT)


def absorb_edge(T4, a, P1, P2):
    """T4'[c1, R, c2] = sum P1[(g,dn), c1] T4[g, l, p] a[u, l, dn, R] P2[c2, (p,u)]."""
    g, _, p = T4.shape
    du, _, dd, _ = a.shape
    Ta = np.einsum("glp,uldr->gdrpu", T4, a, optimize=True)
    X = np.einsum("gdc,gdrpu->crpu", P1.reshape(g, dd, -1), Ta, optimize=True)
    return np.einsum("crpu,epu->cre", X, P2.reshape(-1, p, du), optimize=True)


def absorb_corner_down(C4, T3, P2):
    """C4'[z, c] = sum_(g,dn) (T3 C4)[z, dn, g] P2[c, (g, dn)]."""
    X = np.einsum("zdq,qg->zdg", T3, C4)
    _, dn, g = X.shape
    return np.einsum("zdg,cgd->zc", X, P2.reshape(-1, g, dn))


def _fnorm(t):
    n = np.linalg.norm(t)
    return t / n if n > 0 else t


def column_step(cell, env, k, xp, cutoff=1e-12, normalize=True, info=None):
    """One column step of the move in direction k (0=L, 1=U, 2=R, 3=D).

    In the turned picture: projectors for every row from the current
    environment, then C1, T4, C4 of column xp+1 from those of column xp.
    """
    fr = _Frame(cell, env, k)
    chi = env.chi
    P1, P2 = {}, {}
    for yp in range(fr.Ly):
        Qs = plaquette_corners(fr, xp, yp)
        P1[yp], P2[yp], inf = projectors(*Qs, chi, cutoff, return_info=True)
        if info is not None:
            info.append(inf)
    new = []
    for yp in range(fr.Ly):
        up, dn = P1[(yp - 1) % fr.Ly], P2[(yp - 1) % fr.Ly]
        c1 = absorb_corner_up(fr.C(0, xp, yp), fr.T(0, xp, yp), up)
        t4 = absorb_edge(fr.T(3, xp, yp), fr.a(xp, yp), P1[yp], dn)
        c4 = absorb_corner_down(fr.C(3, xp, yp), fr.T(2, xp, yp), P2[yp])
        if normalize:
            c1, t4, c4 = _fnorm(c1), _fnorm(t4), _fnorm(c4)
        new.append((c1, t4, c4))
    for yp, (c1, t4, c4) in enumerate(new):
        fr.setC(0, xp + 1, yp, c1)
        fr.setT(3, xp + 1, yp, t4)
        fr.setC(3, xp + 1, yp, c4)


def move(cell, env, direction, cutoff=1e-12, normalize=True):
    """A full move in one direction: every column of the turned picture in order."""
    k = DIRS[direction] if isinstance(direction, str) else int(direction)
    lx, _ = frame_dims(k, cell.Lx, cell.Ly)
    for xp in range(lx):
        column_step(cell, env, k, xp, cutoff, normalize)


def sweep(cell, env, cutoff=1e-12, normalize=True):
    """One sweep: left, right, up and down moves."""
    for dname in SWEEP_ORDER:
        move(cell, env, dname, cutoff, normalize)


# --------------------------------------------------------------------------
# Convergence measure
# --------------------------------------------------------------------------
def corner_spectra(env):
    """s = sigma(C) / sum sigma(C) for every corner, as {(x, y): [s1..s4]}."""
    out = {}
    for y in range(env.Ly):
        for x in range(env.Lx):
            row = []
            for i in range(4):
                s = np.linalg.svd(env.C[i][(x, y)], compute_uv=False)
                tot = s.sum()
                row.append(s / tot if tot > 0 else s)
            out[(x, y)] = row
    return out


def spectra_delta(s_new, s_old):
    """max over corners and positions of the l1 distance of normalised spectra."""
    return max(np.abs(a - b).sum()
               for key in s_new for a, b in zip(s_new[key], s_old[key]))


def converge(cell, env, tol=1e-10, max_sweeps=500, cutoff=1e-12,
             min_sweeps=1):
    """Sweep until the corner spectra change by less than `tol` (l1, max).

    Returns (sweeps_done, last_delta, converged_flag).
    """
    s_old = corner_spectra(env)
    delta = np.inf
    for it in range(1, max_sweeps + 1):
        sweep(cell, env, cutoff)
        s_new = corner_spectra(env)
        delta = spectra_delta(s_new, s_old)
        s_old = s_new
        if it >= min_sweeps and delta < tol:
            return it, delta, True
    return max_sweeps, delta, False
