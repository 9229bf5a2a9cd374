"""Oracle: simple update of the 2x2 checkerboard iPEPS (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II B writes e^{-beta H} as m first-order Suzuki-Trotter factors
e^{-dtau H_r} e^{-dtau H_l} e^{-dtau H_u} e^{-dtau H_d}, each a product of
two-body gates g = e^{-dtau h} on one type of link.  Sec. II D starts the
ground-state search with the simple update (the weighted-bond truncation of
Jiang, Weng and Xiang, which the paper cites and does not restate).

Readings (the paper gives no steps of the simple update):
* Every bond carries a weight vector lambda (length D).  The 2x2 checkerboard
  (A at x + y even) has four bond types, named after the term acting on them:
  h0 = A.r - B.l (H_r), h1 = B.r - A.l (H_l), v0 = A.d - B.u (H_u),
  v1 = B.d - A.u (H_d); the first site of a bond is the left (upper) one.
* One Trotter step updates h0, h1, v0, v1 in that order (r, l, u, d).
* A bond update: multiply the weights of the two tensors' other legs in;
  reduce each tensor by a QR decomposition of [(other legs) x (s, bond)];
  form theta = R_X lambda R_Y, apply the gate to the two physical indices;
  SVD theta and keep the D largest singular values that exceed 1e-12 times
  the largest (the rest of the D slots are zero); the kept values divided by
  their Euclidean norm are the new weights; rebuild the tensors from the Q
  factors and the singular vectors, divide the other legs' weights out
  (weights below 1e-12 times the largest of their bond count as zero, their
  inverse as zero) and divide each tensor by its Frobenius norm.
* Gates from the symmetric bond Hamiltonian h by its eigendecomposition:
  g = V diag(exp(-dtau w)) V^T; g[(i, j), (k, l)] maps the physical indices
  (k, l) of the (first, second) site to (i, j).
* Convergence: the largest absolute change of any weight over one step.
"""
import numpy as np

__all__ = ["BONDS", "ENDS", "LEG_BOND", "gates_from", "init_weights", "bond_update", "step", "evolve",
           "peps_tensors"]

BONDS = ("h0", "h1", "v0", "v1")
# (tensor, leg) of the first and the second site of each bond; legs of
# T[s, u, l, d, r] are numbered u = 1, l = 2, d = 3, r = 4; tensor 0 = A, 1 = B
ENDS = {"h0": ((0, 4), (1, 2)), "h1": ((1, 4), (0, 2)), "v0": ((0, 3), (1, 1)), "v1": ((1, 3), (0, 1))}
# the bond each leg of A and of B belongs to
LEG_BOND = {0: {1: "v1", 2: "h1", 3: "v0", 4: "h0"}, 1: {1: "v0", 2: "h0", 3: "v1", 4: "h1"}}
EPS = 1e-12


def gates_from(bond_h, dtau):
    """Gates of the four bond types; bond_h(x, y, vertical) as in
    models.ruby_bond_h (first site at (x, y), A at x + y even)."""
    where = {"h0": (0, 0, False), "h1": (1, 0, False), "v0": (0, 0, True), "v1": (1, 0, True)}
    out = {}
    for b, (x, y, v) in where.items():
        h = np.asarray(bond_h(x, y, v), dtype=np.float64)
        w, V = np.linalg.eigh(0.5 * (h + h.T))
        out[b] = (V * np.exp(-dtau * w)) @ V.T
    return out


def init_weights(D, rank=None):
    """Uniform weights 1/sqrt(r) on the first r slots (r = D by default)."""
    rank = rank or {}
    lam = {}
    for b in BONDS:
        r = rank.get(b, D)
        v = np.zeros(D)
        v[:r] = 1.0 / np.sqrt(r)
        lam[b] = v
    return lam


def _scale_legs(X, t, skip, lam, inverse):
    for leg in range(1, 5):
        if leg == skip:
            continue
        w = lam[LEG_BOND[t][leg]]
        if inverse:
            big = w > EPS * max(w.max(), 0.0)
            w = np.where(big, 1.0 / np.where(big, w, 1.0), 0.0)
        shape = [1] * 5
        shape[leg] = -1
        X = X * w.reshape(shape)
    return X


def bond_update(T, lam, bond, G, D):
    """One simple-update step on `bond` with gate G (d^2 x d^2); T = [A, B]
    and lam are updated in place."""
    (t1, p1), (t2, p2) = ENDS[bond]
    d = T[t1].shape[0]
    mats = []
    for t, p in ((t1, p1), (t2, p2)):
        Xt = _scale_legs(T[t], t, p, lam, False)
        Xm = np.moveaxis(Xt, [0, p], [-2, -1])       # [others..., s, bond]
        oshape = Xm.shape[:3]
        Q, R = np.linalg.qr(Xm.reshape(-1, d * D))    # R: k x (s, bond)
        mats.append((Q, R.reshape(-1, d, D), oshape))
    (QX, RX, osx), (QY, RY, osy) = mats
    theta = np.einsum("aip,p,bjp->aibj", RX, lam[bond], RY)
    theta = np.einsum("ijkl,akbl->aibj", G.reshape(d, d, d, d), theta)
    ka, kb = RX.shape[0], RY.shape[0]
    U, S, Vh = np.linalg.svd(theta.reshape(ka * d, kb * d), full_matrices=False)
    keep = int(np.sum(S[:D] > EPS * S[0])) if S[0] > 0 else 0
    lam_new = np.zeros(D)
    lam_new[:keep] = S[:keep] / np.linalg.norm(S[:keep])
    RXn = np.zeros((ka * d, D))
    RYn = np.zeros((kb * d, D))
    RXn[:, :keep] = U[:, :keep]
    RYn[:, :keep] = Vh[:keep].T
    lam[bond] = lam_new
    for t, p, Q, Rn, k, osh in ((t1, p1, QX, RXn, ka, osx), (t2, p2, QY, RYn, kb, osy)):
        Xm = (Q @ Rn.reshape(k, d * D)).reshape(*osh, d, D)
        X = np.moveaxis(Xm, [-2, -1], [0, p])
        X = _scale_legs(X, t, p, lam, True)
        T[t] = X / np.linalg.norm(X)


def step(T, lam, gates, D):
    """One first-order Trotter step: bonds r, l, u, d in turn."""
    for b in BONDS:
        bond_update(T, lam, b, gates[b], D)


def evolve(T, lam, gates, D, max_steps, tol=0.0):
    """Trotter steps until the weights change by less than tol (or max_steps);
    returns (steps done, last change)."""
    change = np.inf
    for n in range(1, max_steps + 1):
        old = {b: v.copy() for b, v in lam.items()}
        step(T, lam, gates, D)
        change = max(np.abs(lam[b] - old[b]).max() for b in BONDS)
        if change < tol:
            return n, change
    return max_steps, change


def peps_tensors(T, lam):
    """The iPEPS tensors of the state: every bond's weight split as sqrt(lambda)
    onto the legs of its two ends."""
    out = []
    for t in (0, 1):
        X = T[t]
        for leg in range(1, 5):
            shape = [1] * 5
            shape[leg] = -1
            X = X * np.sqrt(lam[LEG_BOND[t][leg]]).reshape(shape)
        out.append(X)
    return out
