"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  Every PEPS tensor is a real array in C order with legs
[s, u, l, d, r] (physical index first, then the up, left, down and right bond
indices), drawn i.i.d. from N(0, 1) in float64 by ``numpy.random.default_rng``
and scaled to unit Frobenius norm.  The paper's tensors carry a physical index
of dimension d and four bond indices of dimension D (Sec. II A, Eq. 1); for the
ruby lattice a block site has d = 2^3 = 8 (Sec. II B, caption of Fig. 1(d)).
"""
import numpy as np

__all__ = [
    "peps_tensor", "cell_tensors", "batched_instances", "warm_family",
    "warm_thetas",
]


def peps_tensor(rng, d, D):
    """One tensor of shape (d, D, D, D, D), N(0,1) entries, Frobenius norm 1."""
    A = rng.standard_normal((d, D, D, D, D))
    return A / np.linalg.norm(A)


def cell_tensors(seed, d, D, n_tensors):
    """`n_tensors` tensors drawn in order from one generator seeded with `seed`."""
    rng = np.random.default_rng(seed)
    return [peps_tensor(rng, d, D) for _ in range(n_tensors)]


def batched_instances(seed, n_inst, d=8, Ds=(3, 4, 5), chis=(32, 64, 100)):
    """Independent 1x1-cell instances with (D, chi) drawn uniformly per instance.

    For each instance in turn: D from `Ds`, chi from `chis`, then the tensor,
    all from one generator seeded with `seed`.  Returns a list of (D, chi, A).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        D = int(Ds[rng.integers(len(Ds))])
        chi = int(chis[rng.integers(len(chis))])
        out.append((D, chi, peps_tensor(rng, d, D)))
    return out


def warm_family(seed, d=8, D=4):
    """The three seeded base tensors A0, A1, A2 of the one-parameter family."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((d, D, D, D, D)) for _ in range(3)]


def warm_member(base, theta):
    """A(theta) = normalize(cos t1 * A0 + sin t1 * A1 + t2 * A2)."""
    A0, A1, A2 = base
    A = np.cos(theta[0]) * A0 + np.sin(theta[0]) * A1 + theta[1] * A2
    return A / np.linalg.norm(A)


def warm_thetas(seed, n):
    """n parameter pairs: t1 ~ U[0, 2 pi), t2 ~ U[-0.5, 0.5]."""
    rng = np.random.default_rng(seed)
    t1 = rng.uniform(0.0, 2.0 * np.pi, n)
    t2 = rng.uniform(-0.5, 0.5, n)
    return np.stack([t1, t2], axis=1)
