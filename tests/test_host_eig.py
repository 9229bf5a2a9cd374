"""The host eigensolver of the boundary operator's projected matrix
(Householder tridiagonalisation, implicit symmetric QR with Wilkinson
shifts) against numpy.linalg.eigh and its own residuals, on the CPU:
random symmetric matrices of several orders, and the degenerate inputs a
Lanczos projection produces (repeated eigenvalues from translations around
the cylinder, diagonal and already tridiagonal matrices, zero, rank one)."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1711_04798_amd", "libctm.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1711_04798_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(ctypes.c_double)
    lib.ctm_debug_sym_eig.argtypes = [ctypes.c_int32, P, P, P]
    lib.ctm_debug_sym_eig.restype = ctypes.c_int
    return lib


def _eig(lib, A, vectors=True):
    n = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.float64)
    w = np.zeros(n)
    V = np.zeros((n, n)) if vectors else None
    P = ctypes.POINTER(ctypes.c_double)
    st = lib.ctm_debug_sym_eig(n, A.ctypes.data_as(P), w.ctypes.data_as(P), V.ctypes.data_as(P) if vectors else None)
    assert st == 0
    return w, V


def _cases():
    rng = np.random.default_rng(3)
    out = []
    for n in (1, 2, 3, 5, 17, 64, 256):
        M = rng.standard_normal((n, n))
        out.append(("random%d" % n, M + M.T))
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    out.append(("repeated", Q @ np.diag(np.repeat([3.0, 1.0, -0.5, 1e-9], 10)) @ Q.T))
    out.append(("diagonal", np.diag(rng.standard_normal(30))))
    T = np.diag(rng.standard_normal(25)) + np.diag(rng.standard_normal(24), 1)
    out.append(("tridiagonal", T + np.triu(T, 1).T))
    out.append(("zero", np.zeros((12, 12))))
    x = rng.standard_normal(20)
    out.append(("rank_one", np.outer(x, x)))
    out.append(("graded", Q[:20, :20] @ np.diag(10.0 ** -np.arange(20)) @ Q[:20, :20].T))
    return out


@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] for c in _cases()])
def test_sym_eig(lib, name, A):
    n = A.shape[0]
    w, V = _eig(lib, A)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = max(np.abs(A).max(), 1e-300)
    assert np.abs(w - ref).max() <= 1e-12 * scale * max(1, np.sqrt(n)), name
    assert np.all(np.diff(w) <= 0)
    # eigenvectors: orthonormal, and A V = V diag(w)
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12 * max(1, n)
    assert np.abs(A @ V - V * w).max() <= 1e-12 * scale * max(1, n)
    w2, _ = _eig(lib, A, vectors=False)
    assert np.abs(w2 - w).max() <= 1e-13 * scale * max(1, n)
