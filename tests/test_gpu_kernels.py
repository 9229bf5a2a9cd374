"""Kernel-level checks through the unit-test entry points of include/ctm_debug.h:
the MFMA GEMM (float64, float32, bfloat16 operand layouts) and the split-K
GEMM for few columns against NumPy, and the one-sided Jacobi SVD against
LAPACK."""
import ctypes
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1711_04798_amd import binding
    lib = binding.load()
    lib.ctm_debug_gemm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.ctm_debug_gemm.restype = ctypes.c_int
    lib.ctm_debug_tsgemm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.ctm_debug_tsgemm.restype = ctypes.c_int
    lib.ctm_debug_tsgemm_dual.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p, ctypes.c_int32] + \
        [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_void_p]
    lib.ctm_debug_tsgemm_dual.restype = ctypes.c_int
    lib.ctm_debug_rmul.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32] + [ctypes.c_void_p] * 4
    lib.ctm_debug_rmul.restype = ctypes.c_int
    lib.ctm_debug_chol.argtypes = [ctypes.c_int32, ctypes.c_double] + [ctypes.c_void_p] * 5
    lib.ctm_debug_chol.restype = ctypes.c_int
    lib.ctm_debug_gram.argtypes = [ctypes.c_int64, ctypes.c_int32] + [ctypes.c_void_p] * 4 + \
        [ctypes.c_int64, ctypes.c_void_p]
    lib.ctm_debug_gram.restype = ctypes.c_int
    lib.ctm_debug_corner_bf16.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p] * 4
    lib.ctm_debug_corner_bf16.restype = ctypes.c_int
    lib.ctm_debug_corner_bf16_packed.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p] * 5
    lib.ctm_debug_corner_bf16_packed.restype = ctypes.c_int
    lib.ctm_debug_corner_bf16_packed_bytes.argtypes = [ctypes.c_int64] * 2
    lib.ctm_debug_corner_bf16_packed_bytes.restype = ctypes.c_size_t
    lib.ctm_debug_svd.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 6
    lib.ctm_debug_svd.restype = ctypes.c_int
    return lib


TT = {0: "float64", 1: "float32", 2: "bfloat16"}


@pytest.mark.parametrize("ta,tc", [(0, 0), (1, 1), (2, 1), (2, 0)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (67, 45, 33), (130, 97, 200)])
@pytest.mark.parametrize("transA,transB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm(gpu, ta, tc, M, N, K, transA, transB):
    import torch
    lib = _lib()
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if transA else (M, K))
    B = rng.standard_normal((N, K) if transB else (K, N))
    dt = getattr(torch, TT[ta])
    At = torch.tensor(A, dtype=torch.float64).to(dt).cuda().contiguous()
    Bt = torch.tensor(B, dtype=torch.float64).to(dt).cuda().contiguous()
    Ct = torch.zeros((M, N), dtype=getattr(torch, TT[tc]), device="cuda")
    print("gemm case", ta, tc, M, N, K, transA, transB, flush=True)
    st = lib.ctm_debug_gemm(ta, tc, M, N, K, At.data_ptr(), transA, Bt.data_ptr(), transB, Ct.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    # reference from the operands as rounded to the input type, in float64
    Ar = At.to(torch.float64).cpu().numpy()
    Br = Bt.to(torch.float64).cpu().numpy()
    ref = (Ar.T if transA else Ar) @ (Br.T if transB else Br)
    got = Ct.to(torch.float64).cpu().numpy()
    scale = np.abs(Ar).max() * np.abs(Br).max() * K
    tol = {0: 1e-14, 1: 2e-6, 2: 2e-6}[ta] * scale
    if tc == 2:
        tol = max(tol, 1e-2 * np.abs(ref).max())
    assert np.abs(got - ref).max() <= tol + 1e-300


@pytest.mark.parametrize("n,k,part", [(1728, 48, 64), (5184, 64, 64), (100, 17, 64), (4, 1, 64), (65, 64, 64),
                                        (1, 3, 64), (1728, 48, 1), (5184, 33, 3), (37, 16, 64)])
def test_gram_small(gpu, n, k, part):
    """Gram matrix of a tall block against numpy: chunks of 64 rows (and of
    more rows per wave when the scratch holds fewer chunks: part = partial
    sums the scratch holds), ragged row and column blocks, k from 1 to 64;
    the result is exactly symmetric.  For k <= 48 also the cross form X^T Y
    of the Rayleigh-Ritz step."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(n + 3 * k)
    Y = rng.standard_normal((n, k))
    Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
    Gt = torch.full((k, k), 7.0, dtype=torch.float64, device="cuda")
    P = torch.full((part * k * k,), float("nan"), dtype=torch.float64, device="cuda")
    print("gram case", n, k, part, flush=True)
    st = lib.ctm_debug_gram(n, k, None, Yt.data_ptr(), Gt.data_ptr(), P.data_ptr(), P.numel(),
                            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    G = Gt.cpu().numpy()
    ref = Y.T @ Y
    assert np.abs(G - ref).max() <= 4 * n * 2.0 ** -53 * np.abs(Y).max() ** 2
    assert np.array_equal(G, G.T)
    if k <= 48:
        # the cross form X^T Y (every tile formed)
        X = rng.standard_normal((n, k))
        Xt = torch.tensor(X, dtype=torch.float64, device="cuda")
        Gt.fill_(7.0)
        P.fill_(float("nan"))
        st = lib.ctm_debug_gram(n, k, Xt.data_ptr(), Yt.data_ptr(), Gt.data_ptr(), P.data_ptr(), P.numel(),
                                torch.cuda.current_stream().cuda_stream)
        assert st == 0
        ref = X.T @ Y
        assert np.abs(Gt.cpu().numpy() - ref).max() <= 4 * n * 2.0 ** -53 * np.abs(X).max() * np.abs(Y).max()


@pytest.mark.parametrize("n,K,N", [(1728, 48, 48), (5184, 64, 64), (100, 17, 33), (7, 1, 1), (65, 64, 5),
                                   (16, 3, 64)])
def test_rmul_small(gpu, n, K, N):
    """The solver's right-multiplication by a small matrix against numpy:
    ragged row, K and column blocks; in place (C = A) bit for bit equal to
    the out-of-place result."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(n + 5 * K + 11 * N)
    A = rng.standard_normal((n, K))
    B = rng.standard_normal((K, N))
    At = torch.tensor(A, dtype=torch.float64, device="cuda")
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda")
    Ct = torch.full((n, N), 7.0, dtype=torch.float64, device="cuda")
    print("rmul case", n, K, N, flush=True)
    st = lib.ctm_debug_rmul(n, K, N, At.data_ptr(), Bt.data_ptr(), Ct.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    assert np.abs(Ct.cpu().numpy() - A @ B).max() <= 4 * K * 2.0 ** -53 * np.abs(A).max() * np.abs(B).max()
    if K == N:
        # in place: C = A
        st = lib.ctm_debug_rmul(n, K, N, At.data_ptr(), Bt.data_ptr(), At.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
        assert st == 0
        assert np.array_equal(At.cpu().numpy(), Ct.cpu().numpy())


def _chol(lib, G, coef):
    import torch
    k = G.shape[0]
    Gt = torch.tensor(G, dtype=torch.float64, device="cuda")
    Rt = torch.full((k, k), 7.0, dtype=torch.float64, device="cuda")
    work = torch.zeros(256, dtype=torch.uint8, device="cuda")
    fail = ctypes.c_int32(-1)
    st = lib.ctm_debug_chol(k, coef, Gt.data_ptr(), Rt.data_ptr(), work.data_ptr(), ctypes.byref(fail),
                            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    return Rt.cpu().numpy(), fail.value


@pytest.mark.parametrize("k", [1, 3, 4, 5, 17, 48, 63, 64])
def test_chol_factor(gpu, k):
    """Shifted Cholesky of the Cholesky-QR step against numpy's factor: a
    well-conditioned Gram matrix without shift (only the upper triangle is
    read: the strict lower one holds NaN), and a rank-deficient Gram matrix
    with the first pass's shift, where R^T R must reproduce G + sI."""
    lib = _lib()
    rng = np.random.default_rng(100 + k)
    print("chol case", k, flush=True)
    Y = rng.standard_normal((300, k))
    G = Y.T @ Y
    Gn = G.copy()
    Gn[np.tril_indices(k, -1)] = np.nan
    R, fail = _chol(lib, Gn, 0.0)
    assert fail == 0
    Rnp = np.linalg.cholesky(np.triu(G) + np.triu(G, 1).T).T
    assert np.array_equal(R, np.triu(R)) and (np.diag(R) > 0).all()
    assert np.abs(R - Rnp).max() <= 1e-13 * np.abs(Rnp).max()
    # rank k // 2 + 1: the shift keeps every pivot positive
    Y2 = rng.standard_normal((300, k // 2 + 1)) @ rng.standard_normal((k // 2 + 1, k))
    G2 = Y2.T @ Y2
    G2 = np.triu(G2) + np.triu(G2, 1).T
    u = 2.0 ** -53
    coef = 11.0 * (300 * k + k * (k + 1)) * u
    R2, fail2 = _chol(lib, G2, coef)
    assert fail2 == 0
    S = G2 + coef * np.trace(G2) * np.eye(k)
    assert np.abs(R2.T @ R2 - S).max() <= 64 * k * u * np.trace(G2)


def test_chol_reports_failure(gpu):
    """A negative pivot sets the failure flag and the factor stays finite."""
    lib = _lib()
    k = 40
    G = np.eye(k)
    G[7, 7] = -1.0
    R, fail = _chol(lib, G, 0.0)
    assert fail == 1
    assert np.isfinite(R).all()


TS64_RUN = r"""
import ctypes, sys
import numpy as np
import torch
sys.path.insert(0, %(root)r)
from paper_1711_04798_amd import binding
lib = binding.load()
lib.ctm_debug_tsgemm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p]
worst = 0.0
for M, N, K, transA in ((1728, 48, 1728, 0), (1728, 48, 1728, 1), (68, 45, 1036, 0), (68, 45, 1036, 1),
                        (1000, 64, 772, 1)):
    rng = np.random.default_rng(M + N + K + transA)
    A = rng.standard_normal((K, M) if transA else (M, K))
    B = rng.standard_normal((K, N))
    At = torch.tensor(A, dtype=torch.float32, device="cuda")
    Bt = torch.tensor(B, dtype=torch.float32, device="cuda")
    Ct = torch.full((M, N), 7.0, dtype=torch.float32, device="cuda")
    scratch = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    assert lib.ctm_debug_tsgemm(1, 1, M, N, K, At.data_ptr(), transA, Bt.data_ptr(), Ct.data_ptr(),
                                scratch.data_ptr(), scratch.numel(), torch.cuda.current_stream().cuda_stream) == 0
    Ar = At.double().cpu().numpy(); Br = Bt.double().cpu().numpy()
    ref = (Ar.T if transA else Ar) @ Br
    err = np.abs(Ct.double().cpu().numpy() - ref).max() / (np.abs(Ar).max() * np.abs(Br).max() * K)
    worst = max(worst, err)
print(worst)
"""


def test_tsgemm_64_rows(gpu):
    """The streaming form with 64 rows per wave (CTM_TS_ROWS=64 and
    CTM_TS_ROWS_M=64: four row blocks, m-fast A in 16-byte loads) against
    numpy, both layouts of A, ragged K blocks (the default runs 32 rows)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    env.update({"CTM_TS_ROWS": "64", "CTM_TS_ROWS_M": "64"})
    print("tsgemm 64-row run", flush=True)
    r = subprocess.run([sys.executable, "-c", TS64_RUN % {"root": root}], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert float(r.stdout.strip().splitlines()[-1]) <= 2e-6


@pytest.mark.parametrize("M,N,K,transA", [(1728, 48, 1728, 0), (1728, 48, 1728, 1), (67, 45, 1030, 0),
                                          (700, 192, 2500, 1), (4, 3, 8, 0)])
def test_tsgemm_dual_output(gpu, M, N, K, transA):
    """The float32 product with a float64 second output: the first output
    within the float32 bound of the float64 product, the second equal to it
    bit for bit after widening (both forms: N <= 64 streams, N = 192 takes
    the tiled form)."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(3 * M + N + K)
    A = rng.standard_normal((K, M) if transA else (M, K))
    B = rng.standard_normal((K, N))
    At = torch.tensor(A, dtype=torch.float32, device="cuda")
    Bt = torch.tensor(B, dtype=torch.float32, device="cuda")
    Ct = torch.full((M, N), 7.0, dtype=torch.float32, device="cuda")
    C2 = torch.full((M, N), 7.0, dtype=torch.float64, device="cuda")
    scratch = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    print("tsgemm dual case", M, N, K, transA, flush=True)
    st = lib.ctm_debug_tsgemm_dual(M, N, K, At.data_ptr(), transA, Bt.data_ptr(), Ct.data_ptr(), C2.data_ptr(),
                                   scratch.data_ptr(), scratch.numel(), torch.cuda.current_stream().cuda_stream)
    assert st == 0
    Ar = At.to(torch.float64).cpu().numpy()
    Br = Bt.to(torch.float64).cpu().numpy()
    ref = (Ar.T if transA else Ar) @ Br
    got = Ct.to(torch.float64).cpu().numpy()
    assert np.abs(got - ref).max() <= 2e-6 * np.abs(Ar).max() * np.abs(Br).max() * K
    assert np.array_equal(C2.cpu().numpy(), got)


@pytest.mark.parametrize("ta,tc", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 16, 32), (67, 45, 1030), (5184, 50, 5184), (700, 192, 2500),
                                   (144, 144, 5184), (130, 1, 4097), (68, 45, 1036), (1000, 64, 772), (4, 3, 8)])
@pytest.mark.parametrize("transA", [0, 1])
def test_tsgemm(gpu, ta, tc, M, N, K, transA):
    """Split-K product for few columns: several K chunks, ragged row tiles
    (M not a multiple of 64), N from 1 to 192, both layouts of A.  float32
    with k-fast A, M, K and the leading dimension multiples of 4 and N <= 64
    takes the register-streaming form (ragged 16-wide K blocks: K = 1036, 772,
    8)."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(M + 7 * N + 13 * K)
    A = rng.standard_normal((K, M) if transA else (M, K))
    B = rng.standard_normal((K, N))
    dt = getattr(torch, TT[ta])
    At = torch.tensor(A, dtype=dt, device="cuda")
    Bt = torch.tensor(B, dtype=dt, device="cuda")
    Ct = torch.full((M, N), 7.0, dtype=getattr(torch, TT[tc]), device="cuda")
    scratch = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    print("tsgemm case", ta, tc, M, N, K, transA, flush=True)
    st = lib.ctm_debug_tsgemm(ta, tc, M, N, K, At.data_ptr(), transA, Bt.data_ptr(), Ct.data_ptr(),
                              scratch.data_ptr(), scratch.numel(), torch.cuda.current_stream().cuda_stream)
    assert st == 0
    Ar = At.to(torch.float64).cpu().numpy()
    Br = Bt.to(torch.float64).cpu().numpy()
    ref = (Ar.T if transA else Ar) @ Br
    got = Ct.to(torch.float64).cpu().numpy()
    scale = np.abs(Ar).max() * np.abs(Br).max() * K
    tol = {0: 1e-14, 1: 2e-6}[ta] * scale
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("M,N,K", [(16, 16, 8), (256, 144, 32), (300, 150, 1296), (20736, 1296, 1296),
                                   (1000, 81, 264), (513, 290, 64)])
def test_corner_bf16(gpu, M, N, K):
    """The bf16 double-layer kernel: full tiles, ragged M and N, K with and
    without a partial last step (K = D^4 = 1296 for D = 6)."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(M + N + K)
    A = torch.tensor(rng.standard_normal((M, K)), dtype=torch.bfloat16, device="cuda")
    Bt = torch.tensor(rng.standard_normal((N, K)), dtype=torch.bfloat16, device="cuda")
    C = torch.full((M, N), 3.0, dtype=torch.float32, device="cuda")
    print("corner_bf16 case", M, N, K, flush=True)
    st = lib.ctm_debug_corner_bf16(M, N, K, A.data_ptr(), Bt.data_ptr(), C.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert st == 0
    rows = np.unique(np.concatenate([np.arange(min(M, 64)), rng.integers(0, M, 64), [M - 1]]))
    Ar = A.to(torch.float64).cpu().numpy()[rows]
    Br = Bt.to(torch.float64).cpu().numpy()
    ref = Ar @ Br.T
    got = C.to(torch.float64).cpu().numpy()[rows]
    # fp32 accumulation of exact bf16 products
    assert np.abs(got - ref).max() <= 1e-5 * np.sqrt(K) * np.abs(ref).max()


@pytest.mark.parametrize("M,N,K", [(20736, 1296, 1296), (2304, 1296, 1296), (300, 200, 296), (7, 5, 8),
                                   (256, 144, 32), (513, 289, 1040)])
def test_corner_bf16_packed(gpu, M, N, K):
    """The double-layer kernel with B in the packed fragment layout (the form
    the moves use) against the row-major form, bitwise: the same K order and
    the same MFMA sequence; full and ragged tiles, a partial last K step."""
    import torch
    lib = _lib()
    rng = np.random.default_rng(M + 7 * N + K)
    A = torch.tensor(rng.standard_normal((M, K)), dtype=torch.bfloat16, device="cuda")
    Bt = torch.tensor(rng.standard_normal((N, K)), dtype=torch.bfloat16, device="cuda")
    C0 = torch.full((M, N), 3.0, dtype=torch.float32, device="cuda")
    C1 = torch.full((M, N), -3.0, dtype=torch.float32, device="cuda")
    nb = lib.ctm_debug_corner_bf16_packed_bytes(N, K)
    assert nb == ((K + 31) // 32) * ((N + 143) // 144 * 9) * 1024
    P = torch.full((nb // 2,), 7.0, dtype=torch.bfloat16, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    print("corner_bf16 packed case", M, N, K, flush=True)
    assert lib.ctm_debug_corner_bf16(M, N, K, A.data_ptr(), Bt.data_ptr(), C0.data_ptr(), stream) == 0
    assert lib.ctm_debug_corner_bf16_packed(M, N, K, A.data_ptr(), Bt.data_ptr(), P.data_ptr(), C1.data_ptr(),
                                            stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(C0, C1)
    # the packed layout itself: block (kb, rb), lane l holds Bt[16 rb + l % 16][32 kb + 8 (l / 16) + j]
    rbp = (N + 143) // 144 * 9
    pk = P.view(-1, rbp, 64, 8).to(torch.float32).cpu().numpy()
    Bn = Bt.to(torch.float32).cpu().numpy()
    for kb, rb, l in [(0, 0, 0), (0, 0, 17), (K // 32, (N - 1) // 16, 63), ((K - 1) // 32, rbp - 1, 5)]:
        for j in range(8):
            row, k = 16 * rb + l % 16, 32 * kb + 8 * (l // 16) + j
            want = Bn[row, k] if row < N and k < K else 0.0
            if kb < pk.shape[0]:
                assert pk[kb, rb, l, j] == want


@pytest.mark.parametrize("k", [1, 2, 7, 16, 33, 80, 144, 160])
def test_jacobi_svd(gpu, k):
    import torch
    lib = _lib()
    rng = np.random.default_rng(k)
    # graded spectrum over ~12 decades, as in the projector problem
    U0, _ = np.linalg.qr(rng.standard_normal((k, k)))
    V0, _ = np.linalg.qr(rng.standard_normal((k, k)))
    s0 = 10.0 ** (-12.0 * np.arange(k) / max(k - 1, 1))
    M = (U0 * s0) @ V0.T
    Mt = torch.tensor(M, device="cuda")
    U = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    W = torch.zeros_like(U)
    S = torch.zeros(k, dtype=torch.float64, device="cuda")
    work = torch.zeros(3 * k * k, dtype=torch.float64, device="cuda")
    print("svd case", k, flush=True)
    st = lib.ctm_debug_svd(k, Mt.data_ptr(), U.data_ptr(), S.data_ptr(), W.data_ptr(), work.data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
    assert st == 0
    S, U, W = S.cpu().numpy(), U.cpu().numpy(), W.cpu().numpy()
    sref = np.linalg.svd(M, compute_uv=False)
    # one-sided Jacobi has high relative accuracy on graded matrices
    assert np.all(np.abs(S - sref) <= 1e-10 * sref + 1e-15 * sref[0])
    # accumulated rotations: O(k * sweeps * u) loss of orthogonality
    assert np.abs(W.T @ W - np.eye(k)).max() < 4e-15 * max(k, 8)
    assert np.abs(M @ W - U * S).max() < 4e-15 * max(k, 8) * sref[0]


PACKED_RUN = r'''
import hashlib, json, sys
sys.path.insert(0, %(root)r)
sys.path.insert(0, %(tests)r)
import numpy as np
import synth
from paper_1711_04798_amd import CTM
out = {}
for D, chi in ((6, 144), (4, 64), (6, 36)):
    tens = synth.cell_tensors(0, 8, D, 2)
    g = CTM([tens], Lx=2, Ly=2, pattern=[0, 1, 1, 0], chi=chi, prec="bf16", max_iters=2, resid_tol=0.0,
            cutoff=1e-7)
    g.sweep(2)
    sp = g.spectra()
    out["%%d_%%d" %% (D, chi)] = [hashlib.sha1(sp.tobytes()).hexdigest(), g.norm()]
    g.close()
print(json.dumps(out))
'''


def test_packed_layouts_bitwise(gpu):
    """The moves with the double layer and the intermediate Y in the packed
    fragment layouts (the default, and with 128, 192 and 256 rows per
    work-group forced), with only the double layer packed, and with both
    row-major give bitwise-equal spectra and norms after two bf16 sweeps: the benchmark workload (d = 8, D = 6, chi = 144, live extent
    below chi), D = 4 (K = 256, whole K steps) and chi = 36 (a live extent
    that is not a multiple of 8 sends the second product to the generic GEMM,
    so only the double layer is packed)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = PACKED_RUN % {"root": root, "tests": os.path.join(root, "tests")}
    res = {}
    for name, extra in (("packed", {}), ("b_only", {"CTM_CORNER_A": "rowmajor"}),
                        ("rowmajor", {"CTM_CORNER_B": "rowmajor"}), ("rows128", {"CTM_CORNER_ROWS": "128"}),
                        ("rows192", {"CTM_CORNER_ROWS": "192"}), ("rows256", {"CTM_CORNER_ROWS": "256"})):
        env = dict(os.environ)
        env.update(extra)
        print("packed layouts run", name, flush=True)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        res[name] = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    for name in res:
        assert res[name] == res["rowmajor"], name
