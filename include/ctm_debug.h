/*
 * ctm_debug.h -- unit-test entry points of the gfx950 CTM library.
 *
 * These expose internal building blocks so that their numerics can be
 * checked in isolation against a CPU reference.  They are not needed to use
 * the library.  All pointers are device pointers; all calls are enqueued on
 * `stream` and synchronise it before returning.
 */
#ifndef CTM_DEBUG_H
#define CTM_DEBUG_H

#include <stdint.h>
#include "ctm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * C = op(A) op(B) on the MFMA GEMM kernel.  A is M x K (K x M if transA),
 * B is K x N (N x K if transB), C is M x N, all row-major and dense.
 * ta: element type of A and B, tc: of C (0 = float64, 1 = float32,
 * 2 = bfloat16); supported pairs: (0,0), (1,1), (1,0), (2,1), (2,0), (2,2), (1,2).
 * Returns CTM_E_INVALID for other pairs or non-positive sizes.
 */
ctm_status ctm_debug_gemm(int32_t ta, int32_t tc, int64_t M, int64_t N, int64_t K,
                          const void* A, int32_t transA, const void* B, int32_t transB,
                          void* C, void* stream);

/*
 * C = op(A) B on the split-K kernel for few columns (1 <= N <= 192): A is
 * M x K (K x M if transA), B is K x N, C is M x N, row-major and dense.
 * (ta, tc) in {(1,1), (1,0), (0,0)}; scratch: device buffer of scratch_bytes
 * for the partial products.
 */
ctm_status ctm_debug_tsgemm(int32_t ta, int32_t tc, int64_t M, int64_t N, int64_t K,
                            const void* A, int32_t transA, const void* B, void* C,
                            void* scratch, int64_t scratch_bytes, void* stream);

/*
 * C = A B for row-major float64 A (n x K), B (K x N), C (n x N) on the
 * solver's small right-multiplication kernel (1 <= K, N <= 64; device
 * buffers).
 */
ctm_status ctm_debug_rmul(int64_t n, int32_t K, int32_t N, const double* A, const double* B, double* C,
                          void* stream);

/*
 * Gram matrix of the solver's Cholesky-QR: G = Y^T Y (k x k row-major) for a
 * row-major n x k float64 Y, 1 <= k <= 64 (X null); or the Rayleigh-Ritz
 * product G = X^T Y of two such blocks, 1 <= k <= 48.  Through part_elems
 * doubles of device scratch `part` (at least k * k).  All buffers on the
 * device.
 */
ctm_status ctm_debug_gram(int64_t n, int32_t k, const double* X, const double* Y, double* G, double* part,
                          int64_t part_elems, void* stream);

/*
 * Shifted Cholesky factor of the solver's Cholesky-QR: R upper triangular
 * (row-major k x k, positive diagonal) with R^T R = G + s I, s = shift_coef
 * * trace(G), for a symmetric k x k row-major G whose upper triangle is read
 * (1 <= k <= 64; all three buffers on the device, work >= 256 bytes).
 * *fail_out is 1 when a pivot was not positive (it is then replaced by
 * 1e-300 trace(G) and the factorisation goes on), else 0.
 */
ctm_status ctm_debug_chol(int32_t k, double shift_coef, const double* G, double* R, void* work,
                          int32_t* fail_out, void* stream);

/*
 * The float32 form of ctm_debug_tsgemm ((ta, tc) = (1, 1)) with a second
 * output: C2 (float64, M x N row-major) receives the same sums as C, written
 * by the same reduction.
 */
ctm_status ctm_debug_tsgemm_dual(int64_t M, int64_t N, int64_t K, const float* A, int32_t transA,
                                 const float* B, float* C, double* C2, void* scratch,
                                 int64_t scratch_bytes, void* stream);

/*
 * C = A Bt^T on the bf16 enlarged-corner kernel: A bf16 M x K row-major, Bt
 * bf16 N x K row-major (both 16-byte aligned, K a multiple of 8), C float32
 * M x N row-major.
 */
ctm_status ctm_debug_corner_bf16(int64_t M, int64_t N, int64_t K, const void* A, const void* Bt,
                                 void* C, void* stream);

/*
 * The same product with Bt first packed into the kernel's fragment layout
 * (the form the CTM moves use for the double layer): `packed` is a device
 * buffer of ctm_debug_corner_bf16_packed_bytes(N, K) bytes that receives
 * the packed Bt.  The result is bitwise equal to ctm_debug_corner_bf16's.
 */
size_t ctm_debug_corner_bf16_packed_bytes(int64_t N, int64_t K);
ctm_status ctm_debug_corner_bf16_packed(int64_t M, int64_t N, int64_t K, const void* A, const void* Bt,
                                        void* packed, void* C, void* stream);

/*
 * One-sided Jacobi SVD of the k x k float64 row-major matrix M (1 <= k <= 192):
 * M W = U diag(S), singular values descending.  U, W: k x k row-major; S: k.
 * work: 3 k^2 doubles.
 */
ctm_status ctm_debug_svd(int32_t k, const double* M, double* U, double* S, double* W,
                         double* work, void* stream);

/*
 * Copies an internal buffer of the last column step of instance 0 to the host
 * (n and chi at the live extent; equal to chi D^2 and chi while the subspace
 * has its full width):
 *   what = 0: enlarged corner Q_(q+1) of row r, float64 n x n row-major,
 *             index = 4 r + q (float32 when the context's precision is not fp64);
 *   what = 1: projector P1 of row r (float64 n x chi), index = r;
 *   what = 2: projector P2^T of row r (float64 n x chi), index = r;
 *   what = 3: solver status of row r {chi_eff, converged, iters, chol_fail as
 *             int32, sigma0, max_resid as float64, Jacobi sweeps of the last
 *             Rayleigh-Ritz step, subspace columns, subspace rows, padding as
 *             int32, discarded weight as float64} (56 bytes), index = r.
 * `bytes` must equal the buffer size.  Syncs.
 */
ctm_status ctm_debug_dump(ctm_ctx ctx, int32_t what, int32_t index, void* host_buf, size_t bytes);

/*
 * Sets the projector subspace width of every instance to `width` (clamped
 * to 1 .. chi + oversample) and re-lays the environment out at the live
 * extent that follows, as the convergence loop does when the kept count
 * changes, and pins it (the convergence loop and moves keep it) until a
 * call with width <= 0; *live_out (may be NULL) receives the live extent of
 * instance 0.  Lets host-only runs (CTM_DRY_RUN) walk the narrowed-extent
 * code paths, and timing runs hold the contractions at a chosen extent.
 */
ctm_status ctm_debug_set_width(ctm_ctx ctx, int32_t width, int32_t* live_out);

/*
 * Rows per GEMM launch of the boundary operator's ring application
 * (ctm_boundary_spectrum): rows <= 0 restores the default, 65535 x 32 (the
 * grid's row-tile dimension at the smallest tile); a smaller cap splits each
 * ring site into more launches (whole groups of rows with the same leading
 * indices, or pieces of one group when the group alone is longer), so that
 * tests reach the split path at small sizes.  Process-wide; the split does
 * not change any output element's summation.
 */
ctm_status ctm_debug_set_ring_rows(int64_t rows);

/*
 * The host eigensolver of the boundary operator's projected Lanczos matrix
 * (Householder tridiagonalisation and the implicit symmetric QR algorithm):
 * A host float64 n x n symmetric (row-major, read only), w host [n] the
 * eigenvalues descending, V (may be NULL) host n x n with the eigenvectors
 * in its columns.  No GPU work.
 */
ctm_status ctm_debug_sym_eig(int32_t n, const double* A, double* w, double* V);

#ifdef __cplusplus
}
#endif

#endif /* CTM_DEBUG_H */
