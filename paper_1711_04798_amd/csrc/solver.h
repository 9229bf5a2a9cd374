// Internal float64 solver kernels for the truncated SVD of the half-system
// product (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ctmk {

// Per-problem solver status, kept in device memory.
struct SolveStatus {
  int32_t chi_eff;     // kept singular values (sigma_i > cutoff * sigma_0, i < chi)
  int32_t converged;   // every kept residual below tol * sigma_0
  int32_t iters;       // iterations done
  int32_t chol_fail;   // a Cholesky pivot was not positive
  double sigma0;       // largest singular value
  double max_resid;    // largest kept residual / sigma_0
  int32_t jsweeps;     // Jacobi sweeps of the last Rayleigh-Ritz step
  int32_t kcols;       // columns of the subspace this status belongs to
  int32_t nrows;       // rows (cut dimension) of that subspace
  int32_t pad_;
  double discarded;    // sum_{i >= chi_eff} s_i^2 / sum_i s_i^2 over the k computed values
};

constexpr int MAXP = 32;  // problems per small-kernel launch

struct PtrSet {
  double* p[MAXP];
};
struct CPtrSet {
  const double* p[MAXP];
};
struct StatSet {
  SolveStatus* p[MAXP];
};

// For each problem: R^T R = G + s I with s = shift_coef * trace(G) (G is k x k,
// row-major), written back as R^{-1} (upper triangular, row-major k x k) into
// Rinv.  G is left unchanged.
// With want_inverse false (k <= 64 only) R itself is written instead.
hipError_t chol_shift_inv(hipStream_t s, int k, double shift_coef, const CPtrSet& G,
                          const PtrSet& Rinv, const StatSet& st, int nprob, bool want_inverse = true);

// Largest k of the four-wave Cholesky (R alone) and of trsm_rows.
constexpr int CHOL_WAVE_MAX = 64;

// G = Y^T Y (k x k row-major) for each problem's n x k row-major float64 Y,
// k <= 64.  part: device scratch of part_elems doubles for the per-chunk
// partial sums (at least k * k * nprob; more allows shorter chunks).
hipError_t gram_small(hipStream_t s, int64_t n, int k, const CPtrSet& Y, const PtrSet& G, int nprob, double* part,
                      int64_t part_elems);
// C = A B for row-major float64 A (n x K), B (K x N), C (n x N) per problem,
// K, N <= 64, on the float64 MFMA with fragments loaded straight from memory;
// C may be A (in place, N == K).
hipError_t rmul_small(hipStream_t s, int64_t n, int K, int N, const CPtrSet& A, const CPtrSet& B, const PtrSet& C,
                      int nprob);
// G = X^T Y for two n x k row-major float64 blocks, k <= 48, the same way.
hipError_t gram_cross_small(hipStream_t s, int64_t n, int k, const CPtrSet& X, const CPtrSet& Y, const PtrSet& G,
                            int nprob, double* part, int64_t part_elems);

// Y <- Y R^{-1} in place, Y n x k row-major, R k x k upper triangular
// row-major (k <= 64), for each problem; with Y32, the result rounded to
// float32 is also written there (n x k row-major); with Yin, Y <- Yin R^{-1}
// (Yin read, Y written).
hipError_t trsm_rows(hipStream_t s, int64_t n, int k, const PtrSet& Y, const CPtrSet& R, int nprob,
                     const PtrSet* Y32 = nullptr, const CPtrSet* Yin = nullptr);

// One-sided Jacobi SVD of the k x k row-major matrix M (k <= 192): M W = U S with singular
// values in descending order.  U, W row-major k x k; S length k.  Columns of U
// with a zero singular value are zero.  The working columns live in LDS when
// they fit; otherwise `work` holds them: 2 k*k16 doubles per problem (k*k16
// when only the singular values are wanted), k16 = k rounded up to a multiple
// of 16.  When only the singular values are wanted, U and W are untouched and
// rows and columns that are exactly zero are dropped before the sweeps.
// With transpose_in the rotations act on the columns of M^T (the rows of M):
// M^T W = U S, i.e. M = W S U^T.  Columns whose norm stays below noise_rel
// (at least 4 u) times the largest are left unrotated; their singular values
// and vectors are then only bounds.  A pair of columns is rotated while the
// cosine between them exceeds max(k u, rot_rel): rot_rel = 0 runs to full
// float64 orthogonality, a larger value stops once the columns are that
// close to orthogonal (the rotations themselves stay exactly orthogonal).
hipError_t jacobi_svd(hipStream_t s, int k, const CPtrSet& M, const PtrSet& U,
                      const PtrSet& S, const PtrSet& W, const PtrSet& work, int nprob,
                      bool want_vectors = true, bool transpose_in = false,
                      const StatSet* st = nullptr, double noise_rel = 0.0, double rot_rel = 0.0);

// Residuals r_i = ||Z_i - S_i V_i|| of the columns of the n x k row-major
// blocks; sets chi_eff (from S, chi, cutoff), converged (tol), sigma0,
// max_resid and increments iters.  scratch: at least 64 k nprob doubles for
// full parallelism (fewer row chunks otherwise).  With Z.p[0] null the
// residuals are not formed: max_resid = -1, converged = 0, the rest as above.
hipError_t residual_status(hipStream_t s, int64_t n, int k, int chi, double cutoff, double tol,
                           const CPtrSet& Z, const CPtrSet& V, const CPtrSet& S,
                           const StatSet& st, int nprob, double* scratch, int64_t scratch_elems);

// Wp[j][c] = W[j][c] * (c < chi_eff ? S_c^{-1/2} : 0) for c < chi (k x chi out);
// a null W stands for the identity.
hipError_t scale_kept(hipStream_t s, int k, int chi, const CPtrSet& W, const CPtrSet& S,
                      const PtrSet& Wp, const StatSet& st, int nprob);

// V0 (n x k) = the chi_eff kept columns of Vprev (stored prev->nrows x
// prev->kcols, buffer n_cap x kmax; rows past prev->nrows read as zero: the
// kept vectors have no component along cut directions that were not live
// when they were found), then counter-based normals.  keep = 0 if prev is
// null or holds no previous solve.
hipError_t warm_start(hipStream_t s, int64_t n, int64_t n_cap, int k, int kmax, const PtrSet& V0,
                      const CPtrSet& Vprev, const StatSet& prev, uint64_t seed, int nprob);

// Resets the iteration counters of the statuses.
hipError_t reset_status(hipStream_t s, const StatSet& st, int nprob);

}  // namespace ctmk
