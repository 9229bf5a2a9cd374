// float64 kernels of the truncated-SVD solver: shifted Cholesky with
// triangular inverse (for Cholesky-QR), one-sided Jacobi SVD of small square
// matrices, residual / cutoff bookkeeping and the warm-start block.
#include "solver.h"
#include "kernels.h"

#include <cmath>

namespace ctmk {

// ---------------------------------------------------------------------------
// Shifted Cholesky and inverse.  One workgroup per problem.  The upper
// triangle of G + sI is held packed in LDS: row i starts at i*k - i*(i-1)/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int upk(int i, int l, int k) { return i * k - (i * (i - 1)) / 2 + (l - i); }

__global__ void __launch_bounds__(256)
chol_shift_inv_kernel(int k, double shift_coef, CPtrSet G, PtrSet Rinv, StatSet st) {
  extern __shared__ double sm[];
  __shared__ double s_tr;
  __shared__ double s_piv;
  const int pb = blockIdx.x;
  const double* g = G.p[pb];
  double* ri = Rinv.p[pb];
  const int tid = threadIdx.x, nt = blockDim.x;

  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += g[i * k + i];
    s_tr = tr;
  }
  __syncthreads();
  const double shift = shift_coef * s_tr;
  for (int i = 0; i < k; ++i)
    for (int l = i + tid; l < k; l += nt) sm[upk(i, l, k)] = g[i * k + l] + (l == i ? shift : 0.0);
  __syncthreads();

  int fail = 0;
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      double dj = sm[upk(j, j, k)];
      double floor_v = (s_tr > 0.0 ? s_tr : 1.0) * 1e-300;
      if (!(dj > floor_v)) { dj = floor_v; s_piv = -sqrt(dj); }
      else s_piv = sqrt(dj);
    }
    __syncthreads();
    double r = s_piv;
    if (r < 0) { fail = 1; r = -r; }
    for (int l = j + tid; l < k; l += nt) sm[upk(j, l, k)] = (l == j) ? r : sm[upk(j, l, k)] / r;
    __syncthreads();
    // trailing update of rows i > j (upper part)
    // 32 threads per row, nt/32 rows at a time
    for (int i = j + 1 + tid / 32; i < k; i += nt / 32) {
      const double rji = sm[upk(j, i, k)];
      for (int l = i + (tid & 31); l < k; l += 32) sm[upk(i, l, k)] -= rji * sm[upk(j, l, k)];
    }
    __syncthreads();
  }
  // inverse of the upper-triangular R, one column per thread:
  // column c: x_c = 1/R_cc; x_i = -(sum_{l=i+1..c} R_il x_l) / R_ii, i < c
  for (int c = tid; c < k; c += nt) {
    for (int i = c + 1; i < k; ++i) ri[i * k + c] = 0.0;
    ri[c * k + c] = 1.0 / sm[upk(c, c, k)];
    for (int i = c - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int l = i + 1; l <= c; ++l) acc += sm[upk(i, l, k)] * ri[l * k + c];
      ri[i * k + c] = -acc / sm[upk(i, i, k)];
    }
  }
  if (fail && tid == 0 && st.p[pb]) st.p[pb]->chol_fail = 1;
}

hipError_t chol_shift_inv(hipStream_t s, int k, double shift_coef, const CPtrSet& G,
                          const PtrSet& Rinv, const StatSet& st, int nprob) {
  size_t lds = (size_t)k * (k + 1) / 2 * sizeof(double);
  if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(G.p[i], (size_t)k * k * 8, "chol G") || !span_ok(Rinv.p[i], (size_t)k * k * 8, "chol Rinv") ||
        !span_ok(st.p[i], sizeof(SolveStatus), "chol status"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)chol_shift_inv_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(chol_shift_inv_kernel, dim3(nprob), dim3(256), lds, s, k, shift_coef, G, Rinv, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of a k x k matrix, one workgroup per
// problem.  Columns are kept column-major in `work` (A then W); each round
// rotates k/2 disjoint column pairs of the round-robin schedule, one pair per
// wave at a time.  A pair (p, q) with Gram entries a = |x_p|^2, b = |x_q|^2,
// g = x_p . x_q is rotated when |g| > eps sqrt(a b); the rotation makes the
// two columns orthogonal (Golub & Van Loan, Sec. 8.6.3 / Hestenes 1958).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// round-robin partner schedule on kk (even) players: player 0 fixed, others
// rotate.  pair j of round r: (pos j, pos kk-1-j) with pos 0 = player 0 and
// pos t>0 = 1 + ((t - 1 + r) mod (kk - 1)).
__device__ __forceinline__ int rr_player(int pos, int r, int kk) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (kk - 1));
}

__global__ void __launch_bounds__(512)
jacobi_svd_kernel(int k, CPtrSet Min, PtrSet Uout, PtrSet Sout, PtrSet Wout, PtrSet work) {
  const int pb = blockIdx.x;
  double* A = work.p[pb];          // column-major k x k, column c at A + c*k
  double* W = A + (size_t)k * k;   // column-major
  const double* M = Min.p[pb];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  __shared__ int s_rot;
  __shared__ double s_norm[256];
  __shared__ int s_perm[256];

  for (int e = tid; e < k * k; e += nt) {
    int r = e / k, c = e % k;
    A[c * k + r] = M[e];
    W[c * k + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kk = (k + 1) & ~1;  // even number of players; player k (if odd) is a dummy
  const double eps = 2.220446049250313e-16 * (double)k;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    int rotated = 0;
    for (int r = 0; r < kk - 1; ++r) {
      for (int j = wave; j < kk / 2; j += nw) {
        int p = rr_player(j, r, kk), q = rr_player(kk - 1 - j, r, kk);
        if (p >= k || q >= k) continue;
        if (p > q) { int t = p; p = q; q = t; }
        double* xp = A + (size_t)p * k;
        double* xq = A + (size_t)q * k;
        double a = 0, b = 0, g = 0;
        for (int i = lane; i < k; i += 64) {
          double u = xp[i], v = xq[i];
          a += u * u; b += v * v; g += u * v;
        }
        a = wsum(a); b = wsum(b); g = wsum(g);
        if (fabs(g) > eps * sqrt(a * b) && fabs(g) > 1e-300) {
          double zeta = (b - a) / (2.0 * g);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int i = lane; i < k; i += 64) {
            double u = xp[i], v = xq[i];
            xp[i] = c * u - sn * v;
            xq[i] = sn * u + c * v;
          }
          double* wp = W + (size_t)p * k;
          double* wq = W + (size_t)q * k;
          for (int i = lane; i < k; i += 64) {
            double u = wp[i], v = wq[i];
            wp[i] = c * u - sn * v;
            wq[i] = sn * u + c * v;
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated && lane == 0) s_rot = 1;
    __syncthreads();
    if (!s_rot) break;
    __syncthreads();
  }
  // singular values = column norms, sorted descending (stable)
  for (int c = wave; c < k; c += nw) {
    double a = 0;
    for (int i = lane; i < k; i += 64) a += A[(size_t)c * k + i] * A[(size_t)c * k + i];
    a = wsum(a);
    if (lane == 0) s_norm[c] = sqrt(a);
  }
  __syncthreads();
  // non-finite norms sort last (key -1), so the ranks form a permutation
  for (int c = tid; c < k; c += nt) {
    double v = isfinite(s_norm[c]) ? s_norm[c] : -1.0;
    int rank = 0;
    for (int o = 0; o < k; ++o) {
      double w = isfinite(s_norm[o]) ? s_norm[o] : -1.0;
      rank += (w > v) || (w == v && o < c);
    }
    s_perm[rank] = c;
  }
  __syncthreads();
  double* U = Uout.p[pb];
  double* S = Sout.p[pb];
  double* Wo = Wout.p[pb];
  for (int e = tid; e < k * k; e += nt) {
    int r = e / k, j = e % k;
    int c = s_perm[j];
    double sv = s_norm[c];
    U[e] = sv > 0 ? A[(size_t)c * k + r] / sv : 0.0;
    Wo[e] = W[(size_t)c * k + r];
  }
  for (int j = tid; j < k; j += nt) S[j] = s_norm[s_perm[j]];
}

hipError_t jacobi_svd(hipStream_t s, int k, const CPtrSet& M, const PtrSet& U, const PtrSet& S,
                      const PtrSet& W, const PtrSet& work, int nprob) {
  if (k > 256) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(M.p[i], (size_t)k * k * 8, "jacobi M") || !span_ok(U.p[i], (size_t)k * k * 8, "jacobi U") ||
        !span_ok(S.p[i], (size_t)k * 8, "jacobi S") || !span_ok(W.p[i], (size_t)k * k * 8, "jacobi W") ||
        !span_ok(work.p[i], (size_t)2 * k * k * 8, "jacobi work"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(nprob), dim3(512), 0, s, k, M, U, S, W, work);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residuals and cutoff
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
residual_kernel(int64_t n, int k, int chi, double cutoff, double tol, CPtrSet Z, CPtrSet V,
                CPtrSet S, StatSet st) {
  const int pb = blockIdx.x;
  const double* z = Z.p[pb];
  const double* v = V.p[pb];
  const double* sv = S.p[pb];
  __shared__ double s_res[256];
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double sc = sv[c], acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d = z[i * k + c] - sc * v[i * k + c];
      acc += d * d;
    }
    s_res[c] = sqrt(acc);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    SolveStatus* o = st.p[pb];
    double s0 = sv[0];
    int keep = 0;
    if (s0 > 0)
      for (int c = 0; c < k && c < chi; ++c)
        if (sv[c] > cutoff * s0) keep = c + 1;
    double mr = 0.0;
    for (int c = 0; c < keep; ++c) mr = fmax(mr, s_res[c]);
    mr = s0 > 0 ? mr / s0 : 0.0;
    o->chi_eff = keep;
    o->sigma0 = s0;
    o->max_resid = mr;
    o->converged = (mr <= tol) ? 1 : 0;
    o->iters += 1;
  }
}

hipError_t residual_status(hipStream_t s, int64_t n, int k, int chi, double cutoff, double tol,
                           const CPtrSet& Z, const CPtrSet& V, const CPtrSet& S,
                           const StatSet& st, int nprob) {
  if (k > 256) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(Z.p[i], (size_t)n * k * 8, "resid Z") || !span_ok(V.p[i], (size_t)n * k * 8, "resid V") ||
        !span_ok(S.p[i], (size_t)k * 8, "resid S") || !span_ok(st.p[i], sizeof(SolveStatus), "resid st"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(residual_kernel, dim3(nprob), dim3(256), 0, s, n, k, chi, cutoff, tol, Z, V, S, st);
  return hipGetLastError();
}

__global__ void scale_kept_kernel(int k, int chi, CPtrSet W, CPtrSet S, PtrSet Wp, StatSet st) {
  const int pb = blockIdx.x;
  const int keep = st.p[pb]->chi_eff;
  const double* w = W.p[pb];
  const double* sv = S.p[pb];
  double* o = Wp.p[pb];
  for (int e = threadIdx.x; e < k * chi; e += blockDim.x) {
    int j = e / chi, c = e % chi;
    double wv = w ? w[j * k + c] : (j == c ? 1.0 : 0.0);
    o[e] = (c < keep && c < k) ? wv / sqrt(sv[c]) : 0.0;
  }
}

hipError_t scale_kept(hipStream_t s, int k, int chi, const CPtrSet& W, const CPtrSet& S,
                      const PtrSet& Wp, const StatSet& st, int nprob) {
  for (int i = 0; i < nprob; ++i)
    if ((W.p[i] && !span_ok(W.p[i], (size_t)k * k * 8, "scale W")) || !span_ok(S.p[i], (size_t)k * 8, "scale S") ||
        !span_ok(Wp.p[i], (size_t)k * chi * 8, "scale Wp") || !span_ok(st.p[i], sizeof(SolveStatus), "scale st"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(scale_kept_kernel, dim3(nprob), dim3(256), 0, s, k, chi, W, S, Wp, st);
  return hipGetLastError();
}

__device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void warm_start_kernel(int64_t n, int k, PtrSet V0, CPtrSet Vprev, StatSet prev, uint64_t seed) {
  const int pb = blockIdx.y;
  double* v0 = V0.p[pb];
  const double* vp = Vprev.p[pb];
  int keep = (prev.p[pb] && vp) ? prev.p[pb]->chi_eff : 0;
  if (keep > k) keep = k;
  const uint64_t sd = seed + 0x1000193ull * (uint64_t)pb * (uint64_t)n * (uint64_t)k * 2ull;
  const int64_t tot = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int c = (int)(e % k);
    if (c < keep) { v0[e] = vp[e]; continue; }
    uint64_t a = sm64(sd + 2ull * (uint64_t)e), b = sm64(sd + 2ull * (uint64_t)e + 1ull);
    double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    v0[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

hipError_t warm_start(hipStream_t s, int64_t n, int k, const PtrSet& V0, const CPtrSet& Vprev,
                      const StatSet& prev, uint64_t seed, int nprob) {
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(V0.p[i], (size_t)n * k * 8, "warm V0") ||
        (Vprev.p[i] && !span_ok(Vprev.p[i], (size_t)n * k * 8, "warm Vprev")) ||
        (prev.p[i] && !span_ok(prev.p[i], sizeof(SolveStatus), "warm prev")))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n * k + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(warm_start_kernel, dim3((unsigned)blocks, nprob), dim3(256), 0, s, n, k, V0, Vprev, prev, seed);
  return hipGetLastError();
}

__global__ void reset_status_kernel(StatSet st) {
  SolveStatus* o = st.p[threadIdx.x];
  o->iters = 0;
  o->converged = 0;
  o->chol_fail = 0;
}

hipError_t reset_status(hipStream_t s, const StatSet& st, int nprob) {
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(st.p[i], sizeof(SolveStatus), "reset st")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(reset_status_kernel, dim3(1), dim3(nprob), 0, s, st);
  return hipGetLastError();
}

}  // namespace ctmk
