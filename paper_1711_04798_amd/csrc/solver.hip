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

__global__ void __launch_bounds__(1024)
chol_shift_inv_kernel(int k, double shift_coef, CPtrSet G, PtrSet Rinv, StatSet st) {
  extern __shared__ double sm[];
  __shared__ double s_tr;
  const int pb = blockIdx.x;
  const double* g = G.p[pb];
  double* ri = Rinv.p[pb];
  const int tid = threadIdx.x, nt = blockDim.x;

  __shared__ double s_red[16];
  double tr = 0.0;
  for (int i = tid; i < k; i += nt) tr += g[i * k + i];
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = tr;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < (nt >> 6); ++w) t += s_red[w];
    s_tr = t;
  }
  __syncthreads();
  const double shift = shift_coef * s_tr;
  for (int e = tid; e < k * k; e += nt) {
    int i = e / k, l = e - i * k;
    if (l >= i) sm[upk(i, l, k)] = g[e] + (l == i ? shift : 0.0);
  }
  __syncthreads();

  // Right-looking Cholesky, two barriers per column.  Every thread forms the
  // pivot itself; pivots and their reciprocals live in s_diag / s_rinv, so
  // the diagonal entry read at the start of step j is never overwritten.
  __shared__ double s_diag[256], s_rinv[256];
  int fail = 0;
  const double floor_v = (s_tr > 0.0 ? s_tr : 1.0) * 1e-300;
  for (int j = 0; j < k; ++j) {
    double dj = sm[upk(j, j, k)];
    if (!(dj > floor_v)) { dj = floor_v; fail = 1; }
    const double r = sqrt(dj), rinv = 1.0 / r;
    if (tid == 0) { s_diag[j] = r; s_rinv[j] = rinv; }
    for (int l = j + 1 + tid; l < k; l += nt) sm[upk(j, l, k)] *= rinv;
    __syncthreads();
    // trailing update of rows i > j (upper part), 32 threads per row
    for (int i = j + 1 + tid / 32; i < k; i += nt / 32) {
      const double rji = sm[upk(j, i, k)];
      for (int l = i + (tid & 31); l < k; l += 32) sm[upk(i, l, k)] -= rji * sm[upk(j, l, k)];
    }
    __syncthreads();
  }
  // inverse of the upper-triangular R by back substitution, column c:
  //   x_c = 1 / R_cc,  x_i = -(sum_{l=i+1..c} R_il x_l) / R_ii  (i < c).
  // 16 lanes per column, CH = 16 columns at a time; lane j owns the entries
  // l = j (mod 16) of its column's x (kept in LDS, read back only by the
  // same lane), partial sums are combined with width-16 shuffles.
  double* xs = sm + (k * (k + 1)) / 2;  // [CH][k]
  constexpr int CH = 16;
  const int grp = tid >> 4, lj = tid & 15;   // threads beyond 16 groups idle here
  for (int c0 = 0; c0 < k; c0 += CH) {
    const int c = c0 + grp;
    const bool active = (c < k) && (grp < CH);
    double* x = xs + grp * k;
    for (int i = (active ? c : -1); i >= 0; --i) {
      double part = 0.0;
      for (int l = i + 1 + ((lj - (i + 1)) & 15); l <= c; l += 16) part += sm[upk(i, l, k)] * x[l];
      part += __shfl_xor(part, 8, 16);
      part += __shfl_xor(part, 4, 16);
      part += __shfl_xor(part, 2, 16);
      part += __shfl_xor(part, 1, 16);
      const double xi = (i == c) ? s_rinv[c] : -part * s_rinv[i];
      if ((i & 15) == lj) x[i] = xi;
    }
    if (active)
      for (int i = lj; i < k; i += 16) ri[i * k + c] = (i <= c) ? x[i] : 0.0;
    __syncthreads();
  }
  if (fail && tid == 0 && st.p[pb]) st.p[pb]->chol_fail = 1;
}

hipError_t chol_shift_inv(hipStream_t s, int k, double shift_coef, const CPtrSet& G,
                          const PtrSet& Rinv, const StatSet& st, int nprob) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  // dynamic LDS: packed R plus 16 columns of the inverse; 8 KiB of the CU's
  // 160 KiB stay for the kernel's static arrays
  constexpr size_t kMaxDyn = 160 * 1024 - 8192;
  size_t lds = ((size_t)k * (k + 1) / 2 + (size_t)16 * k) * sizeof(double);
  if (lds > kMaxDyn) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(G.p[i], (size_t)k * k * 8, "chol G") || !span_ok(Rinv.p[i], (size_t)k * k * 8, "chol Rinv") ||
        !span_ok(st.p[i], sizeof(SolveStatus), "chol status"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)chol_shift_inv_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDyn);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // do not leave the error pending for later calls
      return e;
    }
    attr_set = true;
  }
  hipLaunchKernelGGL(chol_shift_inv_kernel, dim3(nprob), dim3(1024), lds, s, k, shift_coef, G, Rinv, st);
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

__global__ void __launch_bounds__(1024)
jacobi_svd_kernel(int k, CPtrSet Min, PtrSet Uout, PtrSet Sout, PtrSet Wout, PtrSet work, int want_vectors,
                  int transpose_in, StatSet st, double noise_rel, int in_lds) {
  extern __shared__ double jsm[];         // A, Gram and W when they fit in LDS
  const int pb = blockIdx.x;
  double* A = in_lds ? jsm : work.p[pb];  // column-major k x k, column c at A + c*k
  double* Gm = A + (size_t)k * k;         // Gram of the columns at the start of a sweep
  double* W = Gm + (size_t)k * k;         // column-major right rotations
  const double* M = Min.p[pb];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  __shared__ int s_rot;
  __shared__ double s_norm[256];
  __shared__ int s_perm[256];
  __shared__ int s_touched[256];
  __shared__ unsigned s_sig[256 * 256 / 32];  // bit (p*k+q): pair significant at sweep start
  __shared__ double s_amax;

  // A holds M (or M^T when transpose_in) column-major
  for (int e = tid; e < k * k; e += nt) {
    int r = e / k, c = e % k;
    A[c * k + r] = transpose_in ? M[c * k + r] : M[e];
    if (want_vectors) W[c * k + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kk = (k + 1) & ~1;  // even number of players; player k (if odd) is a dummy
  const double eps = 2.220446049250313e-16 * (double)k;
  int sweeps_done = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    sweeps_done = sweep + 1;
    for (int e = tid; e < (k * k + 31) / 32; e += nt) s_sig[e] = 0u;
    __syncthreads();
    // Gram of all column pairs (upper triangle incl. diagonal): wave w holds
    // column p = w, w + nw, ... in registers (lanes over rows, k <= 256) and
    // forms its dot products with every later column, coalesced.
    for (int p = wave; p < k; p += nw) {
      double xp[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int i = lane + 64 * t;
        xp[t] = (i < k) ? A[(size_t)p * k + i] : 0.0;
      }
      for (int q = p; q < k; ++q) {
        const double* xq = A + (size_t)q * k;
        double g = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int i = lane + 64 * t;
          if (i < k) g += xp[t] * xq[i];
        }
        g = wsum(g);
        if (lane == 0) Gm[(size_t)p * k + q] = g;
      }
    }
    if (tid < k) s_touched[tid] = 0;
    if (tid == 0) s_rot = 0;
    __syncthreads();
    if (tid == 0) {
      double m = 0;
      for (int c = 0; c < k; ++c) m = fmax(m, Gm[(size_t)c * k + c]);
      s_amax = m;
    }
    __syncthreads();
    // columns whose norm is below noise_rel (at least 4 u) of the largest are
    // noise for the caller and are not rotated: they cannot move anything
    // above that level
    const double nr = fmax(noise_rel, 4.0 * 1.1102230246251565e-16);
    const double noise = s_amax * nr * nr;
    // significance bits of all pairs from the sweep's Gram
    for (int e = tid; e < k * k; e += nt) {
      int p = e / k, q = e - p * k;
      if (q <= p) continue;
      double a0 = Gm[(size_t)p * k + p], b0 = Gm[(size_t)q * k + q], g0 = Gm[(size_t)p * k + q];
      if (fmin(a0, b0) > noise && fabs(g0) > eps * sqrt(a0 * b0)) atomicOr(&s_sig[e >> 5], 1u << (e & 31));
    }
    __syncthreads();
    int rotated = 0;
    for (int r = 0; r < kk - 1; ++r) {
      for (int j = wave; j < kk / 2; j += nw) {
        int p = rr_player(j, r, kk), q = rr_player(kk - 1 - j, r, kk);
        if (p >= k || q >= k) continue;
        if (p > q) { int t = p; p = q; q = t; }
        if (!s_touched[p] && !s_touched[q]) {
          // both columns unchanged since the sweep's Gram: screen on it
          const int e = p * k + q;
          if (!((s_sig[e >> 5] >> (e & 31)) & 1u)) continue;
        }
        double* xp = A + (size_t)p * k;
        double* xq = A + (size_t)q * k;
        double a = 0, b = 0, g = 0;
        for (int i = lane; i < k; i += 64) {
          double u = xp[i], v = xq[i];
          a += u * u; b += v * v; g += u * v;
        }
        a = wsum(a); b = wsum(b); g = wsum(g);
        if (fmin(a, b) > noise && fabs(g) > eps * sqrt(a * b)) {
          double zeta = (b - a) / (2.0 * g);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int i = lane; i < k; i += 64) {
            double u = xp[i], v = xq[i];
            xp[i] = c * u - sn * v;
            xq[i] = sn * u + c * v;
          }
          if (want_vectors) {
            double* wp = W + (size_t)p * k;
            double* wq = W + (size_t)q * k;
            for (int i = lane; i < k; i += 64) {
              double u = wp[i], v = wq[i];
              wp[i] = c * u - sn * v;
              wq[i] = sn * u + c * v;
            }
          }
          if (lane == 0) { s_touched[p] = 1; s_touched[q] = 1; }
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
  double* S = Sout.p[pb];
  for (int j = tid; j < k; j += nt) S[j] = s_norm[s_perm[j]];
  if (tid == 0 && st.p[pb]) st.p[pb]->jsweeps = sweeps_done;
  if (!want_vectors) return;
  double* U = Uout.p[pb];
  double* Wo = Wout.p[pb];
  for (int e = tid; e < k * k; e += nt) {
    int r = e / k, j = e % k;
    int c = s_perm[j];
    double sv = s_norm[c];
    U[e] = sv > 0 ? A[(size_t)c * k + r] / sv : 0.0;
    Wo[e] = W[(size_t)c * k + r];
  }
}

hipError_t jacobi_svd(hipStream_t s, int k, const CPtrSet& M, const PtrSet& U, const PtrSet& S,
                      const PtrSet& W, const PtrSet& work, int nprob, bool want_vectors, bool transpose_in,
                      const StatSet* st, double noise_rel) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  if (k > 192) return hipErrorInvalidValue;  // 16 waves x 6 pairs, 3 rows per lane
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(M.p[i], (size_t)k * k * 8, "jacobi M") || !span_ok(S.p[i], (size_t)k * 8, "jacobi S") ||
        !span_ok(work.p[i], (size_t)(want_vectors ? 3 : 2) * k * k * 8, "jacobi work") ||
        (want_vectors && (!span_ok(U.p[i], (size_t)k * k * 8, "jacobi U") ||
                          !span_ok(W.p[i], (size_t)k * k * 8, "jacobi W"))))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  StatSet none{};
  // the columns, their Gram matrix and the rotations live in LDS when they fit
  // next to the kernel's static arrays (about 12 KiB)
  constexpr size_t kJMaxDyn = 160 * 1024 - 16384;
  const size_t lds = (size_t)(want_vectors ? 3 : 2) * k * k * sizeof(double);
  const bool in_lds = lds <= kJMaxDyn;
  static bool attr_set = false;
  if (in_lds && !attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)jacobi_svd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kJMaxDyn);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    attr_set = true;
  }
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(nprob), dim3(1024), in_lds ? lds : 0, s, k, M, U, S, W, work,
                     want_vectors ? 1 : 0, transpose_in ? 1 : 0, st ? *st : none, noise_rel, in_lds ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residuals and cutoff
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
residual_kernel(int64_t n, int k, int chi, double cutoff, double tol, CPtrSet Z, CPtrSet V,
                CPtrSet S, StatSet st) {
  // 16 waves; lane = column within a chunk of 64, wave = row phase
  const int pb = blockIdx.x;
  const double* z = Z.p[pb];
  const double* v = V.p[pb];
  const double* sv = S.p[pb];
  __shared__ double s_part[16][64];
  __shared__ double s_res[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    if (c < k) {
      const double sc = sv[c];
      for (int64_t i = wave; i < n; i += 16) {
        double d = z[i * k + c] - sc * v[i * k + c];
        acc += d * d;
      }
    }
    s_part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && c < k) {
      double t = 0.0;
      for (int w = 0; w < 16; ++w) t += s_part[w][lane];
      s_res[c] = sqrt(t);
    }
    __syncthreads();
  }
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
    o->kcols = k;
  }
}

hipError_t residual_status(hipStream_t s, int64_t n, int k, int chi, double cutoff, double tol,
                           const CPtrSet& Z, const CPtrSet& V, const CPtrSet& S,
                           const StatSet& st, int nprob) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(Z.p[i], (size_t)n * k * 8, "resid Z") || !span_ok(V.p[i], (size_t)n * k * 8, "resid V") ||
        !span_ok(S.p[i], (size_t)k * 8, "resid S") || !span_ok(st.p[i], sizeof(SolveStatus), "resid st"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(residual_kernel, dim3(nprob), dim3(1024), 0, s, n, k, chi, cutoff, tol, Z, V, S, st);
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
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
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

__global__ void warm_start_kernel(int64_t n, int k, int kmax, PtrSet V0, CPtrSet Vprev, StatSet prev, uint64_t seed) {
  const int pb = blockIdx.y;
  double* v0 = V0.p[pb];
  const double* vp = Vprev.p[pb];
  // the kept block was stored with its own column count (leading dimension)
  int kp = (prev.p[pb] && vp) ? prev.p[pb]->kcols : 0;
  if (kp < 0 || kp > kmax) kp = 0;  // never read past the kept buffer (n x kmax)
  int keep = (prev.p[pb] && vp && kp > 0) ? prev.p[pb]->chi_eff : 0;
  if (keep > k) keep = k;
  if (keep > kp) keep = kp;
  const uint64_t sd = seed + 0x1000193ull * (uint64_t)pb * (uint64_t)n * (uint64_t)k * 2ull;
  const int64_t tot = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int c = (int)(e % k);
    if (c < keep) { v0[e] = vp[(e / k) * kp + c]; continue; }
    uint64_t a = sm64(sd + 2ull * (uint64_t)e), b = sm64(sd + 2ull * (uint64_t)e + 1ull);
    double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    v0[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

hipError_t warm_start(hipStream_t s, int64_t n, int k, int kmax, const PtrSet& V0, const CPtrSet& Vprev,
                      const StatSet& prev, uint64_t seed, int nprob) {
  if (k > kmax) return hipErrorInvalidValue;
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(V0.p[i], (size_t)n * k * 8, "warm V0") ||
        (Vprev.p[i] && !span_ok(Vprev.p[i], (size_t)n * kmax * 8, "warm Vprev")) ||
        (prev.p[i] && !span_ok(prev.p[i], sizeof(SolveStatus), "warm prev")))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n * k + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(warm_start_kernel, dim3((unsigned)blocks, nprob), dim3(256), 0, s, n, k, kmax, V0, Vprev, prev,
                     seed);
  return hipGetLastError();
}

__global__ void reset_status_kernel(StatSet st) {
  SolveStatus* o = st.p[threadIdx.x];
  o->iters = 0;
  o->converged = 0;
  o->chol_fail = 0;
}

hipError_t reset_status(hipStream_t s, const StatSet& st, int nprob) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(st.p[i], sizeof(SolveStatus), "reset st")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(reset_status_kernel, dim3(1), dim3(nprob), 0, s, st);
  return hipGetLastError();
}

}  // namespace ctmk
