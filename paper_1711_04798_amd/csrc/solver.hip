// float64 kernels of the truncated-SVD solver: shifted Cholesky with
// triangular inverse (for Cholesky-QR), one-sided Jacobi SVD of small square
// matrices, residual / cutoff bookkeeping and the warm-start block.
#include "solver.h"
#include "kernels.h"

#include <algorithm>
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

// a double of lane l (a wave-uniform lane index)
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------------------
// R alone for k <= 64 with four waves per problem: right-looking in blocks of
// four columns with a lookahead of one block.  Wave w owns the column blocks
// w, w + 4, w + 8, w + 12 and keeps them in registers (lane = row; a column of
// L is one double per lane).  A finished block is published row-major in LDS
// (entry (r, t) of block B at r * 4 + t), so a lane reads its own row of the
// block, and every lane of a wave the row c of a column it reduces, as one
// 32-byte load (the latter a broadcast).  Two panels alternate: while the
// other waves read block jb from one, the owner of block jb + 1 subtracts
// block jb from it, finishes it (the 4 x 4 diagonal block in registers, rows
// of the pivots through readlane) and publishes it in the other; then every
// wave subtracts block jb from its later blocks.  One barrier per block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
chol_quad_kernel(int k, double shift_coef, CPtrSet G, PtrSet R, StatSet st) {
  __shared__ double4 P[2][64];  // P[buf][r]: row r of the published block
  __shared__ int s_fail;
  const int pb = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_fail = 0;  // ordered before other waves' writes by the first barrier
  const double* g = G.p[pb];
  double* ro = R.p[pb];
  // the trace, by every wave in the same order
  double tr = lane < k ? g[lane * k + lane] : 0.0;
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
  const double shift = shift_coef * tr;
  const double floor_v = (tr > 0.0 ? tr : 1.0) * 1e-300;
  // v[i][t]: entry (lane, c) of column c = 4 (w + 4 i) + t; column c of the
  // lower input is row c of G's upper triangle
  double v[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 4 * (w + 4 * i) + t;
      v[i][t] = (c < k && lane < k && lane >= c) ? g[c * k + lane] + (lane == c ? shift : 0.0) : 0.0;
    }
  int fail = 0;
  // finish owned block i (already reduced by every earlier block), publish it
  auto finish = [&](int i, double4* out) {
    const int c0 = 4 * (w + 4 * i);
    double lb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = c0 + t;
      lb[t] = 0.0;
      if (j < k) {
        double sb = v[i][t];
#pragma unroll
        for (int m = 0; m < t; ++m) sb -= lb[m] * readlane_f64(lb[m], j);
        double d = readlane_f64(sb, j);
        if (!(d > floor_v)) { d = floor_v; fail = 1; }
        const double rinv = rsqrt(d), r = d * rinv;
        lb[t] = lane == j ? r : (lane > j ? sb * rinv : 0.0);
      }
      v[i][t] = lb[t];
    }
    out[lane] = make_double4(lb[0], lb[1], lb[2], lb[3]);
  };
  // owned block i minus the published block (lr: this lane's row of it)
  auto reduce = [&](int i, const double4& lr, const double4* pub) {
    const int c0 = 4 * (w + 4 * i);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double4 lc = pub[c0 + t];
      double x = v[i][t];
      x = fma(-lr.x, lc.x, x);
      x = fma(-lr.y, lc.y, x);
      x = fma(-lr.z, lc.z, x);
      x = fma(-lr.w, lc.w, x);
      v[i][t] = x;
    }
  };
  if (w == 0) finish(0, P[0]);
  __syncthreads();
  const int nblk = (k + 3) / 4;
  for (int jb = 0; jb + 1 < nblk; ++jb) {
    const int nb = jb + 1;
    const double4* pub = P[jb & 1];
    const double4 lr = pub[lane];
    if ((nb & 3) == w) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (w + 4 * i == nb) {
          reduce(i, lr, pub);
          finish(i, P[nb & 1]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int B = w + 4 * i;
      if (B > nb && B < nblk) reduce(i, lr, pub);
    }
    __syncthreads();
  }
  // R_rc = L_cr: row c of R is column c of L
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 4 * (w + 4 * i) + t;
      if (c < k && lane < k) ro[c * k + lane] = lane >= c ? v[i][t] : 0.0;
    }
  if (fail) s_fail = 1;
  __syncthreads();
  if (s_fail && tid == 0 && st.p[pb]) st.p[pb]->chol_fail = 1;
}

hipError_t chol_shift_inv(hipStream_t s, int k, double shift_coef, const CPtrSet& G,
                          const PtrSet& Rinv, const StatSet& st, int nprob, bool want_inverse) {
  if (!want_inverse && k > CHOL_WAVE_MAX) return hipErrorInvalidValue;
  if (nprob < 0 || nprob > MAXP || k < 1) return hipErrorInvalidValue;
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
  if (!want_inverse) {
    hipLaunchKernelGGL(chol_quad_kernel, dim3(nprob), dim3(256), 0, s, k, shift_coef, G, Rinv, st);
    return hipGetLastError();
  }
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
// Y <- Y R^{-1} in place for n x k row-major Y and upper-triangular R (k <= 64):
// right-looking substitution
//   x_j = v_j / R_jj,  then v_l -= x_j R_jl for every l > j,
// with four lanes per row: lane s of a quad holds the columns 4 t + s of its
// row in registers, the owner of column j forms x_j and a DPP quad broadcast
// hands it to the other three, which update their later columns (R read from
// LDS, laid out so that a lane's entries of a row of R are contiguous).  The
// dependent chain per column is a product, a broadcast and an FMA; 16 rows
// per wave, 64 per work-group.  Columns past k are carried as identity (their
// x stays 0 and never reaches a real column).
// ---------------------------------------------------------------------------
// DPP move of a double across lanes (two 32-bit moves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int KP>
__global__ void __launch_bounds__(256)
trsm_quad_kernel(int64_t n, int k, PtrSet Y, CPtrSet R, PtrSet Y32, int w32, CPtrSet Yin, int r_in) {
  constexpr int NT4 = KP / 4;
  // Rq[(4 j + s) NT4 + t] = R[j][4 t + s] for j < 4 t + s < k, else 0
  __shared__ __attribute__((aligned(16))) double Rq[KP * KP];
  __shared__ double rdq[KP];  // 1 / R_jj (1 past k)
  const int pb = blockIdx.y, tid = threadIdx.x;
  const double* __restrict__ r = R.p[pb];
  // this lane's part of its row of Y, loaded before R is staged so that the
  // two loads' latencies overlap
  const int lane = tid & 63, s = lane & 3;
  const int64_t row = (int64_t)blockIdx.x * 64 + (tid >> 6) * 16 + (lane >> 2);
  double* yr = Y.p[pb] + min<int64_t>(row, n - 1) * k;
  const double* yi = (r_in ? Yin.p[pb] : Y.p[pb]) + min<int64_t>(row, n - 1) * k;
  double tv[NT4];
#pragma unroll
  for (int t = 0; t < NT4; ++t) tv[t] = yi[min(4 * t + s, k - 1)];
  {
    constexpr int PER = (KP * KP + 255) / 256;
    double rv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = min(tid + 256 * q, KP * KP - 1), j = e / KP, rem = e - j * KP;
      const int l = 4 * (rem % NT4) + rem / NT4;
      rv[q] = r[min(j, k - 1) * k + min(l, k - 1)];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      if (e >= KP * KP) break;
      const int j = e / KP, rem = e - j * KP;
      const int l = 4 * (rem % NT4) + rem / NT4;
      Rq[e] = (j < l && l < k) ? rv[q] : 0.0;
    }
    if (tid < KP) {
      const double d = r[min(tid, k - 1) * (k + 1)];
      rdq[tid] = tid < k ? 1.0 / d : 1.0;
    }
  }
  __syncthreads();
  double y[NT4];
#pragma unroll
  for (int t = 0; t < NT4; ++t) y[t] = 4 * t + s < k ? tv[t] : 0.0;
  const double* rq = Rq + s * NT4;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int tj = j >> 2;
    const double v = y[tj] * rdq[j];
    double xj;
    switch (j & 3) {
      case 0: xj = dpp_f64<0x00>(v); break;
      case 1: xj = dpp_f64<0x55>(v); break;
      case 2: xj = dpp_f64<0xAA>(v); break;
      default: xj = dpp_f64<0xFF>(v); break;
    }
    if (s == (j & 3)) y[tj] = v;
#pragma unroll
    for (int t = tj; t < NT4; ++t) y[t] -= xj * rq[j * 4 * NT4 + t];
  }
  if (row < n) {
#pragma unroll
    for (int t = 0; t < NT4; ++t)
      if (4 * t + s < k) yr[4 * t + s] = y[t];
    if (w32) {
      float* __restrict__ y32 = (float*)Y32.p[pb] + row * k;
#pragma unroll
      for (int t = 0; t < NT4; ++t)
        if (4 * t + s < k) y32[4 * t + s] = (float)y[t];
    }
  }
}

hipError_t trsm_rows(hipStream_t s, int64_t n, int k, const PtrSet& Y, const CPtrSet& R, int nprob,
                     const PtrSet* Y32, const CPtrSet* Yin) {
  if (nprob < 0 || nprob > MAXP || k < 1 || k > CHOL_WAVE_MAX || n < 1) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(Y.p[i], (size_t)n * k * 8, "trsm Y") || !span_ok(R.p[i], (size_t)k * k * 8, "trsm R") ||
        (Y32 && (!Y32->p[i] || !span_ok(Y32->p[i], (size_t)n * k * 4, "trsm Y32"))) ||
        (Yin && (!Yin->p[i] || !span_ok(Yin->p[i], (size_t)n * k * 8, "trsm Yin"))))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const PtrSet y32 = Y32 ? *Y32 : PtrSet{};
  const CPtrSet yin = Yin ? *Yin : CPtrSet{};
  const int w32 = Y32 ? 1 : 0, r_in = Yin ? 1 : 0;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)nprob);
  if (k <= 16) hipLaunchKernelGGL(trsm_quad_kernel<16>, grid, dim3(256), 0, s, n, k, Y, R, y32, w32, yin, r_in);
  else if (k <= 32) hipLaunchKernelGGL(trsm_quad_kernel<32>, grid, dim3(256), 0, s, n, k, Y, R, y32, w32, yin, r_in);
  else if (k <= 48) hipLaunchKernelGGL(trsm_quad_kernel<48>, grid, dim3(256), 0, s, n, k, Y, R, y32, w32, yin, r_in);
  else hipLaunchKernelGGL(trsm_quad_kernel<64>, grid, dim3(256), 0, s, n, k, Y, R, y32, w32, yin, r_in);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram matrix of a tall block, k <= 64: G = Y^T Y (and the cross form
// G = X^T Y of two blocks, k <= 48).  A work-group takes a
// chunk of 4 rpw rows, wave w the rows w rpw .. (w + 1) rpw - 1 of it.  Four
// rows of Y are one K step of the float64 MFMA for both operands: lane l
// loads Y[r + l / 16][16 b + l % 16] once per column block b, which is the
// A operand of the tiles (b, .) (A = Y^T) and the B operand of the tiles
// (., b).  Only the tiles on and above the block diagonal are formed; wave 0
// adds the other waves' tiles (through LDS) in wave order and writes them
// with their mirror images as the chunk's partial k x k sum.  A second kernel adds the
// chunks in order (64 entries per work-group, a quarter of the chunks per
// wave, the four quarter sums in order).
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

// SYM: G = Y^T Y (X = Y, tiles on and above the block diagonal, mirrored);
// otherwise G = X^T Y (every tile; k <= 48 so that the LDS of the three
// waves' tiles stays within 64 KiB)
template <int KB, bool SYM>
__global__ void __launch_bounds__(256)
gram_partial_kernel(int64_t n, int k, int rpw, CPtrSet X, CPtrSet Y, double* __restrict__ part, int nchunks) {
  constexpr int NTL = SYM ? KB * (KB + 1) / 2 : KB * KB;
  __shared__ v4d red[3][NTL][64];  // waves 1..3
  const int pb = blockIdx.y, chunk = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const double* __restrict__ x = X.p[pb];
  const double* __restrict__ y = Y.p[pb];
  v4d acc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = ((int64_t)chunk * 4 + w) * rpw;
  for (int s0 = 0; s0 < rpw; s0 += 16) {
    // four K steps: every load first, then the products
    double fx[4][KB], fy[4][KB];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t r = r0 + s0 + 4 * st + lg;
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int c = 16 * b + lr;
        const bool in = r < n && c < k;
        fx[st][b] = in ? x[r * k + c] : 0.0;
        if constexpr (!SYM) fy[st][b] = in ? y[r * k + c] : 0.0;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      int t = 0;
#pragma unroll
      for (int i = 0; i < KB; ++i)
#pragma unroll
        for (int j = SYM ? i : 0; j < KB; ++j) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fx[st][i], SYM ? fx[st][j] : fy[st][j], acc[t], 0, 0, 0);
          ++t;
        }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int t = 0; t < NTL; ++t) red[w - 1][t][lane] = acc[t];
  }
  __syncthreads();
  if (w != 0) return;
  // tile t = (i, j): lane l, value q is entry (16 i + l / 16 + 4 q, 16 j + l % 16)
  double* __restrict__ P = part + ((int64_t)pb * nchunks + chunk) * k * k;
  int t = 0;
#pragma unroll
  for (int i = 0; i < KB; ++i)
#pragma unroll
    for (int j = SYM ? i : 0; j < KB; ++j) {
      const v4d v = ((acc[t] + red[0][t][lane]) + red[1][t][lane]) + red[2][t][lane];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = 16 * i + lg + 4 * q, b = 16 * j + lr;
        if (a < k && b < k) {
          P[a * k + b] = v[q];
          if (SYM && i != j) P[b * k + a] = v[q];
        }
      }
      ++t;
    }
}

// ---------------------------------------------------------------------------
// C = A B for row-major float64 A (n x K), B (K x N), C (n x N), K and N up to
// 64: one wave per 16 rows of C, every fragment loaded straight from memory
// (lane l: A[r + l % 16][4 s + l / 16] for K step s, B[4 s + l / 16][16 j +
// l % 16] for column block j), all loads issued before the products.  A wave
// reads its rows of A whole before it writes the same rows of C, so C may be
// A (no restrict on either).
// ---------------------------------------------------------------------------
template <int KS, int NB>
__global__ void __launch_bounds__(256)
rmul_small_kernel(int64_t n, int K, int N, CPtrSet A, CPtrSet B, PtrSet C) {
  const int pb = blockIdx.y, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (r0 >= n) return;  // whole wave
  const double* a = A.p[pb];
  const double* __restrict__ b = B.p[pb];
  double* c = C.p[pb];
  const int64_t ra = r0 + lr;
  double fa[KS], fb[KS][NB];
#pragma unroll
  for (int st = 0; st < KS; ++st) {
    const int ka = 4 * st + lg;
    fa[st] = (ra < n && ka < K) ? a[ra * K + ka] : 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int cb = 16 * j + lr;
      fb[st][j] = (ka < K && cb < N) ? b[ka * N + cb] : 0.0;
    }
  }
  v4d acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < KS; ++st)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[st], fb[st][j], acc[j], 0, 0, 0);
  // lane l, value q: row r0 + l / 16 + 4 q, column 16 j + l % 16
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int cb = 16 * j + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + lg + 4 * q;
      if (r < n && cb < N) c[r * N + cb] = acc[j][q];
    }
  }
}

hipError_t rmul_small(hipStream_t s, int64_t n, int K, int N, const CPtrSet& A, const CPtrSet& B, const PtrSet& C,
                      int nprob) {
  if (nprob < 0 || nprob > MAXP || n < 1 || K < 1 || K > 64 || N < 1 || N > 64) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(A.p[i], (size_t)n * K * 8, "rmul A") || !span_ok(B.p[i], (size_t)K * N * 8, "rmul B") ||
        !span_ok(C.p[i], (size_t)n * N * 8, "rmul C"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)nprob);
  const int ks = (K + 15) / 16, nb = (N + 15) / 16;
#define RMUL(KSV, NBV) \
  hipLaunchKernelGGL((rmul_small_kernel<4 * KSV, NBV>), grid, dim3(256), 0, s, n, K, N, A, B, C)
#define RMUL_N(KSV)                  \
  switch (nb) {                      \
    case 1: RMUL(KSV, 1); break;     \
    case 2: RMUL(KSV, 2); break;     \
    case 3: RMUL(KSV, 3); break;     \
    default: RMUL(KSV, 4); break;    \
  }
  switch (ks) {
    case 1: RMUL_N(1); break;
    case 2: RMUL_N(2); break;
    case 3: RMUL_N(3); break;
    default: RMUL_N(4); break;
  }
#undef RMUL_N
#undef RMUL
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
gram_reduce_kernel(const double* __restrict__ part, int nchunks, int k, PtrSet G) {
  __shared__ double q4[4][64];
  const int pb = blockIdx.y, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kk = k * k, e = blockIdx.x * 64 + lane;
  const double* __restrict__ p = part + (int64_t)pb * nchunks * kk;
  const int per = (nchunks + 3) / 4, c0 = w * per, c1 = min(nchunks, c0 + per);
  const double acc = e < kk ? ordered_sum(p + (int64_t)c0 * kk + e, c1 - c0, kk) : 0.0;
  q4[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < kk) G.p[pb][e] = ((q4[0][lane] + q4[1][lane]) + q4[2][lane]) + q4[3][lane];
}

// X == nullptr: the symmetric form (G = Y^T Y, k <= 64); else G = X^T Y (k <= 48)
static hipError_t gram_launch(hipStream_t s, int64_t n, int k, const CPtrSet* X, const CPtrSet& Y, const PtrSet& G,
                              int nprob, double* part, int64_t part_elems) {
  if (nprob < 0 || nprob > MAXP || k < 1 || k > (X ? 48 : 64) || n < 1) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  const int64_t kk = (int64_t)k * k;
  const int64_t cap = part_elems / (kk * nprob);  // chunks the scratch holds
  if (cap < 1) return hipErrorInvalidValue;
  // rows per wave: multiples of 16, as few as the scratch allows
  const int64_t rpw = 16 * std::max<int64_t>(1, (n + 64 * cap - 1) / (64 * cap));
  const int64_t nchunks = (n + 4 * rpw - 1) / (4 * rpw);
  if (nchunks > cap || rpw > INT32_MAX) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(Y.p[i], (size_t)n * k * 8, "gram Y") || !span_ok(G.p[i], (size_t)kk * 8, "gram G") ||
        (X && !span_ok(X->p[i], (size_t)n * k * 8, "gram X")))
      return hipErrorInvalidValue;
  if (!span_ok(part, (size_t)nchunks * kk * nprob * 8, "gram partials")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const dim3 g1((unsigned)nchunks, (unsigned)nprob);
  const CPtrSet Xs = X ? *X : Y;
  const int r = (int)rpw, nc = (int)nchunks;
#define GRAM_CASE(KBV)                                                                                      \
  case KBV:                                                                                                 \
    if (X) hipLaunchKernelGGL((gram_partial_kernel<KBV, false>), g1, dim3(256), 0, s, n, k, r, Xs, Y, part, nc); \
    else hipLaunchKernelGGL((gram_partial_kernel<KBV, true>), g1, dim3(256), 0, s, n, k, r, Xs, Y, part, nc);    \
    break;
  switch ((k + 15) / 16) {
    GRAM_CASE(1) GRAM_CASE(2) GRAM_CASE(3)
    default: hipLaunchKernelGGL((gram_partial_kernel<4, true>), g1, dim3(256), 0, s, n, k, r, Xs, Y, part, nc); break;
  }
#undef GRAM_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((kk + 63) / 64), (unsigned)nprob), dim3(256), 0, s, part,
                     (int)nchunks, k, G);
  return hipGetLastError();
}

hipError_t gram_small(hipStream_t s, int64_t n, int k, const CPtrSet& Y, const PtrSet& G, int nprob, double* part,
                      int64_t part_elems) {
  return gram_launch(s, n, k, nullptr, Y, G, nprob, part, part_elems);
}

hipError_t gram_cross_small(hipStream_t s, int64_t n, int k, const CPtrSet& X, const CPtrSet& Y, const PtrSet& G,
                            int nprob, double* part, int64_t part_elems) {
  return gram_launch(s, n, k, &X, Y, G, nprob, part, part_elems);
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of a k x k matrix, one workgroup per
// problem (Golub & Van Loan, Sec. 8.6.3; Hestenes 1958).  Columns are kept
// column-major (in LDS when they fit) and rotated in pairs of the round-robin
// schedule: k/2 disjoint pairs per round, every pair once per sweep.  A pair
// (p, q) with a = |x_p|^2, b = |x_q|^2, g = x_p . x_q is rotated when
// |g| > eps sqrt(a b); the rotation makes the two columns orthogonal.
//
// A pair is handled by 16 lanes (one DPP row): lane l holds rows l, l+16, ...
// of both columns in registers and the three dot products are butterfly sums
// within the row (DPP moves, no LDS round trip), so a work-group of nt
// threads rotates nt/16 pairs at a time with one barrier per round.
//
// When only singular values are wanted, rows and columns of the input that
// are exactly zero are dropped first (they contribute only zero singular
// values); a corner of rank chi_eff < chi is then a chi_eff-sized problem.
// ---------------------------------------------------------------------------
constexpr int JMAX = 192;      // largest k
constexpr int JR = JMAX / 16;  // rows per lane

// sum over the 16 lanes of a DPP row; every lane gets the same bits (each
// step adds a value to its mirror image, and fp addition commutes)
__device__ __forceinline__ double sum16(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

// round-robin partner schedule on kk (even) players: player 0 fixed, others
// rotate.  pair j of round r: (pos j, pos kk-1-j) with pos 0 = player 0 and
// pos t>0 = 1 + ((t - 1 + r) mod (kk - 1)).
__device__ __forceinline__ int rr_player(int pos, int r, int kk) {
  int v = pos - 1 + r;            // < 2 (kk - 1) for pos, r < kk - 1
  if (v >= kk - 1) v -= kk - 1;
  return pos == 0 ? 0 : 1 + v;
}

// compacted index list of the set flags fl[0..k) into map, count into *cnt
// (one wave, in order)
__device__ __forceinline__ void compact_flags(const int* fl, int k, int* map, int* cnt, int lane) {
  int base = 0;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + lane;
    const bool f = c < k && fl[c];
    const unsigned long long m = __ballot(f);
    if (f) map[base + __popcll(m & ((1ull << lane) - 1ull))] = c;
    base += __popcll(m);
  }
  if (lane == 0) *cnt = base;
}

extern __shared__ double jsm[];  // dynamic LDS of the Jacobi kernel

// The sweeps on the kr x kc working matrix A (column-major, leading dimension
// 16 NRL, rows kr.. zero) and the kc x kc rotations W right after it (same
// leading dimension): at the start of the dynamic LDS (IN_LDS) or at gA.
// NRL and the memory kind are compile-time constants so that the loads of a
// pair's columns are plain LDS (or global) loads issued together.  Returns the
// number of sweeps.
template <int NRL, bool IN_LDS>
__device__ int jacobi_sweeps(int k, int kc, double* gA, bool want_vectors, double nr, double rot_rel,
                             double* s_cn, double* s_amax, int* s_rot) {
  constexpr int ld = 16 * NRL;
  double* A = IN_LDS ? jsm : gA;
  double* W = A + (size_t)ld * kc;
  const int tid = threadIdx.x, ql = tid & 15, grp = tid >> 4, ngrp = blockDim.x >> 4;
  const int kk = (kc + 1) & ~1;  // even number of players; player kc (if odd) is a dummy
  const int half = kk / 2;
  // a pair is rotated while the cosine of its columns exceeds k u (or the
  // caller's coarser rot_rel)
  const double eps = fmax(2.220446049250313e-16 * (double)k, rot_rel);
  const double eps2 = eps * eps;
  int sweeps_done = 0;
  for (int sweep = 0; sweep < 60 && kc > 1; ++sweep) {
    sweeps_done = sweep + 1;
    for (int c = grp; c < kc; c += ngrp) {
      const double* x = A + (size_t)c * ld;
      double xv[NRL];
#pragma unroll
      for (int t = 0; t < NRL; ++t) xv[t] = x[ql + 16 * t];
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < NRL; ++t) a += xv[t] * xv[t];
      a = sum16(a);
      if (ql == 0) s_cn[c] = a;
    }
    __syncthreads();
    if (tid < 64) {
      double m = 0.0;
      for (int c = tid; c < kc; c += 64) m = fmax(m, s_cn[c]);
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
      if (tid == 0) { *s_amax = m; *s_rot = 0; }
    }
    __syncthreads();
    // columns whose norm is below nr of the largest are noise for the caller
    // and are not rotated: they cannot move anything above that level
    const double noise = *s_amax * nr * nr;
    int rotated = 0;
    for (int r = 0; r < kk - 1; ++r) {
      for (int j = grp; j < half; j += ngrp) {
        int p = rr_player(j, r, kk), q = rr_player(kk - 1 - j, r, kk);
        if (p >= kc || q >= kc) continue;
        if (p > q) { const int t = p; p = q; q = t; }
        double* cp = A + (size_t)p * ld;
        double* cq = A + (size_t)q * ld;
        double* wp = W + (size_t)p * ld;
        double* wq = W + (size_t)q * ld;
        // for short columns the rotations' columns are loaded with the
        // pair's, so that their latency hides behind the rotation arithmetic
        constexpr bool early = NRL <= 6;
        double xp[NRL], xq[NRL], u[NRL], v[NRL];
#pragma unroll
        for (int t = 0; t < NRL; ++t) {
          xp[t] = cp[ql + 16 * t];
          xq[t] = cq[ql + 16 * t];
          if (early && want_vectors) {
            u[t] = wp[ql + 16 * t];
            v[t] = wq[ql + 16 * t];
          }
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int t = 0; t < NRL; ++t) {
          a += xp[t] * xp[t];
          b += xq[t] * xq[t];
          g += xp[t] * xq[t];
        }
        a = sum16(a);
        b = sum16(b);
        g = sum16(g);
        if (fmin(a, b) > noise && g * g > eps2 * (a * b)) {
          // the smaller angle that zeroes g (Rutishauser's form of the
          // tangent, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta =
          // (b - a) / 2g), without a division: with d = b - a, h =
          // sqrt(d^2 + 4 g^2) and e = |d| + h, t = 2 g sign(d) / e, so
          // c = 1 / sqrt(1 + t^2) = e / sqrt(e^2 + 4 g^2) and s = c t =
          // 2 g sign(d) / sqrt(e^2 + 4 g^2).  Both square roots come from
          // reciprocal square roots, the second exactly normalising (c, s).
          const double d = b - a, g2 = 2.0 * g;
          const double h2 = fma(d, d, g2 * g2);
          const double e = fabs(d) + h2 * rsqrt(h2);
          const double r = rsqrt(fma(e, e, g2 * g2));
          const double c = e * r, sn = (d >= 0 ? g2 : -g2) * r;
#pragma unroll
          for (int t = 0; t < NRL; ++t) {
            cp[ql + 16 * t] = c * xp[t] - sn * xq[t];
            cq[ql + 16 * t] = sn * xp[t] + c * xq[t];
          }
          if (want_vectors) {
            if (!early) {
#pragma unroll
              for (int t = 0; t < NRL; ++t) {
                u[t] = wp[ql + 16 * t];
                v[t] = wq[ql + 16 * t];
              }
            }
#pragma unroll
            for (int t = 0; t < NRL; ++t) {
              wp[ql + 16 * t] = c * u[t] - sn * v[t];
              wq[ql + 16 * t] = sn * u[t] + c * v[t];
            }
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated) *s_rot = 1;
    __syncthreads();
    if (!*s_rot) break;
  }
  return sweeps_done;
}

__global__ void __launch_bounds__(1024)
jacobi_svd_kernel(int k, CPtrSet Min, PtrSet Uout, PtrSet Sout, PtrSet Wout, PtrSet work, int want_vectors,
                  int transpose_in, StatSet st, double noise_rel, double rot_rel, size_t lds_cap) {
  const int pb = blockIdx.x;
  const double* M = Min.p[pb];
  const int tid = threadIdx.x, nt = blockDim.x, ql = tid & 15, grp = tid >> 4, ngrp = nt >> 4;
  __shared__ int s_rnz[JMAX], s_cnz[JMAX], s_rmap[JMAX], s_cmap[JMAX];
  __shared__ int s_kr, s_kc, s_rot;
  __shared__ double s_cn[JMAX], s_norm[JMAX], s_amax;
  __shared__ int s_perm[JMAX];
  // X = M (or M^T).  Rows / columns kept: all, or the non-zero ones.
  auto X = [&](int r, int c) { return transpose_in ? M[(size_t)c * k + r] : M[(size_t)r * k + c]; };
  if (want_vectors) {
    for (int c = tid; c < k; c += nt) { s_rmap[c] = c; s_cmap[c] = c; }
    if (tid == 0) { s_kr = k; s_kc = k; }
  } else {
    for (int c = tid; c < k; c += nt) { s_rnz[c] = 0; s_cnz[c] = 0; }
    __syncthreads();
    // scan M in order, eight loads in flight per thread (indices clamped);
    // M(a, b) is X(a, b), or X(b, a) with transpose_in
    const int kk2 = k * k;
    for (int e0 = tid; e0 < kk2; e0 += 8 * nt) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = M[min(e0 + u * nt, kk2 - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * nt, a = e / k, b = e - a * k;
        if (e < kk2 && v[u] != 0.0) {
          s_rnz[transpose_in ? b : a] = 1;
          s_cnz[transpose_in ? a : b] = 1;
        }
      }
    }
    __syncthreads();
    if (tid < 64) compact_flags(s_rnz, k, s_rmap, &s_kr, tid);
    else if (tid < 128) compact_flags(s_cnz, k, s_cmap, &s_kc, tid - 64);
  }
  __syncthreads();
  // the working matrix A: kr rows (padded with zeros to ld = 16 nrl) x kc
  // columns, column-major, with the shorter side as columns when vectors are
  // not wanted
  const bool flip = !want_vectors && s_kc > s_kr;
  const int kr = flip ? s_kc : s_kr, kc = flip ? s_kr : s_kc;
  const int nrl = (kr + 15) >> 4, ld = 16 * nrl;
  const size_t need = (size_t)(want_vectors ? 2 : 1) * ld * kc * sizeof(double);
  const bool in_lds = need <= lds_cap;
  double* A = in_lds ? jsm : work.p[pb];
  double* W = A + (size_t)ld * kc;  // column-major kc x kc right rotations (leading dimension ld)
  // gather, four loads in flight per thread (rows past kr read a valid
  // element that is then replaced by zero)
  for (int e0 = tid; e0 < ld * kc; e0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + u * nt, ld * kc - 1), j = e / ld, i = min(e - j * ld, kr - 1);
      v[u] = flip ? X(s_rmap[j], s_cmap[i]) : X(s_rmap[i], s_cmap[j]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nt;
      if (e < ld * kc) {
        const int j = e / ld, i = e - j * ld;
        A[e] = i >= kr ? 0.0 : v[u];
        if (want_vectors) W[e] = (i == j) ? 1.0 : 0.0;
      }
    }
  }
  __syncthreads();
  const double nr = fmax(noise_rel, 4.0 * 1.1102230246251565e-16);  // at least 4 u
  const bool wv = want_vectors != 0;
  int sweeps_done = 0;
  switch (in_lds ? nrl : nrl + 16) {
    case 1: sweeps_done = jacobi_sweeps<1, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 2: sweeps_done = jacobi_sweeps<2, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 3: sweeps_done = jacobi_sweeps<3, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 4: sweeps_done = jacobi_sweeps<4, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 5: sweeps_done = jacobi_sweeps<5, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 6: sweeps_done = jacobi_sweeps<6, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 7: sweeps_done = jacobi_sweeps<7, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 8: sweeps_done = jacobi_sweeps<8, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 9: sweeps_done = jacobi_sweeps<9, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 10: sweeps_done = jacobi_sweeps<10, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 11: sweeps_done = jacobi_sweeps<11, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 12: sweeps_done = jacobi_sweeps<12, true>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 17: sweeps_done = jacobi_sweeps<1, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 18: sweeps_done = jacobi_sweeps<2, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 19: sweeps_done = jacobi_sweeps<3, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 20: sweeps_done = jacobi_sweeps<4, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 21: sweeps_done = jacobi_sweeps<5, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 22: sweeps_done = jacobi_sweeps<6, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 23: sweeps_done = jacobi_sweeps<7, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 24: sweeps_done = jacobi_sweeps<8, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 25: sweeps_done = jacobi_sweeps<9, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 26: sweeps_done = jacobi_sweeps<10, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 27: sweeps_done = jacobi_sweeps<11, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    case 28: sweeps_done = jacobi_sweeps<12, false>(k, kc, A, wv, nr, rot_rel, s_cn, &s_amax, &s_rot); break;
    default: break;  // kr == 0: an all-zero input
  }
  // singular values = column norms (zero for the dropped part), sorted
  // descending (stable)
  for (int c = grp; c < kc; c += ngrp) {
    const double* x = A + (size_t)c * ld;
    double a = 0.0;
    for (int t = 0; t < nrl; ++t) a += x[ql + 16 * t] * x[ql + 16 * t];
    a = sum16(a);
    if (ql == 0) s_norm[c] = sqrt(a);
  }
  for (int c = kc + tid; c < k; c += nt) s_norm[c] = 0.0;
  __syncthreads();
  // non-finite norms sort last (key -1), so the ranks form a permutation
  for (int c = tid; c < k; c += nt) {
    const double v = isfinite(s_norm[c]) ? s_norm[c] : -1.0;
    int rank = 0;
    for (int o = 0; o < k; ++o) {
      const double w = isfinite(s_norm[o]) ? s_norm[o] : -1.0;
      rank += (w > v) || (w == v && o < c);
    }
    s_perm[rank] = c;
  }
  __syncthreads();
  double* S = Sout.p[pb];
  for (int j = tid; j < k; j += nt) S[j] = s_norm[s_perm[j]];
  if (tid == 0 && st.p[pb]) st.p[pb]->jsweeps = sweeps_done;
  if (!want_vectors) return;
  // vectors: no rows or columns were dropped (kr = kc = k)
  double* U = Uout.p[pb];
  double* Wo = Wout.p[pb];
  for (int e = tid; e < k * k; e += nt) {
    const int r = e / k, j = e - r * k;
    const int c = s_perm[j];
    const double sv = s_norm[c];
    U[e] = sv > 0 ? A[(size_t)c * ld + r] / sv : 0.0;
    Wo[e] = W[(size_t)c * ld + r];
  }
}

hipError_t jacobi_svd(hipStream_t s, int k, const CPtrSet& M, const PtrSet& U, const PtrSet& S,
                      const PtrSet& W, const PtrSet& work, int nprob, bool want_vectors, bool transpose_in,
                      const StatSet* st, double noise_rel, double rot_rel) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  if (k < 1 || k > JMAX) return hipErrorInvalidValue;
  // the columns (and rotations) live in LDS when they fit next to the
  // kernel's static arrays (about 7 KiB); the kernel decides after dropping
  // zero rows and columns.  Otherwise `work` holds them: rows padded to a
  // multiple of 16.
  constexpr size_t kJMaxDyn = 160 * 1024 - 16384;
  const size_t full = (size_t)(want_vectors ? 2 : 1) * (size_t)((k + 15) / 16 * 16) * k * sizeof(double);
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(M.p[i], (size_t)k * k * 8, "jacobi M") || !span_ok(S.p[i], (size_t)k * 8, "jacobi S") ||
        (full > kJMaxDyn && !span_ok(work.p[i], full, "jacobi work")) ||
        (want_vectors && (!span_ok(U.p[i], (size_t)k * k * 8, "jacobi U") ||
                          !span_ok(W.p[i], (size_t)k * k * 8, "jacobi W"))))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  StatSet none{};
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)jacobi_svd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kJMaxDyn);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    attr_set = true;
  }
  // 16 lanes per pair: enough waves for every pair of a round (at most 16)
  const int half = ((k + 1) & ~1) / 2;
  int waves = (half + 3) / 4;
  waves = waves < 2 ? 2 : (waves > 16 ? 16 : waves);
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(nprob), dim3(64 * waves), kJMaxDyn, s, k, M, U, S, W, work,
                     want_vectors ? 1 : 0, transpose_in ? 1 : 0, st ? *st : none, noise_rel, rot_rel, kJMaxDyn);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residuals and cutoff
// ---------------------------------------------------------------------------
// Residual norms in two deterministic stages: work-group (b, problem) adds
// the squared residuals of rows b, b + NB, b + 2 NB, ... per column (lanes over
// columns, waves over rows, all loads of a thread independent), then one
// work-group per problem sums the NB partials of each column in order and
// sets the status.
__global__ void __launch_bounds__(256)
residual_partial_kernel(int64_t n, int k, CPtrSet Z, CPtrSet V, CPtrSet S, double* part) {
  const int b = blockIdx.x, nb = gridDim.x, pb = blockIdx.y;
  const double* z = Z.p[pb];
  const double* v = V.p[pb];
  const double* sv = S.p[pb];
  __shared__ double s_part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* out = part + ((size_t)pb * nb + b) * k;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    if (c < k) {
      const double sc = sv[c];
      for (int64_t i = b + (int64_t)nb * wave; i < n; i += (int64_t)nb * 4) {
        const double d = z[i * k + c] - sc * v[i * k + c];
        acc += d * d;
      }
    }
    s_part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && c < k) out[c] = ((s_part[0][lane] + s_part[1][lane]) + s_part[2][lane]) + s_part[3][lane];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
residual_final_kernel(int64_t n, int k, int nb, int chi, double cutoff, double tol, CPtrSet S,
                      const double* part, StatSet st) {
  const int pb = blockIdx.x;
  const double* sv = S.p[pb];
  __shared__ double s_res[256];
  const double* p = nb > 0 ? part + (size_t)pb * nb * k : nullptr;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    const double t = nb > 0 ? ordered_sum(p + c, nb, k) : 0.0;
    s_res[c] = sqrt(t);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    SolveStatus* o = st.p[pb];
    double s0 = sv[0];
    int keep = 0;
    if (s0 > 0)
      for (int c = 0; c < k && c < chi; ++c)
        if (sv[c] > cutoff * s0) keep = c + 1;
    double tot = 0.0, tail = 0.0;
    for (int c = 0; c < k; ++c) {
      tot += sv[c] * sv[c];
      if (c >= keep) tail += sv[c] * sv[c];
    }
    o->discarded = tot > 0 ? tail / tot : 0.0;
    double mr = 0.0;
    for (int c = 0; c < keep; ++c) mr = fmax(mr, s_res[c]);
    mr = s0 > 0 ? mr / s0 : 0.0;
    if (nb == 0) mr = -1.0;  // residuals not formed
    o->chi_eff = keep;
    o->sigma0 = s0;
    o->max_resid = mr;
    o->converged = (nb > 0 && mr <= tol) ? 1 : 0;
    o->iters += 1;
    o->kcols = k;
    o->nrows = (int32_t)n;
  }
}

hipError_t residual_status(hipStream_t s, int64_t n, int k, int chi, double cutoff, double tol,
                           const CPtrSet& Z, const CPtrSet& V, const CPtrSet& S,
                           const StatSet& st, int nprob, double* scratch, int64_t scratch_elems) {
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  if (k > 256 || k < 1 || n < 1) return hipErrorInvalidValue;
  const bool with_resid = Z.p[0] != nullptr;
  int nb = with_resid ? (int)std::min<int64_t>(64, (n + 63) / 64) : 0;
  while (nb > 1 && (int64_t)nb * k * nprob > scratch_elems) nb /= 2;
  if ((int64_t)nb * k * nprob > scratch_elems) return hipErrorInvalidValue;
  for (int i = 0; i < nprob; ++i)
    if ((with_resid && (!span_ok(Z.p[i], (size_t)n * k * 8, "resid Z") || !span_ok(V.p[i], (size_t)n * k * 8, "resid V"))) ||
        !span_ok(S.p[i], (size_t)k * 8, "resid S") || !span_ok(st.p[i], sizeof(SolveStatus), "resid st"))
      return hipErrorInvalidValue;
  if (!span_ok(scratch, (size_t)nb * k * nprob * 8, "resid scratch")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (nb > 0)
    hipLaunchKernelGGL(residual_partial_kernel, dim3(nb, nprob), dim3(256), 0, s, n, k, Z, V, S, scratch);
  hipLaunchKernelGGL(residual_final_kernel, dim3(nprob), dim3(256), 0, s, n, k, nb, chi, cutoff, tol, S, scratch,
                     st);
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

__global__ void warm_start_kernel(int64_t n, int64_t n_cap, int k, int kmax, PtrSet V0, CPtrSet Vprev, StatSet prev,
                                  uint64_t seed) {
  const int pb = blockIdx.y;
  double* v0 = V0.p[pb];
  const double* vp = Vprev.p[pb];
  // the kept block was stored with its own column count (leading dimension)
  int kp = (prev.p[pb] && vp) ? prev.p[pb]->kcols : 0;
  if (kp < 0 || kp > kmax) kp = 0;  // never read past the kept buffer (n x kmax)
  int keep = (prev.p[pb] && vp && kp > 0) ? prev.p[pb]->chi_eff : 0;
  if (keep > k) keep = k;
  if (keep > kp) keep = kp;
  int64_t np = keep > 0 ? (int64_t)prev.p[pb]->nrows : 0;
  if (np < 0) np = 0;
  if (np > n_cap) np = n_cap;  // never read past the kept buffer (n_cap x kmax)
  const uint64_t sd = seed + 0x1000193ull * (uint64_t)pb * (uint64_t)n * (uint64_t)k * 2ull;
  const int64_t tot = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int c = (int)(e % k);
    if (c < keep) {
      const int64_t r = e / k;
      v0[e] = r < np ? vp[r * kp + c] : 0.0;
      continue;
    }
    uint64_t a = sm64(sd + 2ull * (uint64_t)e), b = sm64(sd + 2ull * (uint64_t)e + 1ull);
    double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    v0[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

hipError_t warm_start(hipStream_t s, int64_t n, int64_t n_cap, int k, int kmax, const PtrSet& V0,
                      const CPtrSet& Vprev, const StatSet& prev, uint64_t seed, int nprob) {
  if (k > kmax || n > n_cap) return hipErrorInvalidValue;
  if (nprob < 0 || nprob > MAXP) return hipErrorInvalidValue;
  if (nprob == 0) return hipSuccess;
  for (int i = 0; i < nprob; ++i)
    if (!span_ok(V0.p[i], (size_t)n * k * 8, "warm V0") ||
        (Vprev.p[i] && !span_ok(Vprev.p[i], (size_t)n_cap * kmax * 8, "warm Vprev")) ||
        (prev.p[i] && !span_ok(prev.p[i], sizeof(SolveStatus), "warm prev")))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n * k + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(warm_start_kernel, dim3((unsigned)blocks, nprob), dim3(256), 0, s, n, n_cap, k, kmax, V0, Vprev,
                     prev, seed);
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
