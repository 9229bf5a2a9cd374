// Boundary density operator of half an infinite cylinder from the CTM edges
// (paper Sec. IV, Eq. "Eq:rho" and the paragraph after it).
//
// The reduced density matrix of half a cylinder of circumference nv is an
// isometry applied to sqrt(sigma_L^T) sigma_R sqrt(sigma_L^T); its spectrum is
// that of sigma_L^T sigma_R.  sigma_L (sigma_R) is approximated by the left
// (right) half-row transfer tensors of the environment wrapped around a
// circle of nv sites: a ring of matrix-product operators on the D^nv virtual
// indices of the bonds that cross the cut.
//
// Everything is float64 on the device:
//   * ring application: the vector is carried as S[a][P][c][Q] (a the ring's
//     opening bond, P the output indices done so far, c the current bond, Q
//     the input indices left); each site is one GEMM over (c, input index)
//     through two-level views, and the ring closes with a trace over a = c;
//   * eigenvalues: block Lanczos on M = sigma_L^T sigma_R in the inner
//     product <x, y> = x^T sigma_R y, in which M is self-adjoint (sigma_L and
//     sigma_R symmetric, sigma_R positive semidefinite), with full
//     reorthogonalisation.  The block (several start vectors) resolves the
//     degenerate eigenvalues that the translations around the cylinder
//     produce, which a single Krylov sequence cannot.  The projected matrix
//     is diagonalised by cyclic Jacobi on the host; a residual estimate per
//     Ritz pair comes from the rows of the projection past the square part;
//   * trace of M, for the normalisation: the ring of the double transfer
//     matrices E_y[(cL, cR), (cL', cR')] = sum over both virtual indices of
//     the two edges, a product of nv chi^2 x chi^2 matrices.
#include "ctm.h"
#include "ctm_debug.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctm_internal.h"
#include "kernels.h"

using namespace ctmk;

namespace {

// rows per ring GEMM launch: 65535 row tiles of the smallest (32-row) tile
constexpr int64_t kRingRowsDefault = 65535LL * 32;
int64_t g_ring_rows = kRingRowsDefault;

#define BCHK(x)                                                                         \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return ctm_internal_fail(CTM_E_HIP, (std::string(#x) + ": " +  \
                                                               hipGetErrorString(e_)).c_str()); \
  } while (0)
#define BOK(x)                        \
  do {                                \
    ctm_status s_ = (x);              \
    if (s_ != CTM_OK) return s_;      \
  } while (0)

struct RegScope {
  Registry* prev;
  explicit RegScope(Registry* r) : prev(g_reg) { g_reg = r; }
  ~RegScope() { g_reg = prev; }
};

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// buffers carved from the caller's workspace (sizes in doubles)
struct Plan {
  int chi = 0, D = 0, Ly = 0, nv = 0, m = 0;
  int64_t dim = 0, state = 0, w4 = 0, e4 = 0;
  double* WL[4] = {};   // left edges as [up][bra][ket][down]
  double* S[2] = {};    // ring state
  double* Qv = nullptr; // Lanczos vectors q_0 .. q_m   (dim each)
  double* Pv = nullptr; // p_i = sigma_R q_i
  double* w = nullptr;
  double* u = nullptr;
  double* coef = nullptr;  // m + 1 inner products, then 2 scalars
  double* E[4] = {};       // double transfer matrices of the rows
  double* X[2] = {};       // ring product
  size_t bytes = 0;
  std::vector<std::pair<uintptr_t, size_t>> allocs;

  void layout(char* base) {
    size_t off = 0;
    allocs.clear();
    auto take = [&](int64_t n) -> double* {
      off = (off + 255) & ~size_t(255);
      double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
      if (base && n) allocs.emplace_back((uintptr_t)p, (size_t)n * 8);
      off += (size_t)n * 8;
      return p;
    };
    for (int y = 0; y < Ly; ++y) WL[y] = take(w4);
    S[0] = take(state);
    S[1] = take(state);
    Qv = take((int64_t)(m + 1) * dim);
    Pv = take((int64_t)(m + 1) * dim);
    w = take(dim);
    u = take(dim);
    coef = take(m + 3);
    for (int y = 0; y < Ly; ++y) E[y] = take(e4);
    X[0] = take(e4);
    X[1] = take(e4);
    bytes = off + 256;
  }
};

ctm_status plan_for(int chi, int D, int Ly, int nv, int m, Plan& p) {
  if (nv < 1 || nv % Ly != 0) return ctm_internal_fail(CTM_E_INVALID, "nv must be a positive multiple of the cell height");
  const double dimd = std::pow((double)D, (double)nv);
  const double stated = (double)chi * chi * dimd;
  if (dimd > 1e9 || stated > 4e9 || (double)chi * D * std::pow((double)D, nv - 1.0) * chi > 2e9)
    return ctm_internal_fail(CTM_E_INVALID, "chi^2 D^nv too large for the ring state");
  p.chi = chi; p.D = D; p.Ly = Ly; p.nv = nv;
  p.dim = ipow(D, nv);
  if (m < 1 || m > p.dim || m > 4096) return ctm_internal_fail(CTM_E_INVALID, "krylov must be in 1 .. min(D^nv, 4096)");
  p.m = m;
  p.state = (int64_t)chi * chi * p.dim;
  p.w4 = (int64_t)chi * D * D * chi;
  p.e4 = (int64_t)chi * chi * chi * chi;
  p.layout(nullptr);
  return CTM_OK;
}

// ---------------------------------------------------------------------------
// small deterministic kernels
// ---------------------------------------------------------------------------
// S[a][c][q] = (a == c) x[q]
__global__ void ring_open_kernel(const double* __restrict__ x, double* __restrict__ S, int chi, int64_t dim) {
  const int64_t tot = (int64_t)chi * chi * dim;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % dim, ac = e / dim;
    const int a = (int)(ac / chi), c = (int)(ac % chi);
    S[e] = a == c ? x[q] : 0.0;
  }
}

// out[p] = sum_a S[a][p][a], a in increasing order
__global__ void ring_close_kernel(const double* __restrict__ S, double* __restrict__ out, int chi, int64_t dim) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < dim; p += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int a = 0; a < chi; ++a) t += S[((int64_t)a * dim + p) * chi + a];
    out[p] = t;
  }
}

// out[i] = sum_e V[i][e] w[e] for i < nvec (one block per vector, fixed order)
__global__ void dots_kernel(const double* __restrict__ V, const double* __restrict__ w, int64_t n,
                            double* __restrict__ out) {
  __shared__ double red[256];
  const double* v = V + (int64_t)blockIdx.x * n;
  double t = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) t += v[e] * w[e];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// w[e] -= sum_{i < nvec} c[i] V[i][e]
__global__ void subtract_kernel(const double* __restrict__ V, const double* __restrict__ c, int nvec, int64_t n,
                                double* __restrict__ w) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double t = w[e];
    for (int i = 0; i < nvec; ++i) t -= c[i] * V[(int64_t)i * n + e];
    w[e] = t;
  }
}

// dst = src * (1 / sqrt(*s2))
__global__ void scale_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                             const double* __restrict__ s2) {
  const double f = 1.0 / sqrt(*s2);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e] * f;
}

// out = sum_i X[i][i] (one block)
__global__ void trace_kernel(const double* __restrict__ X, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) t += X[i * n + i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

struct Ctx {
  hipStream_t s;
  bool dry;
  const Plan* p;
};

hipError_t launch_check(bool dry) { return dry ? hipSuccess : hipGetLastError(); }

ctm_status gemm1(const Ctx& c, int64_t M, int64_t N, int64_t K, const View& va, const double* a, const View& vb,
                 const double* b, const View& vc, double* out) {
  GemmGroup g{};
  g.A[0] = a;
  g.B[0] = b;
  g.C[0] = out;
  BCHK(gemm(c.s, F64, F64, M, N, K, 1.0, va, vb, 0.0, vc, g, 1));
  return CTM_OK;
}

// out = ring(W) x: the operator sum over the ring of W_y[c][o][b][c'] applied
// to x (input index b, output index o), rows 0 .. nv-1 with edge y % Ly
ctm_status ring_apply(const Ctx& c, double* const* W, const double* x, double* out) {
  const Plan& p = *c.p;
  const int chi = p.chi, D = p.D;
  if (!span_ok(x, p.dim * 8, "ring x") || !span_ok(out, p.dim * 8, "ring out") ||
      !span_ok(p.S[0], p.state * 8, "ring state") || !span_ok(p.S[1], p.state * 8, "ring state"))
    return ctm_internal_fail(CTM_E_INVALID, "internal bounds check failed (boundary ring)");
  if (!c.dry) hipLaunchKernelGGL(ring_open_kernel, dim3(blocks_for(p.state)), dim3(256), 0, c.s, x, p.S[0], chi, p.dim);
  BCHK(launch_check(c.dry));
  int cur = 0;
  int64_t P = 1, Q = p.dim;
  for (int y = 0; y < p.nv; ++y) {
    const int64_t Q1 = Q / D;
    const View va{Q1, 1, (int64_t)chi * Q, D, Q1, Q};
    const View vb{D, chi, (int64_t)D * D * chi, chi, 1, (int64_t)D * chi};
    const View vc{Q1, 1, (int64_t)D * chi * Q1, chi, Q1, (int64_t)chi * Q1};
    // rows (h, l) = ((a, P), Q1): input row offset h chi Q + l, output
    // h D chi Q1 + l.  Launches of at most g_ring_rows rows (the GEMM grid's
    // second dimension counts row tiles of 32 or more), whole h at a time,
    // or pieces of one h when Q1 alone is longer.
    const int64_t H = (int64_t)chi * P, cap = g_ring_rows;
    const int64_t hc = Q1 <= cap ? cap / Q1 : 1;
    const int64_t lc = Q1 <= cap ? Q1 : cap;
    for (int64_t h0 = 0; h0 < H; h0 += hc)
      for (int64_t l0 = 0; l0 < Q1; l0 += lc) {
        const int64_t rows = Q1 <= cap ? std::min(hc, H - h0) * Q1 : std::min(lc, Q1 - l0);
        BOK(gemm1(c, rows, (int64_t)D * chi, (int64_t)chi * D, va, p.S[cur] + h0 * chi * Q + l0, vb,
                  W[y % p.Ly], vc, p.S[cur ^ 1] + h0 * D * chi * Q1 + l0));
      }
    cur ^= 1;
    P *= D;
    Q = Q1;
  }
  if (!c.dry) hipLaunchKernelGGL(ring_close_kernel, dim3(blocks_for(p.dim)), dim3(256), 0, c.s, p.S[cur], out, chi, p.dim);
  BCHK(launch_check(c.dry));
  return CTM_OK;
}

// Eigen-decomposition of the symmetric n x n matrix A (row-major, destroyed):
// Householder reduction to tridiagonal form T = Q^T A Q, then the implicit
// symmetric QR algorithm with Wilkinson shifts on T (Golub & Van Loan,
// Matrix Computations, Algorithms 8.3.1 and 8.3.3), the Givens rotations
// accumulated into Q when vectors are wanted.  4/3 n^3 + O(n^2) flops for
// the values (about 4 n^3 more with vectors) instead of about 3 n^3 per
// sweep of cyclic Jacobi.  Eigenvalues descending in w; with want_vectors
// the eigenvectors in the columns of V (row-major n x n).
void sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V, bool want_vectors) {
  w.assign(n, 0.0);
  // Qt = Q^T (row i = column i of Q), so that every update below touches
  // whole contiguous rows
  std::vector<double> Qt;
  if (want_vectors) {
    Qt.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
  }
  if (n == 0) return;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  std::vector<double> v(n), pv(n), q(n), d(n), e(n > 1 ? n - 1 : 1, 0.0);
  // Householder: column k below the subdiagonal -> alpha e_(k+1)
  for (int k = 0; k + 2 < n; ++k) {
    const int m0 = k + 1;
    double xn = 0.0;
    for (int i = m0; i < n; ++i) xn += a(i, k) * a(i, k);
    xn = std::sqrt(xn);
    double tail = 0.0;
    for (int i = m0 + 1; i < n; ++i) tail += a(i, k) * a(i, k);
    if (tail == 0.0) continue;  // already tridiagonal in this column
    const double alpha = a(m0, k) >= 0.0 ? -xn : xn;
    double vn = 0.0;
    for (int i = m0; i < n; ++i) {
      v[i] = a(i, k) - (i == m0 ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    vn = std::sqrt(vn);
    for (int i = m0; i < n; ++i) v[i] /= vn;
    // trailing block B <- H B H with H = I - 2 v v^T: p = B v, K = v.p,
    // q = p - K v, B <- B - 2 (v q^T + q v^T)
    double K = 0.0;
    for (int i = m0; i < n; ++i) {
      double t = 0.0;
      for (int j = m0; j < n; ++j) t += a(i, j) * v[j];
      pv[i] = t;
      K += v[i] * t;
    }
    for (int i = m0; i < n; ++i) q[i] = pv[i] - K * v[i];
    for (int i = m0; i < n; ++i)
      for (int j = m0; j < n; ++j) a(i, j) -= 2.0 * (v[i] * q[j] + q[i] * v[j]);
    a(m0, k) = a(k, m0) = alpha;
    for (int i = m0 + 1; i < n; ++i) a(i, k) = a(k, i) = 0.0;
    if (want_vectors) {
      // Q <- Q H, i.e. Qt <- H Qt: rows m0.. of Qt minus 2 v (v^T Qt)
      std::fill(pv.begin(), pv.end(), 0.0);
      for (int j = m0; j < n; ++j) {
        const double* row = &Qt[(size_t)j * n];
        for (int r = 0; r < n; ++r) pv[r] += v[j] * row[r];
      }
      for (int j = m0; j < n; ++j) {
        double* row = &Qt[(size_t)j * n];
        for (int r = 0; r < n; ++r) row[r] -= 2.0 * v[j] * pv[r];
      }
    }
  }
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
  // implicit symmetric QR on (d, e): deflate from the bottom
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, guard = 0;
  while (hi > 0 && guard < 60 * n) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    ++guard;
    // Wilkinson shift from the trailing 2 x 2 block
    const double dd = 0.5 * (d[hi - 1] - d[hi]), b2 = e[hi - 1] * e[hi - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::sqrt(dd * dd + b2);
    const double mu = den != 0.0 ? d[hi] - b2 / den : d[hi];
    double x = d[lo] - mu, z = e[lo], bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      // rotation on rows / columns k, k+1 that zeroes z against x
      const double r = std::hypot(x, z);
      const double c = r != 0.0 ? x / r : 1.0, s_ = r != 0.0 ? z / r : 0.0;
      if (k > lo) e[k - 1] = r;
      const double ak = d[k], bk = e[k], ck = d[k + 1];
      d[k] = c * c * ak + 2.0 * c * s_ * bk + s_ * s_ * ck;
      d[k + 1] = s_ * s_ * ak - 2.0 * c * s_ * bk + c * c * ck;
      e[k] = c * s_ * (ck - ak) + (c * c - s_ * s_) * bk;
      if (k + 1 < hi) {
        const double t = e[k + 1];
        bulge = s_ * t;
        e[k + 1] = c * t;
        x = e[k];
        z = bulge;
      }
      if (want_vectors) {
        // Q <- Q G: columns k, k+1 of Q are rows k, k+1 of Qt
        double* rk = &Qt[(size_t)k * n];
        double* rk1 = &Qt[(size_t)(k + 1) * n];
        for (int r2 = 0; r2 < n; ++r2) {
          const double vk = rk[r2], vk1 = rk1[r2];
          rk[r2] = c * vk + s_ * vk1;
          rk1[r2] = -s_ * vk + c * vk1;
        }
      }
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x1, int x2) { return d[x1] > d[x2]; });
  for (int j = 0; j < n; ++j) w[j] = d[idx[j]];
  if (want_vectors) {
    V.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
      const double* row = &Qt[(size_t)idx[j] * n];
      for (int r = 0; r < n; ++r) V[(size_t)r * n + j] = row[r];
    }
  }
}

}  // namespace

extern "C" {

ctm_status ctm_debug_sym_eig(int32_t n, const double* A, double* w, double* V) {
  if (n < 1 || !A || !w) return ctm_internal_fail(CTM_E_INVALID, "args");
  std::vector<double> a(A, A + (size_t)n * n), wv, vv;
  sym_eig(n, a, wv, vv, V != nullptr);
  std::copy(wv.begin(), wv.end(), w);
  if (V) std::copy(vv.begin(), vv.end(), V);
  return CTM_OK;
}

ctm_status ctm_debug_set_ring_rows(int64_t rows) {
  g_ring_rows = rows <= 0 ? kRingRowsDefault : std::min(rows, kRingRowsDefault);
  return CTM_OK;
}

ctm_status ctm_boundary_workspace_size(ctm_ctx x, int32_t inst, int32_t nv, int32_t krylov, size_t* bytes) {
  if (!bytes) return ctm_internal_fail(CTM_E_INVALID, "null bytes");
  CtmEdgeRing er;
  BOK(ctm_internal_edge_ring(x, inst, 0, &er));
  Plan p;
  BOK(plan_for(er.chi, er.D, er.Ly, nv, krylov, p));
  *bytes = p.bytes;
  return CTM_OK;
}

ctm_status ctm_boundary_spectrum(ctm_ctx x, int32_t inst, int32_t column, int32_t nv, int32_t krylov,
                                 int32_t block, uint64_t seed, void* ws_dev, size_t ws_bytes, int32_t nev,
                                 double* eig_out, double* resid_out, double* entropy_out, double* weight_out) {
  if (!eig_out || nev < 1) return ctm_internal_fail(CTM_E_INVALID, "eig_out / nev");
  CtmEdgeRing er;
  BOK(ctm_internal_edge_ring(x, inst, column, &er));
  Plan p;
  BOK(plan_for(er.chi, er.D, er.Ly, nv, krylov, p));
  if (block < 1 || block > 64 || block > p.m) return ctm_internal_fail(CTM_E_INVALID, "block must be in 1 .. min(64, krylov)");
  if (!ws_dev || ws_bytes < p.bytes)
    return ctm_internal_fail(CTM_E_NOMEM, ("boundary workspace too small: need " + std::to_string(p.bytes)).c_str());
  if (((uintptr_t)ws_dev) & 255) return ctm_internal_fail(CTM_E_INVALID, "workspace must be 256-byte aligned");
  p.layout((char*)ws_dev);
  Registry reg;
  reg.lo = (uintptr_t)ws_dev;
  reg.hi = (uintptr_t)ws_dev + p.bytes;
  reg.allocs = p.allocs;
  std::sort(reg.allocs.begin(), reg.allocs.end());
  reg.dry = er.dry;
  RegScope scope(&reg);
  const Ctx c{er.stream, er.dry, &p};
  hipStream_t s = er.stream;
  const int chi = p.chi, D = p.D, m = p.m;
  const int64_t dim = p.dim;
  // left edges T4[down][(ket, bra)][up] as [up][bra][ket][down]; the right
  // edges T2[up][(ket, bra)][down] are used as stored
  double* WR[4];
  for (int y = 0; y < p.Ly; ++y) {
    const int64_t dims[4] = {chi, D, D, chi};
    const int perm[4] = {3, 2, 1, 0};
    BCHK(permute(s, F64, er.T4[y], F64, p.WL[y], 4, dims, perm));
    WR[y] = const_cast<double*>(er.T2[y]);
  }
  auto read = [&](const double* dev, int n, double* host) -> ctm_status {
    if (c.dry) {
      for (int i = 0; i < n; ++i) host[i] = 1.0;
      return CTM_OK;
    }
    BCHK(hipMemcpyAsync(host, dev, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    return CTM_OK;
  };
  double* scal = p.coef + m + 1;  // two device scalars
  if (!span_ok(p.coef, (size_t)(m + 3) * 8, "boundary scalars")) return ctm_internal_fail(CTM_E_INVALID, "bounds");
  // trace of sigma_L^T sigma_R: ring of E_y[(cL, cR), (cL', cR')]
  //   = sum_(k, b) WL_y[cL][b][k][cL'] WR_y[cR][k][b][cR']
  double trace_host = 0.0;
  {
    const int64_t c2 = (int64_t)chi * chi;
    for (int y = 0; y < p.Ly; ++y) {
      const View va{chi, 1, (int64_t)D * D * chi, D, (int64_t)D * chi, chi};
      const View vb{D, chi, (int64_t)D * chi, chi, 1, (int64_t)D * D * chi};
      const View vc{chi, chi, (int64_t)chi * c2, chi, 1, c2};
      BOK(gemm1(c, c2, c2, (int64_t)D * D, va, p.WL[y], vb, WR[y], vc, p.E[y]));
    }
    const double* cur = p.E[0];
    int xb = 0;
    for (int y = 1; y < p.nv; ++y) {
      BOK(gemm1(c, c2, c2, c2, rowmajor(c2), cur, rowmajor(c2), p.E[y % p.Ly], rowmajor(c2), p.X[xb]));
      cur = p.X[xb];
      xb ^= 1;
    }
    if (!c.dry) hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, s, cur, c2, scal);
    BCHK(launch_check(c.dry));
    BOK(read(scal, 1, &trace_host));
  }
  const double tr = c.dry ? 1.0 : trace_host;
  if (!(std::fabs(tr) > 0) || !std::isfinite(tr)) return ctm_internal_fail(CTM_E_SOLVER, "zero or non-finite trace");

  // Block Lanczos in the sigma_R inner product.  Basis v_0 .. v_{n-1}
  // (sigma_R-orthonormal) with p_i = sigma_R v_i; column j of H holds the
  // coefficients of M v_j = sigma_L^T p_j on the basis (Arnoldi relation with
  // the block's stride).
  std::vector<double> H((size_t)m * m, 0.0);
  std::vector<double> ch(m + 1);
  int n = 0;                 // basis vectors so far
  uint64_t draws = 0;
  // Gram-Schmidt (two passes) of p.w against the basis; returns the summed
  // coefficients in ch[0..n-1]
  auto orthogonalize = [&]() -> ctm_status {
    std::fill(ch.begin(), ch.end(), 0.0);
    if (n == 0) return CTM_OK;
    std::vector<double> h(n);
    for (int pass = 0; pass < 2; ++pass) {
      if (!c.dry) {
        hipLaunchKernelGGL(dots_kernel, dim3(n), dim3(256), 0, s, p.Pv, p.w, dim, p.coef);
        hipLaunchKernelGGL(subtract_kernel, dim3(blocks_for(dim)), dim3(256), 0, s, p.Qv, p.coef, n, dim, p.w);
      }
      BCHK(launch_check(c.dry));
      BOK(read(p.coef, n, h.data()));
      for (int i = 0; i < n; ++i) ch[i] += h[i];
    }
    return CTM_OK;
  };
  // appends p.w (already orthogonal) to the basis if its sigma_R norm is
  // not negligible against `ref`; *norm_out gets that norm (0 if dropped)
  auto append = [&](double ref, double* norm_out) -> ctm_status {
    double* vn = p.Qv + (int64_t)n * dim;
    double* pn = p.Pv + (int64_t)n * dim;
    BOK(ring_apply(c, WR, p.w, p.u));
    if (!c.dry) hipLaunchKernelGGL(dots_kernel, dim3(1), dim3(256), 0, s, p.u, p.w, dim, scal);
    BCHK(launch_check(c.dry));
    double h2 = 0.0;
    BOK(read(scal, 1, &h2));
    *norm_out = 0.0;
    if (!(h2 > 1e-24 * ref * ref) || !std::isfinite(h2)) return CTM_OK;
    if (!c.dry) {
      hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(dim)), dim3(256), 0, s, p.w, vn, dim, scal);
      hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(dim)), dim3(256), 0, s, p.u, pn, dim, scal);
    }
    BCHK(launch_check(c.dry));
    *norm_out = std::sqrt(h2);
    ++n;
    return CTM_OK;
  };
  // a fresh random direction orthogonal to the basis
  auto add_random = [&](bool* ok) -> ctm_status {
    *ok = false;
    for (int tries = 0; tries < 4 && !*ok; ++tries) {
      BCHK(randn(s, p.w, dim, seed + 0x9E3779B97F4A7C15ull * (++draws)));
      // the start vector's own sigma_R norm sets the scale of "negligible"
      BOK(ring_apply(c, WR, p.w, p.u));
      if (!c.dry) hipLaunchKernelGGL(dots_kernel, dim3(1), dim3(256), 0, s, p.u, p.w, dim, scal);
      BCHK(launch_check(c.dry));
      double r2 = 0.0;
      BOK(read(scal, 1, &r2));
      if (!(r2 > 0)) return ctm_internal_fail(CTM_E_SOLVER, "sigma_R is not positive on a random vector");
      BOK(orthogonalize());
      double nrm = 0.0;
      BOK(append(std::sqrt(r2), &nrm));
      *ok = nrm > 0;
      if (c.dry) *ok = true;
    }
    return CTM_OK;
  };
  for (int b = 0; b < block && n < m; ++b) {
    bool ok = false;
    BOK(add_random(&ok));
    if (!ok) break;
  }
  int done = 0;  // columns of H computed
  double hscale = 0.0;
  while (done < n) {
    const int j = done;
    // w = M v_j = sigma_L^T sigma_R v_j
    BOK(ring_apply(c, p.WL, p.Pv + (int64_t)j * dim, p.w));
    BOK(orthogonalize());
    for (int i = 0; i < n; ++i) H[(size_t)i * m + j] = ch[i];
    hscale = std::max(hscale, std::fabs(ch[j]));
    ++done;
    if (n < m) {
      double nrm = 0.0;
      BOK(append(std::max(hscale, 1e-300), &nrm));
      if (nrm > 0) {
        H[(size_t)(n - 1) * m + j] = nrm;
      } else {
        // an invariant subspace: continue from a new random direction
        bool ok = false;
        BOK(add_random(&ok));
      }
    }
    if (n == m && done >= m - block && m < dim) break;  // the last block's images stay unknown
  }
  const int ns = done;  // columns known: the square part
  std::vector<double> Hs((size_t)ns * ns);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j)
      Hs[(size_t)i * ns + j] = 0.5 * (H[(size_t)i * m + j] + H[(size_t)j * m + i]);
  std::vector<double> ev, V;
  // vectors only for the residuals of a partial basis
  sym_eig(ns, Hs, ev, V, ns < n);
  double S = 0.0, wsum = 0.0;
  for (int i = 0; i < nev; ++i) {
    const double v = i < ns ? ev[i] / tr : 0.0;
    eig_out[i] = v;
    if (resid_out) {
      // |M V s - theta V s| from the rows past the square part
      double r2 = 0.0;
      for (int r = ns; r < n && i < ns; ++r) {
        double t = 0.0;
        for (int k = 0; k < ns; ++k) t += H[(size_t)r * m + k] * V[(size_t)k * ns + i];
        r2 += t * t;
      }
      resid_out[i] = i < ns ? std::sqrt(r2) / std::fabs(tr) : 0.0;
    }
    wsum += v;
    if (v > 0) S -= v * std::log(v);
  }
  if (entropy_out) *entropy_out = S;
  if (weight_out) *weight_out = wsum;
  return CTM_OK;
}

}  // extern "C"
