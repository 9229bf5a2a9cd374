// Simple update of the 2x2 checkerboard iPEPS: imaginary-time evolution by
// first-order Suzuki-Trotter factors e^{-dtau H_r} e^{-dtau H_l}
// e^{-dtau H_u} e^{-dtau H_d}, each a product of two-body gates
// g = e^{-dtau h} (paper Sec. II B), applied with bond weights and SVD
// truncation to D (the simple update that Sec. II D uses to start the
// ground-state search).
//
// Many instances of equal (d, D) (a scan over couplings, each with its own
// gates) move in lock-step: every stage of a bond update is one grouped
// launch over the instances.  Bond types: h0 = A.r - B.l, h1 = B.r - A.l,
// v0 = A.d - B.u, v1 = B.d - A.u (A at x + y even; the first site of a bond
// is the left or upper one); a Trotter step updates h0, h1, v0, v1 in turn.
//
// One bond update, all float64 on the device, k = d D, m = d k:
//   Xm[(o1,o2,o3),(s,p)] = X with the weights of its other legs o1 < o2 < o3
//                          multiplied in (D^3 x k), Ym likewise;
//   G = Xm^T Xm = W diag(S) W^T (one-sided Jacobi; G is positive
//   semidefinite), R = diag(sqrt S) W^T, so that Xm = Q R with orthonormal
//   Q = Xm W diag(S^-1/2) on the support of G;
//   theta[(a,i),(b,j)] = sum_(k,l) g[(i,j),(k,l)] sum_p R_X[a,(k,p)] lam_p R_Y[b,(l,p)]
//   with a, b below the rank bound r = min(D^3, k) of Xm (m = r d square);
//   its D leading singular triplets: one-sided Jacobi of the whole theta
//   when its working set fits LDS (m <= 80), otherwise subspace iteration
//   on a block of b = min(m, D + 16) counter-based normal columns (six
//   rounds of theta and theta^T products, each followed by Cholesky-QR) and
//   Rayleigh-Ritz through a Jacobi SVD of the b x b R factor of theta V;
//   new weights: the D largest sv above 1e-12 sv_1, divided by their norm;
//   X' = Q U[:, :D] = Xm (W diag(S^-1/2) R'_X) with R'_X[a,(i,p)] = U[(a,i),p],
//   then the weights of the other legs divided out (weights below 1e-12 of
//   their bond's largest count as zero) and X' divided by its Frobenius norm.
// The gates come from the bond Hamiltonians on the device: h + c I with
// c = ||h||_F + 1 is positive definite, so its Jacobi SVD is its
// eigendecomposition W diag(e) W^T, and g = W diag(exp(-dtau (e - c))) W^T.
#include "ctm_su.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctm_internal.h"
#include "kernels.h"
#include "solver.h"

using namespace ctmk;

namespace {

#define SCHK(x)                                                                          \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return ctm_internal_fail(CTM_E_HIP, (std::string(#x) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)
#define SOK(x)                   \
  do {                           \
    ctm_status s_ = (x);         \
    if (s_ != CTM_OK) return s_; \
  } while (0)

struct RegScope {
  Registry* prev;
  explicit RegScope(Registry* r) : prev(g_reg) { g_reg = r; }
  ~RegScope() { g_reg = prev; }
};

constexpr int NB = 4;  // bond types h0, h1, v0, v1
// (tensor, leg) of the first and second site of each bond; legs of
// T[s][u][l][d][r]: u = 1, l = 2, d = 3, r = 4; tensor 0 = A, 1 = B
constexpr int END_T[NB][2] = {{0, 1}, {1, 0}, {0, 1}, {1, 0}};
constexpr int END_L[NB][2] = {{4, 2}, {4, 2}, {3, 1}, {3, 1}};
// the bond of each leg (index leg - 1) of A and of B
__host__ __device__ constexpr int leg_bond(int t, int leg) {
  // A: u v1, l h1, d v0, r h0;  B: u v0, l h0, d v1, r h1
  return t == 0 ? (leg == 1 ? 3 : leg == 2 ? 1 : leg == 3 ? 2 : 0)
                : (leg == 1 ? 2 : leg == 2 ? 0 : leg == 3 ? 3 : 1);
}
constexpr double EPS = 1e-12;

struct Inst {
  double* T[2];
  double* lam[NB];
  double* gate[NB];
  double* Xm[2];     // D^3 x k
  double* Gm[2];     // k x k
  double* Ug[2];
  double* Wg[2];
  double* Sg[2];     // k
  double* Rr[2];     // k x k: R, then R scaled by the bond weights (X side)
  double* Pinv[2];   // k x k: W diag(S^-1/2)
  double* th0;       // m x m
  double* thp;       // permuted / gated scratch (m x m)
  double* th;        // m x m
  double* Ut;        // m x m
  double* Wt;
  double* St;        // m
  double* jw;        // Jacobi working columns: 2 m m16
  double* Vb;        // subspace iteration: m x b blocks
  double* Yb;
  double* Gb;        // b x b Gram, R factors
  double* Rb1;
  double* Rb2;
  double* Rb;
  double* Rn[2];     // k x k new R factors
  double* S1[2];     // k x k
  double* Xn[2];     // D^3 x k
  double* change;    // largest weight change since the last reset
  double* hs;        // gate construction: h + c I (d^2 x d^2), then scratch
  double* gU;
  double* gW;
  double* gS;
  double* norm_part; // normalisation partials (2 jobs)
};

}  // namespace

struct ctm_su_s {
  int n = 0, d = 0, D = 0, k = 0, m = 0, D3 = 0;
  int r = 0;          // rank bound of the reduced tensors: min(D^3, k); m = r d
  int b = 0;          // subspace block of the truncated SVD (0: full Jacobi)
  uint64_t updates = 0;  // bond updates done (seeds the subspace start)
  hipStream_t stream = nullptr;
  Registry reg;
  std::vector<Inst> inst;
  size_t ws_need = 0;
};

namespace {

struct Carve {
  char* base = nullptr;
  size_t off = 0;
  Registry* reg = nullptr;
  double* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    if (reg && base && count) reg->allocs.emplace_back((uintptr_t)p, count * sizeof(double));
    off += count * sizeof(double);
    return p;
  }
};

void plan(ctm_su_s& x, Carve& c) {
  const size_t d = x.d, D = x.D, k = x.k, m = x.m, D3 = x.D3, t5 = d * D * D * D * D, d4 = d * d * d * d;
  const size_t m16 = (m + 15) / 16 * 16, k16 = (k + 15) / 16 * 16, dd16 = (d * d + 15) / 16 * 16;
  x.inst.assign(x.n, Inst{});
  for (Inst& I : x.inst) {
    for (int t = 0; t < 2; ++t) I.T[t] = c.take(t5);
    for (int b = 0; b < NB; ++b) I.lam[b] = c.take(D);
    for (int b = 0; b < NB; ++b) I.gate[b] = c.take(d4);
    for (int t = 0; t < 2; ++t) {
      I.Xm[t] = c.take(D3 * k);
      I.Gm[t] = c.take(k * k);
      I.Ug[t] = c.take(k * k);
      I.Wg[t] = c.take(k * k);
      I.Sg[t] = c.take(k);
      I.Rr[t] = c.take(k * k);
      I.Pinv[t] = c.take(k * k);
      I.Rn[t] = c.take(k * k);
      I.S1[t] = c.take(k * k);
      I.Xn[t] = c.take(D3 * k);
    }
    I.th0 = c.take(m * m);
    I.thp = c.take(m * m);
    I.th = c.take(m * m);
    I.Ut = c.take(m * m);
    I.Wt = c.take(m * m);
    I.St = c.take(m);
    if (x.b) {
      I.Vb = c.take(m * x.b);
      I.Yb = c.take(m * x.b);
      I.Gb = c.take((size_t)x.b * x.b);
      I.Rb1 = c.take((size_t)x.b * x.b);
      I.Rb2 = c.take((size_t)x.b * x.b);
      I.Rb = c.take((size_t)x.b * x.b);
    }
    I.jw = c.take(2 * std::max({m * m16, k * k16, d * d * dd16}));
    I.change = c.take(1);
    I.hs = c.take(d4 + 1);  // h + c I, then the shift c
    I.gU = c.take(d4);
    I.gW = c.take(d4);
    I.gS = c.take(d * d);
    I.norm_part = c.take((size_t)MAXJ * 64);
  }
}

// pointer tables of up to MAXP instances for the kernels below
struct Ptrs {
  double* p[MAXP];
};

// Xm[(o1,o2,o3),(s,p)] = T[s][legs] times the weights of the legs other than
// `leg` (o1 < o2 < o3 in leg order); t selects the leg -> bond map
__global__ void su_prep_kernel(Ptrs T, Ptrs L0, Ptrs L1, Ptrs L2, Ptrs L3, Ptrs Xm, int t, int leg, int d, int D) {
  const int i = blockIdx.y;
  const double* lam[NB] = {L0.p[i], L1.p[i], L2.p[i], L3.p[i]};
  const int64_t D3 = (int64_t)D * D * D, k = (int64_t)d * D, n = D3 * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / k, col = e - row * k;
    const int s = (int)(col / D), p = (int)(col % D);
    int idx[5];
    idx[leg] = p;
    int64_t r = row;
    double w = 1.0;
    for (int lg = 4; lg >= 1; --lg) {
      if (lg == leg) continue;
      idx[lg] = (int)(r % D);
      r /= D;
      w *= lam[leg_bond(t, lg)][idx[lg]];
    }
    const int64_t off = (((((int64_t)s * D + idx[1]) * D + idx[2]) * D + idx[3]) * D) + idx[4];
    Xm.p[i][e] = T.p[i][off] * w;
  }
}

// inverse of su_prep_kernel with the other legs' weights divided out
__global__ void su_finish_kernel(Ptrs Xn, Ptrs L0, Ptrs L1, Ptrs L2, Ptrs L3, Ptrs T, int t, int leg, int d, int D) {
  const int i = blockIdx.y;
  const double* lam[NB] = {L0.p[i], L1.p[i], L2.p[i], L3.p[i]};
  double lmax[NB];
  for (int b = 0; b < NB; ++b) {
    double mx = 0.0;
    for (int j = 0; j < D; ++j) mx = fmax(mx, lam[b][j]);
    lmax[b] = mx;
  }
  const int64_t D3 = (int64_t)D * D * D, k = (int64_t)d * D, n = D3 * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / k, col = e - row * k;
    const int s = (int)(col / D), p = (int)(col % D);
    int idx[5];
    idx[leg] = p;
    int64_t r = row;
    double w = 1.0;
    for (int lg = 4; lg >= 1; --lg) {
      if (lg == leg) continue;
      idx[lg] = (int)(r % D);
      r /= D;
      const int b = leg_bond(t, lg);
      const double v = lam[b][idx[lg]];
      w *= v > EPS * lmax[b] ? 1.0 / v : 0.0;
    }
    const int64_t off = (((((int64_t)s * D + idx[1]) * D + idx[2]) * D + idx[3]) * D) + idx[4];
    T.p[i][off] = Xn.p[i][e] * w;
  }
}

// R = diag(sqrt S) W^T and Pinv = W diag(S^-1/2) (S^-1/2 = 0 below 1e-12 of
// the largest singular value of Xm, i.e. S below 1e-24 S_max)
__global__ void su_rfactor_kernel(Ptrs W, Ptrs S, Ptrs R, Ptrs P, int k) {
  const int i = blockIdx.y;
  const double* sv = S.p[i];
  const double smax = sv[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) {
    const int a = e / k, c = e % k;
    const double sa = sv[a] > 1e-24 * smax ? sv[a] : 0.0;
    R.p[i][e] = sqrt(sa) * W.p[i][c * k + a];
    const double sc = sv[c] > 1e-24 * smax ? sv[c] : 0.0;
    P.p[i][e] = sc > 0.0 ? W.p[i][e] / sqrt(sc) : 0.0;
  }
}

// R[a, (i, p)] *= lam_p
__global__ void su_scale_bond_kernel(Ptrs R, Ptrs lam, int k, int D) {
  const int i = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x)
    R.p[i][e] *= lam.p[i][e % D];
}

// new weights from the singular values of theta; the largest change since
// the last reset is kept in *change
__global__ void su_weights_kernel(Ptrs St, Ptrs lam, Ptrs change, int D, int reset) {
  const int i = blockIdx.x;
  if (threadIdx.x != 0) return;
  const double* sv = St.p[i];
  double* l = lam.p[i];
  const double s0 = sv[0];
  int keep = 0;
  if (s0 > 0)
    for (int j = 0; j < D; ++j)
      if (sv[j] > EPS * s0) keep = j + 1;
  double nrm = 0.0;
  for (int j = 0; j < keep; ++j) nrm += sv[j] * sv[j];
  nrm = sqrt(nrm);
  double ch = reset ? 0.0 : *change.p[i];
  for (int j = 0; j < D; ++j) {
    const double v = j < keep ? sv[j] / nrm : 0.0;
    ch = fmax(ch, fabs(v - l[j]));
    l[j] = v;
  }
  *change.p[i] = ch;
}

// R'_X[a, (i, p)] = U[(a, i), p] for a < r and p < keep (zero beyond); U has
// row stride ldu; the Y side from the right singular vectors
__global__ void su_newr_kernel(Ptrs U, Ptrs lam, Ptrs Rn, int k, int d, int D, int ldu, int r) {
  const int i = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) {
    const int a = e / k, c = e % k, s = c / D, p = c % D;
    Rn.p[i][e] = (a < r && lam.p[i][p] > 0.0) ? U.p[i][(int64_t)(a * d + s) * ldu + p] : 0.0;
  }
}

// h + c I with c = ||h||_F + 1 (positive definite), into hs
__global__ void su_shift_kernel(Ptrs h, Ptrs hs, int n) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) acc += h.p[i][e] * h.p[i][e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double c = sqrt(red[0]) + 1.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, q = e % n;
    // symmetrised
    hs.p[i][e] = 0.5 * (h.p[i][e] + h.p[i][q * n + r]) + (r == q ? c : 0.0);
  }
  if (threadIdx.x == 0) hs.p[i][n * n] = c;  // the shift, read by su_gate_scale_kernel
}

// gU <- W diag(exp(-dtau (S - c)))  (c stored after the n x n block of hs)
__global__ void su_gate_scale_kernel(Ptrs W, Ptrs S, Ptrs hs, Ptrs out, int n, double dtau) {
  const int i = blockIdx.x;
  const double c = hs.p[i][n * n];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int q = e % n;
    out.p[i][e] = W.p[i][e] * exp(-dtau * (S.p[i][q] - c));
  }
}

// T out = Gamma tensors times sqrt(weights) on every leg
__global__ void su_peps_kernel(Ptrs T, Ptrs L0, Ptrs L1, Ptrs L2, Ptrs L3, Ptrs out, int t, int d, int D) {
  const int i = blockIdx.y;
  const double* lam[NB] = {L0.p[i], L1.p[i], L2.p[i], L3.p[i]};
  const int64_t n = (int64_t)d * D * D * D * D;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    double w = 1.0;
    for (int lg = 4; lg >= 1; --lg) {
      const int ix = (int)(r % D);
      r /= D;
      w *= sqrt(lam[leg_bond(t, lg)][ix]);
    }
    out.p[i][e] = T.p[i][e] * w;
  }
}

hipError_t check_spans(std::initializer_list<std::pair<const void*, size_t>> l, const char* what) {
  for (auto& e : l)
    if (!span_ok(e.first, e.second, what)) return hipErrorInvalidValue;
  return hipSuccess;
}

struct Chunk {
  int i0, cnt;
};

std::vector<Chunk> chunks(int n) {
  std::vector<Chunk> c;
  for (int i0 = 0; i0 < n; i0 += MAXP) c.push_back({i0, std::min(MAXP, n - i0)});
  return c;
}

// grouped float64 GEMM over the instances of a chunk
ctm_status gemm64(hipStream_t s, int64_t M, int64_t N, int64_t K, const View& va, const View& vb, const View& vc,
                  const std::vector<const double*>& A, const std::vector<const double*>& B,
                  const std::vector<double*>& C) {
  for (size_t j0 = 0; j0 < A.size(); j0 += MAXG) {
    const int cnt = (int)std::min<size_t>(MAXG, A.size() - j0);
    GemmGroup g{};
    for (int j = 0; j < cnt; ++j) {
      g.A[j] = A[j0 + j];
      g.B[j] = B[j0 + j];
      g.C[j] = C[j0 + j];
    }
    SCHK(gemm(s, F64, F64, M, N, K, 1.0, va, vb, 0.0, vc, g, cnt));
  }
  return CTM_OK;
}

// Y <- Y R^{-1} with R from the shifted Cholesky factor of Y^T Y, `passes`
// times (Cholesky-QR with shifts, as in the projector solver); with keep_r
// (two passes) the product R2 R1 of the factors is left in Rb (b x b).
ctm_status cholqr(ctm_su_s& x, const Chunk& ch, const std::vector<double*>& Y, int passes, bool keep_r) {
  hipStream_t s = x.stream;
  const int b = x.b, m = x.m;
  const double u = 1.1102230246251565e-16;
  for (int pass = 0; pass < passes; ++pass) {
    const double coef = pass == 0 ? 11.0 * ((double)m * b + (double)b * (b + 1)) * u : 4.0 * u;
    std::vector<const double*> A;
    std::vector<double*> C;
    CPtrSet Gp{}, Rc{};
    PtrSet Rp{}, Yp{};
    for (int j = 0; j < ch.cnt; ++j) {
      Inst& I = x.inst[ch.i0 + j];
      A.push_back(Y[j]);
      C.push_back(I.Gb);
      double* R = pass == 0 ? I.Rb1 : I.Rb2;
      Gp.p[j] = I.Gb;
      Rp.p[j] = R;
      Rc.p[j] = R;
      Yp.p[j] = Y[j];
    }
    SOK(gemm64(s, b, b, m, transposed(rowmajor(b)), rowmajor(b), rowmajor(b), A, A, C));
    StatSet none{};
    SCHK(chol_shift_inv(s, b, coef, Gp, Rp, none, ch.cnt, false));
    SCHK(trsm_rows(s, m, b, Yp, Rc, ch.cnt));
  }
  if (keep_r) {
    // R = R2 R1 (both upper triangular)
    std::vector<const double*> A, B;
    std::vector<double*> C;
    for (int j = 0; j < ch.cnt; ++j) {
      Inst& I = x.inst[ch.i0 + j];
      A.push_back(I.Rb2);
      B.push_back(I.Rb1);
      C.push_back(I.Rb);
    }
    SOK(gemm64(s, b, b, b, rowmajor(b), rowmajor(b), rowmajor(b), A, B, C));
  }
  return CTM_OK;
}

// The D leading singular triplets of every theta of the chunk by subspace
// iteration: V (m x b) counter-based normals; six rounds of Y = theta V,
// V = theta^T Y, each orthonormalised; then theta V = Y R, R = U_r S W_r^T
// (Jacobi), left vectors Y U_r, right vectors V W_r (both m x b, into th0
// and thp), values S into St.
ctm_status truncated_svd(ctm_su_s& x, const Chunk& ch, std::vector<double*>& lu, std::vector<double*>& lv) {
  hipStream_t s = x.stream;
  const int b = x.b, m = x.m;
  std::vector<double*> V(ch.cnt), Y(ch.cnt);
  std::vector<const double*> th(ch.cnt), Vc(ch.cnt), Yc(ch.cnt);
  for (int j = 0; j < ch.cnt; ++j) {
    Inst& I = x.inst[ch.i0 + j];
    V[j] = I.Vb;
    Y[j] = I.Yb;
    th[j] = I.th;
    Vc[j] = I.Vb;
    Yc[j] = I.Yb;
    SCHK(randn(s, I.Vb, (int64_t)m * b, 0x5eed5eedull ^ (x.updates * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(ch.i0 + j)));
  }
  for (int round = 0; round < 6; ++round) {
    SOK(gemm64(s, m, b, m, rowmajor(m), rowmajor(b), rowmajor(b), th, Vc, Y));
    SOK(cholqr(x, ch, Y, 1, false));
    SOK(gemm64(s, m, b, m, transposed(rowmajor(m)), rowmajor(b), rowmajor(b), th, Yc, V));
    SOK(cholqr(x, ch, V, round == 5 ? 2 : 1, false));
  }
  SOK(gemm64(s, m, b, m, rowmajor(m), rowmajor(b), rowmajor(b), th, Vc, Y));
  SOK(cholqr(x, ch, Y, 2, true));
  CPtrSet M{};
  PtrSet U{}, Sv{}, W{}, J{};
  for (int j = 0; j < ch.cnt; ++j) {
    Inst& I = x.inst[ch.i0 + j];
    M.p[j] = I.Rb;
    U.p[j] = I.Ut;
    Sv.p[j] = I.St;
    W.p[j] = I.Wt;
    J.p[j] = I.jw;
  }
  SCHK(jacobi_svd(s, b, M, U, Sv, W, J, ch.cnt, true, false));
  std::vector<const double*> Ur(ch.cnt), Wr(ch.cnt);
  for (int j = 0; j < ch.cnt; ++j) {
    Inst& I = x.inst[ch.i0 + j];
    Ur[j] = I.Ut;
    Wr[j] = I.Wt;
    lu[j] = I.th0;
    lv[j] = I.thp;
  }
  SOK(gemm64(s, m, b, b, rowmajor(b), rowmajor(b), rowmajor(b), Yc, Ur, lu));
  SOK(gemm64(s, m, b, b, rowmajor(b), rowmajor(b), rowmajor(b), Vc, Wr, lv));
  return CTM_OK;
}

ctm_status bond_update(ctm_su_s& x, int bond, bool reset) {
  hipStream_t s = x.stream;
  const int d = x.d, D = x.D, k = x.k, m = x.m, D3 = x.D3, r = x.r;
  const int64_t t5 = (int64_t)d * D * D * D * D;
  const dim3 blk(256);
  ++x.updates;
  for (const Chunk& ch : chunks(x.n)) {
    auto tab = [&](auto f) {
      Ptrs p{};
      for (int j = 0; j < ch.cnt; ++j) p.p[j] = f(x.inst[ch.i0 + j]);
      return p;
    };
    Ptrs L[NB];
    for (int b = 0; b < NB; ++b) L[b] = tab([&](Inst& I) { return I.lam[b]; });
    const Ptrs lamb = L[bond];
    // reduced tensors of both ends
    for (int e = 0; e < 2; ++e) {
      const int t = END_T[bond][e], leg = END_L[bond][e];
      Ptrs T = tab([&](Inst& I) { return I.T[t]; });
      Ptrs Xm = tab([&](Inst& I) { return I.Xm[e]; });
      for (int j = 0; j < ch.cnt; ++j)
        SCHK(check_spans({{T.p[j], (size_t)t5 * 8}, {Xm.p[j], (size_t)D3 * k * 8}}, "su prep"));
      if (!dry_run())
        hipLaunchKernelGGL(su_prep_kernel, dim3((unsigned)std::min<int64_t>(1024, (t5 + 255) / 256), ch.cnt), blk,
                           0, s, T, L[0], L[1], L[2], L[3], Xm, t, leg, d, D);
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
      std::vector<const double*> A, B;
      std::vector<double*> C;
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        A.push_back(I.Xm[e]);
        B.push_back(I.Xm[e]);
        C.push_back(I.Gm[e]);
      }
      // G = Xm^T Xm
      SOK(gemm64(s, k, k, D3, transposed(rowmajor(k)), rowmajor(k), rowmajor(k), A, B, C));
      CPtrSet Gp{};
      PtrSet U{}, Sv{}, W{}, J{};
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        Gp.p[j] = I.Gm[e];
        U.p[j] = I.Ug[e];
        Sv.p[j] = I.Sg[e];
        W.p[j] = I.Wg[e];
        J.p[j] = I.jw;
      }
      SCHK(jacobi_svd(s, k, Gp, U, Sv, W, J, ch.cnt, true, false));
      Ptrs Wp = tab([&](Inst& I) { return I.Wg[e]; });
      Ptrs Sp = tab([&](Inst& I) { return I.Sg[e]; });
      Ptrs Rp = tab([&](Inst& I) { return I.Rr[e]; });
      Ptrs Pp = tab([&](Inst& I) { return I.Pinv[e]; });
      if (!dry_run()) {
        hipLaunchKernelGGL(su_rfactor_kernel, dim3((unsigned)std::max(1, std::min(64, (k * k + 255) / 256)), ch.cnt),
                           blk, 0, s, Wp, Sp, Rp, Pp, k);
        if (e == 0)
          hipLaunchKernelGGL(su_scale_bond_kernel, dim3((unsigned)std::max(1, std::min(64, (k * k + 255) / 256)),
                                                        ch.cnt), blk, 0, s, Rp, lamb, k, D);
      }
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
    }
    // theta0[(a,i),(b,j)] = sum_p (R_X lam)[(a,i),p] R_Y[(b,j),p], a, b < r
    {
      std::vector<const double*> A, B;
      std::vector<double*> C;
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        A.push_back(I.Rr[0]);
        B.push_back(I.Rr[1]);
        C.push_back(I.th0);
      }
      SOK(gemm64(s, m, m, D, rowmajor(D), transposed(rowmajor(D)), rowmajor(m), A, B, C));
    }
    // gate: [a][k][b][l] -> [(k,l)][(a,b)], times g, back to [a][i][b][j]
    {
      const int64_t dims1[4] = {r, d, r, d};
      const int perm1[4] = {1, 3, 0, 2};
      const int64_t dims2[4] = {d, d, r, r};
      const int perm2[4] = {2, 0, 3, 1};
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        SCHK(permute(s, F64, I.th0, F64, I.thp, 4, dims1, perm1));
      }
      std::vector<const double*> A, B;
      std::vector<double*> C;
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        A.push_back(I.gate[bond]);
        B.push_back(I.thp);
        C.push_back(I.th0);
      }
      SOK(gemm64(s, (int64_t)d * d, (int64_t)r * r, (int64_t)d * d, rowmajor((int64_t)d * d),
                 rowmajor((int64_t)r * r), rowmajor((int64_t)r * r), A, B, C));
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        SCHK(permute(s, F64, I.th0, F64, I.th, 4, dims2, perm2));
      }
    }
    // the D leading singular triplets of theta: left vectors in `lu`, right
    // vectors in `lv` (row stride ldu), values in St (descending)
    std::vector<double*> lu(ch.cnt), lv(ch.cnt);
    int ldu = m;
    if (x.b == 0) {
      CPtrSet M{};
      PtrSet U{}, Sv{}, W{}, J{};
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        M.p[j] = I.th;
        U.p[j] = I.Ut;
        Sv.p[j] = I.St;
        W.p[j] = I.Wt;
        J.p[j] = I.jw;
        lu[j] = I.Ut;
        lv[j] = I.Wt;
      }
      SCHK(jacobi_svd(s, m, M, U, Sv, W, J, ch.cnt, true, false));
    } else {
      SOK(truncated_svd(x, ch, lu, lv));
      ldu = x.b;
    }
    {
      Ptrs St = tab([&](Inst& I) { return I.St; });
      Ptrs Ch = tab([&](Inst& I) { return I.change; });
      Ptrs Lu{}, Lv{};
      for (int j = 0; j < ch.cnt; ++j) {
        Lu.p[j] = lu[j];
        Lv.p[j] = lv[j];
      }
      Ptrs R0 = tab([&](Inst& I) { return I.Rn[0]; });
      Ptrs R1 = tab([&](Inst& I) { return I.Rn[1]; });
      for (int j = 0; j < ch.cnt; ++j)
        SCHK(check_spans({{St.p[j], (size_t)D * 8}, {lamb.p[j], (size_t)D * 8}, {Ch.p[j], 8},
                          {Lu.p[j], (size_t)m * ldu * 8}, {Lv.p[j], (size_t)m * ldu * 8}}, "su weights"));
      if (!dry_run()) {
        hipLaunchKernelGGL(su_weights_kernel, dim3(ch.cnt), dim3(64), 0, s, St, lamb, Ch, D, reset ? 1 : 0);
        const dim3 g((unsigned)std::max(1, std::min(64, (k * k + 255) / 256)), ch.cnt);
        hipLaunchKernelGGL(su_newr_kernel, g, blk, 0, s, Lu, lamb, R0, k, d, D, ldu, r);
        hipLaunchKernelGGL(su_newr_kernel, g, blk, 0, s, Lv, lamb, R1, k, d, D, ldu, r);
      }
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
    }
    // X' = Xm (Pinv R'), weights of the other legs out, normalised
    for (int e = 0; e < 2; ++e) {
      std::vector<const double*> A, B, A2, B2;
      std::vector<double*> C, C2;
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x.inst[ch.i0 + j];
        A.push_back(I.Pinv[e]);
        B.push_back(I.Rn[e]);
        C.push_back(I.S1[e]);
        A2.push_back(I.Xm[e]);
        B2.push_back(I.S1[e]);
        C2.push_back(I.Xn[e]);
      }
      SOK(gemm64(s, k, k, k, rowmajor(k), rowmajor(k), rowmajor(k), A, B, C));
      SOK(gemm64(s, D3, k, k, rowmajor(k), rowmajor(k), rowmajor(k), A2, B2, C2));
      const int t = END_T[bond][e], leg = END_L[bond][e];
      Ptrs Xn = tab([&](Inst& I) { return I.Xn[e]; });
      Ptrs T = tab([&](Inst& I) { return I.T[t]; });
      if (!dry_run())
        hipLaunchKernelGGL(su_finish_kernel, dim3((unsigned)std::min<int64_t>(1024, (t5 + 255) / 256), ch.cnt), blk,
                           0, s, Xn, L[0], L[1], L[2], L[3], T, t, leg, d, D);
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
      for (int j = 0; j < ch.cnt; ++j) {
        NormSet ns{};
        ns.p[0] = x.inst[ch.i0 + j].T[t];
        ns.n[0] = t5;
        SCHK(normalize_group(s, ns, 1, x.inst[ch.i0 + j].norm_part));
      }
    }
  }
  return CTM_OK;
}

ctm_status build(int n, int d, int D, ctm_su_s& x) {
  if (n < 1 || d < 1 || D < 1 || d > 64 || D > 16) return ctm_internal_fail(CTM_E_INVALID, "n >= 1, d in 1..64, D in 1..16");
  x.n = n;
  x.d = d;
  x.D = D;
  x.k = d * D;
  x.D3 = D * D * D;
  x.r = std::min(x.D3, x.k);
  x.m = x.r * d;
  x.b = x.m <= 80 ? 0 : std::min(x.m, D + 16);
  if (x.k > 192) return ctm_internal_fail(CTM_E_INVALID, "d D must be <= 192 (reduced-tensor factor size)");
  if (x.m > 4096) return ctm_internal_fail(CTM_E_INVALID, "min(D^3, d D) d must be <= 4096");
  if (d * d > 192) return ctm_internal_fail(CTM_E_INVALID, "d^2 must be <= 192 (gate eigensolver size)");
  Carve c;
  plan(x, c);
  x.ws_need = c.off + 256;
  return CTM_OK;
}

}  // namespace

extern "C" {

ctm_status ctm_su_workspace_size(int32_t n_inst, int32_t d, int32_t D, size_t* bytes) {
  if (!bytes) return ctm_internal_fail(CTM_E_INVALID, "null bytes");
  ctm_su_s x;
  SOK(build(n_inst, d, D, x));
  *bytes = x.ws_need;
  return CTM_OK;
}

ctm_status ctm_su_init(int32_t n_inst, int32_t d, int32_t D, const double* T_dev, const double* lam_dev, void* ws,
                       size_t ws_bytes, void* stream, ctm_su* out) {
  if (!out || !T_dev || !lam_dev || !ws) return ctm_internal_fail(CTM_E_INVALID, "null argument");
  *out = nullptr;
  ctm_su_s* x = new ctm_su_s();
  ctm_status st = build(n_inst, d, D, *x);
  if (st != CTM_OK) { delete x; return st; }
  if (ws_bytes < x->ws_need || ((uintptr_t)ws & 255)) {
    delete x;
    return ctm_internal_fail(ws_bytes < x->ws_need ? CTM_E_NOMEM : CTM_E_INVALID,
                             "workspace too small or not 256-byte aligned");
  }
  x->stream = (hipStream_t)stream;
  const char* dr = std::getenv("CTM_DRY_RUN");
  x->reg.dry = dr && dr[0] == '1';
  x->reg.lo = (uintptr_t)ws;
  x->reg.hi = (uintptr_t)ws + x->ws_need;
  Carve c;
  c.base = (char*)ws;
  c.reg = &x->reg;
  plan(*x, c);
  std::sort(x->reg.allocs.begin(), x->reg.allocs.end());
  RegScope rs(&x->reg);
  const size_t t5 = (size_t)d * D * D * D * D;
  for (int i = 0; i < n_inst; ++i) {
    Inst& I = x->inst[i];
    for (int t = 0; t < 2; ++t) {
      if (!span_ok(I.T[t], t5 * 8, "su tensors")) { delete x; return ctm_internal_fail(CTM_E_INVALID, "bounds"); }
      if (!dry_run() && hipMemcpyAsync(I.T[t], T_dev + ((size_t)i * 2 + t) * t5, t5 * 8, hipMemcpyDeviceToDevice,
                                       x->stream) != hipSuccess) {
        delete x;
        return ctm_internal_fail(CTM_E_HIP, "tensor copy");
      }
    }
    for (int b = 0; b < NB; ++b)
      if (!dry_run() && hipMemcpyAsync(I.lam[b], lam_dev + ((size_t)i * NB + b) * D, (size_t)D * 8,
                                       hipMemcpyDeviceToDevice, x->stream) != hipSuccess) {
        delete x;
        return ctm_internal_fail(CTM_E_HIP, "weight copy");
      }
  }
  *out = x;
  return CTM_OK;
}

ctm_status ctm_su_set_gates(ctm_su x, const double* h_dev, double dtau) {
  if (!x || !h_dev || !(dtau >= 0)) return ctm_internal_fail(CTM_E_INVALID, "args");
  RegScope rs(&x->reg);
  hipStream_t s = x->stream;
  const int dd = x->d * x->d;
  const size_t d4 = (size_t)dd * dd;
  // bond Hamiltonians [n][4][d^2][d^2] -> gates; each instance has one set of
  // gate scratch, so the passes go bond by bond
  for (int b = 0; b < NB; ++b) {
    for (const Chunk& ch : chunks(x->n)) {
      Ptrs h{}, hs{}, gU{}, gW{}, gS{}, G{};
      CPtrSet Hc{};
      PtrSet U{}, S{}, W{}, J{};
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x->inst[ch.i0 + j];
        h.p[j] = const_cast<double*>(h_dev) + ((size_t)(ch.i0 + j) * NB + b) * d4;
        hs.p[j] = I.hs;
        gU.p[j] = I.gU;
        gW.p[j] = I.gW;
        gS.p[j] = I.gS;
        G.p[j] = I.gate[b];
        Hc.p[j] = I.hs;
        U.p[j] = I.gU;
        S.p[j] = I.gS;
        W.p[j] = I.gW;
        J.p[j] = I.jw;
        SCHK(check_spans({{I.hs, (d4 + 1) * 8}, {I.gU, d4 * 8}, {I.gW, d4 * 8}, {I.gS, (size_t)dd * 8}}, "su gates"));
      }
      if (!dry_run()) hipLaunchKernelGGL(su_shift_kernel, dim3(ch.cnt), dim3(256), 0, s, h, hs, dd);
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
      SCHK(jacobi_svd(s, dd, Hc, U, S, W, J, ch.cnt, true, false));
      // gU <- W exp(-dtau (e - c)), then g = gU W^T
      if (!dry_run()) hipLaunchKernelGGL(su_gate_scale_kernel, dim3(ch.cnt), dim3(256), 0, s, gW, gS, hs, gU, dd, dtau);
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
      std::vector<const double*> A, B;
      std::vector<double*> C;
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x->inst[ch.i0 + j];
        A.push_back(I.gU);
        B.push_back(I.gW);
        C.push_back(I.gate[b]);
      }
      SOK(gemm64(s, dd, dd, dd, rowmajor(dd), transposed(rowmajor(dd)), rowmajor(dd), A, B, C));
    }
  }
  SCHK(dry_run() ? hipSuccess : hipStreamSynchronize(s));
  return CTM_OK;
}

ctm_status ctm_su_evolve(ctm_su x, int32_t max_steps, double tol, int32_t check_every, int32_t* steps_out,
                         double* change_out) {
  if (!x || max_steps < 0 || !(tol >= 0)) return ctm_internal_fail(CTM_E_INVALID, "args");
  RegScope rs(&x->reg);
  if (check_every < 1) check_every = 1;
  std::vector<double> ch(x->n, INFINITY);
  int steps = 0;
  while (steps < max_steps) {
    for (int b = 0; b < NB; ++b) SOK(bond_update(*x, b, b == 0));
    ++steps;
    if (steps % check_every == 0 || steps == max_steps) {
      for (int i = 0; i < x->n; ++i) {
        if (!span_ok(x->inst[i].change, 8, "su change")) return ctm_internal_fail(CTM_E_INVALID, "bounds");
        if (dry_run()) ch[i] = 0.0;
        else SCHK(hipMemcpyAsync(&ch[i], x->inst[i].change, 8, hipMemcpyDeviceToHost, x->stream));
      }
      SCHK(dry_run() ? hipSuccess : hipStreamSynchronize(x->stream));
      bool all = true;
      for (double c : ch) all = all && c < tol;
      if (all) break;
    }
  }
  if (steps_out) *steps_out = steps;
  if (change_out)
    for (int i = 0; i < x->n; ++i) change_out[i] = ch[i];
  for (double c : ch)
    if (!std::isfinite(c)) return ctm_internal_fail(CTM_E_NONFINITE, "non-finite bond weights");
  return CTM_OK;
}

ctm_status ctm_su_state(ctm_su x, double* T_out_dev, double* lam_out_dev) {
  if (!x) return ctm_internal_fail(CTM_E_INVALID, "null su");
  RegScope rs(&x->reg);
  const size_t t5 = (size_t)x->d * x->D * x->D * x->D * x->D;
  for (int i = 0; i < x->n; ++i) {
    Inst& I = x->inst[i];
    if (T_out_dev)
      for (int t = 0; t < 2; ++t)
        SCHK(dry_run() ? hipSuccess
                       : hipMemcpyAsync(T_out_dev + ((size_t)i * 2 + t) * t5, I.T[t], t5 * 8, hipMemcpyDeviceToDevice,
                                        x->stream));
    if (lam_out_dev)
      for (int b = 0; b < NB; ++b)
        SCHK(dry_run() ? hipSuccess
                       : hipMemcpyAsync(lam_out_dev + ((size_t)i * NB + b) * x->D, I.lam[b], (size_t)x->D * 8,
                                        hipMemcpyDeviceToDevice, x->stream));
  }
  SCHK(dry_run() ? hipSuccess : hipStreamSynchronize(x->stream));
  return CTM_OK;
}

ctm_status ctm_su_peps(ctm_su x, double* A_out_dev) {
  if (!x || !A_out_dev) return ctm_internal_fail(CTM_E_INVALID, "args");
  RegScope rs(&x->reg);
  const int64_t t5 = (int64_t)x->d * x->D * x->D * x->D * x->D;
  for (const Chunk& ch : chunks(x->n))
    for (int t = 0; t < 2; ++t) {
      Ptrs T{}, L[NB] = {}, O{};
      for (int j = 0; j < ch.cnt; ++j) {
        Inst& I = x->inst[ch.i0 + j];
        T.p[j] = I.T[t];
        for (int b = 0; b < NB; ++b) L[b].p[j] = I.lam[b];
        O.p[j] = A_out_dev + ((size_t)(ch.i0 + j) * 2 + t) * t5;
      }
      if (!dry_run())
        hipLaunchKernelGGL(su_peps_kernel, dim3((unsigned)std::min<int64_t>(1024, (t5 + 255) / 256), ch.cnt),
                           dim3(256), 0, x->stream, T, L[0], L[1], L[2], L[3], O, t, x->d, x->D);
      SCHK(dry_run() ? hipSuccess : hipGetLastError());
    }
  SCHK(dry_run() ? hipSuccess : hipStreamSynchronize(x->stream));
  return CTM_OK;
}

void ctm_su_destroy(ctm_su x) { delete x; }

}  // extern "C"
