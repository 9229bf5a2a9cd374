// Host orchestration and C ABI of the gfx950 CTM library.
//
// Method (paper Sec. II C, captions of Figs. 3 and 4; Sec. III): directional
// corner-transfer-matrix renormalisation of the double-layer network around
// an Lx x Ly cell.  A move in direction k (0 = L, 1 = U, 2 = R, 3 = D) is the
// left move of the picture turned by k counter-clockwise quarter turns: the
// environment tensors keep their clockwise leg order, so turning only relabels
// which stored corner/edge plays which role and which rotated copy of the
// double-layer tensor is used (the rotated copies are built once).
//
// Storage (all row-major, float64 master copies):
//   A[s][u][l][d][r]                   PEPS tensors (ket A, bra B)
//   b_k[L'][U'][D'][R']                double layer turned by k quarter turns,
//                                      laid out as a (L',U') x (D',R') matrix
//   C_i[prev][next]    (chi x chi)     corner i at each site
//   T_i[prev][inner][next] (chi x D^2 x chi)
//   Q   [cut_in][cut_out]  (n x n, n = chi D^2) enlarged corner, cut = (chi, D^2)
#include "ctm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <string>
#include <array>
#include <vector>
#include <chrono>

#include "ctm_internal.h"
#include "kernels.h"
#include "solver.h"

using namespace ctmk;

namespace {

thread_local std::string g_err;

ctm_status fail(ctm_status s, const std::string& m) {
  g_err = m;
  return s;
}

ctm_status hip_fail(hipError_t e, const char* what) {
  if (ctmk::g_reg && ctmk::g_reg->last && ctmk::g_reg->violations)
    return fail(CTM_E_INVALID, std::string("internal bounds check failed (") + ctmk::g_reg->last + ") in " + what);
  return fail(CTM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return hip_fail(e_, #x);                                       \
  } while (0)

#define CHK(x)                          \
  do {                                  \
    ctm_status s_ = (x);                \
    if (s_ != CTM_OK) return s_;        \
  } while (0)

struct RegGuard {
  Registry* prev;
  explicit RegGuard(Registry* r) : prev(g_reg) { g_reg = r; }
  ~RegGuard() { g_reg = prev; }
};

struct TuneGuard {
  explicit TuneGuard(bool on) { set_tuning(on); }
  ~TuneGuard() { set_tuning(false); }
};

hipError_t d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!span_ok(dst, bytes, "copy dst") || !span_ok(src, bytes, "copy src")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}
hipError_t d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!span_ok(src, bytes, "readback src")) return hipErrorInvalidValue;
  if (dry_run()) { std::memset(dst, 0, bytes); return hipSuccess; }
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
}
hipError_t h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!span_ok(dst, bytes, "upload dst")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
}
hipError_t dmemset(void* p, int v, size_t bytes, hipStream_t s) {
  if (!span_ok(p, bytes, "memset")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  return hipMemsetAsync(p, v, bytes, s);
}
hipError_t last_err() { return dry_run() ? hipSuccess : hipGetLastError(); }
hipError_t ssync(hipStream_t s) {
  if (dry_run()) return hipSuccess;
  return hipStreamSynchronize(s);
}
hipError_t spans(std::initializer_list<std::pair<const void*, size_t>> l, const char* what) {
  for (auto& e : l)
    if (!span_ok(e.first, e.second, what)) return hipErrorInvalidValue;
  return hipSuccess;
}

constexpr int MAXT = 4;     // distinct tensors per instance
constexpr int MAXPOS = 16;  // sites per cell (Lx, Ly <= 4)
constexpr int MAXROWS = 4;  // rows per column step

// ---------------------------------------------------------------------------
// workspace arena: the same code path sizes (dry run) and assigns the buffers
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  Registry* reg = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    if (reg && base && count) reg->allocs.emplace_back((uintptr_t)p, count * sizeof(T));
    off += count * sizeof(T);
    return p;
  }
  void* take_bytes(size_t bytes) { return take<char>(bytes); }
};

struct Row {  // scratch for one row of a column step
  void* Q[4] = {};
  void* X[4] = {};
  void* Y[4] = {};
  double *V = nullptr, *Yb = nullptr, *Qb = nullptr, *Z = nullptr, *LV = nullptr, *UU = nullptr,
         *Ub = nullptr, *Vp = nullptr, *tmp = nullptr;
  void *qin = nullptr, *q1 = nullptr, *q2 = nullptr;  // N-apply scratch in the Q type
  double *G = nullptr, *Rinv = nullptr, *Rm = nullptr, *UR = nullptr, *WR = nullptr,
         *S = nullptr, *Wp = nullptr, *Up = nullptr, *jw = nullptr;
  SolveStatus* st = nullptr;
  double *P1 = nullptr, *P2T = nullptr;
  void *P1w = nullptr, *P2Tw = nullptr;
  void *CT = nullptr, *W1 = nullptr, *W2 = nullptr, *X6 = nullptr;
  void* A3 = nullptr;  // bf16 mode: [hi | hi | lo] split of W1 for the three-term product
  void* T3s = nullptr; // bf16 mode: three-term splits of T4 (A side) and P2T (B side) for W1
  void* P3s = nullptr;
  void* W2t = nullptr; // fp32 working type: W2 as [(g,dn)][(R,c2)]
  double *nC1 = nullptr, *nT4 = nullptr, *nC4 = nullptr;
  double *red = nullptr, *sums = nullptr;
};

struct Inst {
  // chi_cap: the environment dimension chi of the configuration (buffers are
  // sized for it); chi: the live extent, the number of leading indices of
  // every corner / edge leg that can be nonzero.  Every kept projector column
  // comes from a subspace of k_act columns, so beyond min(chi_cap, k_act) all
  // entries of C and T are exact zeros; the tensors are stored compactly at
  // the live extent and every contraction runs at it.  n = chi D^2 is the
  // live cut dimension, n_cap = chi_cap D^2.
  int d = 0, D = 0, D2 = 0, chi = 0, n = 0, k = 0;
  int chi_cap = 0, n_cap = 0;
  int k_act = 0;                 // subspace columns in use (<= k, follows chi_eff)
  double* A[MAXT] = {};
  double* B[MAXT] = {};
  double* b64[MAXT][4] = {};
  void* bw[MAXT][4] = {};
  void* bT[MAXT][4] = {};        // bf16 mode: double layer transposed, [(D',R') x (L',U')]
  double* C[4][MAXPOS] = {};
  double* T[4][MAXPOS] = {};
  void* Cw[4][MAXPOS] = {};
  void* Tw[4][MAXPOS] = {};
  void* TwP[4][MAXPOS] = {};     // bf16 mode: edges as [prev][next][inner]
  void* TwR[4][MAXPOS] = {};     // bf16 mode: bf16 edges as [next][inner][prev]
  // working copies (Cw, Tw, TwP, TwR) that no longer match their float64 master
  bool staleC[4][MAXPOS] = {};
  bool staleT[4][MAXPOS] = {};
  void* bT3[MAXT][4] = {};       // bf16 mode: [hi | lo | hi] split of bT, N x 3K
  void* bTp[MAXT][4] = {};       // bf16 mode: bT in the corner kernel's packed fragment layout
  void* bT3p[MAXT][4] = {};      // bf16 mode: bT3 in that layout (the absorption's B operand)
  double* Ac[MAXT] = {};         // complex kets (real, imaginary interleaved)
  // single-layer mode: the ket (Sk) and bra (Sb) tensor of each rotation in
  // the working type, legs [L'][U'][s][D'][R'] of the rotated frame
  void* Sk[MAXT][4] = {};
  void* Sb[MAXT][4] = {};
  void* Sk16[MAXT][4] = {};      // single-layer in CTM_BF16: bf16 copies for the enlarged corners
  void* Sb16[MAXT][4] = {};
  // ... and as operands of the bf16 corner kernel:
  // SkT16[(D',R',s)][(L',U') padded to a multiple of 8], SbT16[(D',R')][(L',U',s)]
  void* SkT16[MAXT][4] = {};
  void* SbT16[MAXT][4] = {};
  double* spec_old = nullptr;  // [pos][4][chi_cap]
  double* spec_new = nullptr;
  double* delta = nullptr;     // device scalar
  int* flag = nullptr;         // device: non-finite flag
  double* Vkeep[4][MAXPOS] = {};
  SolveStatus* skeep[4][MAXPOS] = {};
  SolveStatus* skeep_all = nullptr;  // the statuses above, contiguous [4][npos]
  bool has_keep[4][MAXPOS] = {};
  int cursor[4] = {0, 0, 0, 0};
  uint64_t solves = 0;
  std::vector<Row> rows;        // scratch of the rows of one column step
};

struct Obs {  // float64 scratch of the observables
  double *Q[4] = {}, *X = nullptr, *Y = nullptr, *Uh = nullptr, *LhT = nullptr;
  double *G1 = nullptr, *B1 = nullptr, *H = nullptr, *CT = nullptr, *ab = nullptr;
  double *Lall = nullptr, *Rall = nullptr, *Rp = nullptr;
  double *t0 = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  double *rho = nullptr, *red = nullptr, *vals = nullptr;
  size_t big = 0;
  bool rows_ok = false;  // t0..t3 are large enough for the row-transfer norm
};

}  // namespace

struct ctm_ctx_s {
  ctm_config cfg{};
  std::vector<int> pattern, dv, Dv, chiv;
  int Lx = 1, Ly = 1, ntens = 1, ninst = 1;
  int prec = CTM_FP64;
  int wt = F64, qt = F64;  // contraction operand type, enlarged-corner type
  hipStream_t stream = nullptr;
  std::vector<Inst> inst;
  std::vector<std::vector<int>> classes;  // instances with equal (d, D, chi), moved in lock-step
  Obs obs;
  double* norm_part = nullptr;   // grouped-normalisation partial sums
  double* delta_all = nullptr;   // [n_inst] convergence measure of each instance
  int* flag_all = nullptr;       // [n_inst][4] non-finite flags
  int max_prob = 1;              // largest number of solver problems per launch
  hipGraphExec_t gexec = nullptr;  // captured sweep of every class (graph mode)
  double* splitk = nullptr;      // split-K partial products of the solver
  int64_t splitk_elems = 0;
  void* ts_scratch = nullptr;    // K-chunk partials of the tall-skinny products
  int64_t ts_bytes = 0;
  double* spec_tmp_U = nullptr;  // corner SVD scratch
  double* spec_tmp_W = nullptr;
  double* spec_tmp_S = nullptr;
  double* spec_tmp_J = nullptr;
  void *sl_y = nullptr, *sl_z = nullptr, *sl_p = nullptr;  // single-layer scratch (current set)
  size_t sl_ybytes = 0, sl_zbytes = 0;                      // capacity of sl_y / sl_p and of sl_z
  // the scratch above (split-K partials, tall-skinny partials, normalisation
  // partials, corner SVD) in sets: set 0 serves the eager path, and in graph
  // mode with concurrent classes class i's branch of the captured sweep uses
  // set i; use_scratch() points the fields above at one set
  struct ScratchSet {
    double *splitk, *norm_part, *U, *W, *S, *J;
    void* ts;
    void *sl_y, *sl_z, *sl_p;  // single-layer products: permuted input, intermediate, output
  };
  std::vector<ScratchSet> scratch_sets;
  std::vector<hipStream_t> class_streams;  // branches of the captured sweep
  std::vector<hipEvent_t> class_events;    // fork (0) and joins (1 ..)
  size_t ws_need = 0;
  bool timing = false;
  double t_corner = 0, t_solver = 0, t_absorb = 0, t_stage3 = 0, stage3_flop = 0, stage3_flop_nom = 0;
  int live_chi = 0;
  int64_t corner_launches = 0, stage3_launches = 0, moves = 0;
  // timing (ctm_set_timing): one record of four phase events per timed column
  // step and one event pair per timed stage-3 launch, recorded without waiting
  // and read when timing is queried (a wait per column step would drain the
  // stream between column steps)
  bool phase_timing = false;
  bool resid_step = true;  // fixed-count solver: form the residuals in this column step
  bool width_pinned = false;  // ctm_debug_set_width: the convergence loop keeps the width
  // ctm_set_metrics: one JSON line per instance and convergence check
  std::FILE* metrics = nullptr;
  bool metrics_own = false;
  int metrics_flags = 0;
  std::vector<std::array<hipEvent_t, 4>> tpool;
  std::vector<std::array<hipEvent_t, 2>> spool;
  size_t tused = 0, sused = 0;
  Registry reg;
};

namespace {

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
// working type of corners, edges, projectors and every contraction except
// the double-layer stage of the enlarged corners, which is bf16 in CTM_BF16
int wtype_of(int prec) { return prec == CTM_FP64 ? F64 : F32; }
int qtype_of(int prec) { return prec == CTM_FP64 ? F64 : F32; }

int subspace_dim(const ctm_config& c, int chi, int n) {
  int p = c.svd_oversample > 0 ? c.svd_oversample : 0;
  return std::min(n, chi + p);
}

// graph mode with several shape classes: each class's sweep is a concurrent
// branch of the captured graph, with a scratch set of its own
bool concurrent_classes(const ctm_ctx_s& x) {
  return x.cfg.use_graph && x.cfg.concurrent_classes && x.classes.size() > 1;
}

void use_scratch(ctm_ctx_s& x, size_t i) {
  const auto& ss = x.scratch_sets[i];
  x.splitk = ss.splitk;
  x.ts_scratch = ss.ts;
  x.norm_part = ss.norm_part;
  x.spec_tmp_U = ss.U;
  x.spec_tmp_W = ss.W;
  x.spec_tmp_S = ss.S;
  x.spec_tmp_J = ss.J;
  x.sl_y = ss.sl_y;
  x.sl_z = ss.sl_z;
  x.sl_p = ss.sl_p;
}

void plan_row(ctm_ctx_s& x, Arena& ar, const Inst& I, Row& R) {
  const size_t ws = dtype_size(x.wt), qs = dtype_size(x.qt);
  const size_t n = I.n_cap, k = I.k, chi = I.chi_cap, D2 = I.D2;
  const size_t nk = n * k, c2 = chi * chi, t3 = c2 * D2, y4 = t3 * D2;
  for (int q = 0; q < 4; ++q) {
    R.Q[q] = ar.take_bytes(n * n * qs);
    R.X[q] = ar.take_bytes(t3 * ws);
    // bf16: also room for Y in the corner kernel's packed layout
    R.Y[q] = ar.take_bytes(x.prec == CTM_BF16
                               ? std::max(y4 * ws, (size_t)corner_bf16_packed_a_elems(c2, D2 * D2) * 2)
                               : y4 * ws);
  }
  R.V = ar.take<double>(nk); R.Yb = ar.take<double>(nk); R.Qb = ar.take<double>(nk);
  R.Z = ar.take<double>(nk); R.LV = ar.take<double>(nk); R.UU = ar.take<double>(nk);
  R.Ub = ar.take<double>(nk); R.Vp = ar.take<double>(nk); R.tmp = ar.take<double>(nk);
  if (x.qt != F64) {
    R.qin = ar.take_bytes(nk * qs); R.q1 = ar.take_bytes(nk * qs); R.q2 = ar.take_bytes(nk * qs);
  }
  R.G = ar.take<double>(k * k); R.Rinv = ar.take<double>(k * k); R.Rm = ar.take<double>(k * k);
  R.UR = ar.take<double>(k * k); R.WR = ar.take<double>(k * k); R.S = ar.take<double>(k);
  R.Wp = ar.take<double>(k * chi); R.Up = ar.take<double>(k * chi); R.jw = ar.take<double>(3 * k * k);
  R.st = ar.take<SolveStatus>(1);
  R.P1 = ar.take<double>(n * chi); R.P2T = ar.take<double>(n * chi);
  R.P1w = (x.wt == F64) ? (void*)R.P1 : ar.take_bytes(n * chi * ws);
  R.P2Tw = (x.wt == F64) ? (void*)R.P2T : ar.take_bytes(n * chi * ws);
  R.CT = ar.take_bytes(t3 * ws); R.W1 = ar.take_bytes(y4 * ws); R.W2 = ar.take_bytes(y4 * ws);
  R.X6 = ar.take_bytes(t3 * ws);
  if (x.prec == CTM_BF16 && !x.cfg.single_layer) {
    R.A3 = ar.take_bytes(3 * y4 * dtype_size(BF16));
    R.T3s = ar.take_bytes(3 * t3 * dtype_size(BF16));
    R.P3s = ar.take_bytes(3 * t3 * dtype_size(BF16));
  }
  if (x.wt == F32) R.W2t = ar.take_bytes(y4 * ws);
  R.nC1 = ar.take<double>(c2); R.nT4 = ar.take<double>(t3); R.nC4 = ar.take<double>(c2);
}

void plan(ctm_ctx_s& x, Arena& ar) {
  const int npos = x.Lx * x.Ly;
  const size_t ws = dtype_size(x.wt);
  const int rows = std::max(x.Lx, x.Ly);
  size_t mx_n = 0, mx_k = 0, mx_chi = 0, mx_D2 = 0, mx_d = 0;
  for (int i = 0; i < x.ninst; ++i) {
    Inst& I = x.inst[i];
    mx_n = std::max(mx_n, (size_t)I.n_cap);
    mx_k = std::max(mx_k, (size_t)I.k);
    mx_chi = std::max(mx_chi, (size_t)I.chi_cap);
    mx_D2 = std::max(mx_D2, (size_t)I.D2);
    mx_d = std::max(mx_d, (size_t)I.d);
  }
  x.delta_all = ar.take<double>((size_t)x.ninst);
  x.flag_all = ar.take<int>((size_t)4 * x.ninst);
  for (int i = 0; i < x.ninst; ++i) {
    Inst& I = x.inst[i];
    const size_t t5 = (size_t)I.d * I.D2 * I.D2;
    const size_t a8 = (size_t)I.D2 * I.D2 * I.D2 * I.D2;
    const size_t c2 = (size_t)I.chi_cap * I.chi_cap, t3 = c2 * I.D2;
    for (int t = 0; t < x.ntens; ++t) {
      I.A[t] = ar.take<double>(t5);
      I.B[t] = ar.take<double>(t5);
      if (x.cfg.complex_tensors) I.Ac[t] = ar.take<double>(2 * t5);
      for (int r = 0; r < 4; ++r) {
        I.b64[t][r] = ar.take<double>(a8);
        // the single-layer mode contracts with Sk / Sb instead of a working copy
        I.bw[t][r] = (x.wt == F64) ? (void*)I.b64[t][r] : (x.cfg.single_layer ? nullptr : ar.take_bytes(a8 * ws));
        if (x.cfg.single_layer) {
          I.Sk[t][r] = ar.take_bytes(t5 * ws);
          I.Sb[t][r] = ar.take_bytes(t5 * ws);
          if (x.prec == CTM_BF16) {
            I.Sk16[t][r] = ar.take_bytes(t5 * dtype_size(BF16));
            I.Sb16[t][r] = ar.take_bytes(t5 * dtype_size(BF16));
            const size_t kp = ((size_t)I.D2 + 7) / 8 * 8;
            I.SkT16[t][r] = ar.take_bytes((size_t)I.d * I.D2 * kp * dtype_size(BF16));
            I.SbT16[t][r] = ar.take_bytes(t5 * dtype_size(BF16));
          }
        }
        if (x.prec == CTM_BF16 && !x.cfg.single_layer) {
          I.bT[t][r] = ar.take_bytes(a8 * dtype_size(BF16));
          I.bT3[t][r] = ar.take_bytes(3 * a8 * dtype_size(BF16));
          const int64_t K4 = (int64_t)I.D2 * I.D2;
          if (K4 % 8 == 0) {
            I.bTp[t][r] = ar.take_bytes((size_t)corner_bf16_packed_b_elems(K4, K4) * 2);
            I.bT3p[t][r] = ar.take_bytes((size_t)corner_bf16_packed_b_elems(K4, 3 * K4) * 2);
          }
        }
      }
    }
    for (int c = 0; c < 4; ++c)
      for (int p = 0; p < npos; ++p) {
        I.C[c][p] = ar.take<double>(c2);
        I.T[c][p] = ar.take<double>(t3);
        I.staleC[c][p] = I.staleT[c][p] = true;
        I.Cw[c][p] = (x.wt == F64) ? (void*)I.C[c][p] : ar.take_bytes(c2 * ws);
        I.Tw[c][p] = (x.wt == F64) ? (void*)I.T[c][p] : ar.take_bytes(t3 * ws);
        if (x.prec == CTM_BF16) {
          I.TwP[c][p] = ar.take_bytes(t3 * ws);
          I.TwR[c][p] = ar.take_bytes(t3 * dtype_size(BF16));
        }
      }
    I.spec_old = ar.take<double>((size_t)npos * 4 * I.chi_cap);
    I.spec_new = ar.take<double>((size_t)npos * 4 * I.chi_cap);
    I.delta = x.delta_all ? x.delta_all + i : nullptr;
    I.flag = x.flag_all ? x.flag_all + 4 * i : nullptr;
    I.skeep_all = ar.take<SolveStatus>((size_t)4 * npos);
    for (int c = 0; c < 4; ++c)
      for (int p = 0; p < npos; ++p) {
        I.Vkeep[c][p] = ar.take<double>((size_t)I.n_cap * I.k);
        I.skeep[c][p] = I.skeep_all ? I.skeep_all + c * npos + p : nullptr;
      }
    // row scratch of this instance (all instances of a class step together)
    I.rows.assign(rows, Row());
    for (int r = 0; r < rows; ++r) plan_row(x, ar, I, I.rows[r]);
  }
  // problems per solver launch: every row of every instance of a class, at most MAXP
  x.max_prob = 1;
  for (auto& cls : x.classes) x.max_prob = std::max(x.max_prob, std::min<int>(MAXP, (int)cls.size() * rows));
  const size_t n = mx_n, k = mx_k, chi = mx_chi, D2 = mx_D2;
  const size_t c2 = chi * chi, t3 = c2 * D2, y4 = t3 * D2;
  // split-K partials of the k x n x k products (all problems of a launch)
  x.splitk_elems = (int64_t)64 * k * k * x.max_prob;
  // K-chunk partials of the tall-skinny products (n x k and chi x chi outputs)
  {
    const int64_t cols = (int64_t)std::max(k, chi);
    const int64_t want = (int64_t)16 * (int64_t)std::max(n, chi) * cols * std::min(MAXG, x.max_prob) * 8;
    x.ts_bytes = std::min<int64_t>(want, (int64_t)256 << 20);
  }
  // corner-spectrum SVD scratch (MAXP corners per launch)
  // (the Jacobi kernel's working set with vectors: 2 chi chi16 per problem)
  const size_t chi16 = (chi + 15) / 16 * 16;
  // single-layer products at the full extent: as many jobs per pass as fit
  // 1 GiB of intermediates, at least one
  if (x.cfg.single_layer) {
    size_t yb = 0, zb = 0;
    for (const Inst& I : x.inst) {
      const size_t y = (size_t)I.chi_cap * I.chi_cap * I.D2 * I.D2 * ws;
      yb = std::max(yb, y);
      zb = std::max(zb, y * (size_t)I.d);
    }
    const size_t per = 2 * yb + zb;
    const size_t nb = std::max<size_t>(1, std::min<size_t>(MAXG, ((size_t)1 << 30) / std::max<size_t>(per, 1)));
    x.sl_ybytes = nb * yb;
    x.sl_zbytes = nb * zb;
  }
  const size_t nsets = concurrent_classes(x) ? x.classes.size() : 1;
  x.scratch_sets.assign(nsets, ctm_ctx_s::ScratchSet{});
  for (auto& ss : x.scratch_sets) {
    ss.splitk = ar.take<double>((size_t)x.splitk_elems);
    ss.ts = ar.take_bytes((size_t)x.ts_bytes);
    ss.norm_part = ar.take<double>((size_t)MAXJ * 64);
    ss.U = ar.take<double>(MAXP * c2);
    ss.W = ar.take<double>(MAXP * c2);
    ss.S = ar.take<double>(MAXP * chi);
    ss.J = ar.take<double>(MAXP * 2 * chi * chi16);
    ss.sl_y = ss.sl_z = ss.sl_p = nullptr;
    if (x.cfg.single_layer) {
      ss.sl_y = ar.take_bytes(x.sl_ybytes);
      ss.sl_z = ar.take_bytes(x.sl_zbytes);
      ss.sl_p = ar.take_bytes(x.sl_ybytes);
    }
  }
  use_scratch(x, 0);
  // observables (float64)
  const size_t d = mx_d, a8 = D2 * D2 * D2 * D2;
  Obs& O = x.obs;
  const bool plaq = (x.Lx >= 2 && x.Ly >= 2);
  if (plaq) {
    for (int q = 0; q < 4; ++q) O.Q[q] = ar.take<double>(n * n);
    O.Uh = ar.take<double>(n * n);
    O.LhT = ar.take<double>(n * n);
  }
  O.X = ar.take<double>(t3);
  O.Y = ar.take<double>(y4);
  O.G1 = ar.take<double>(y4);
  O.B1 = ar.take<double>(t3);
  O.H = ar.take<double>(y4);
  O.CT = ar.take<double>(t3);
  O.ab = ar.take<double>(4 * a8);
  O.Lall = ar.take<double>(d * d * t3);
  O.Rall = ar.take<double>(d * d * t3);
  O.Rp = ar.take<double>(d * d * t3);
  size_t big = std::max(y4, c2 * (size_t)std::pow((double)D2, (double)std::max(x.Lx, x.Ly)));
  // the norm per site of cells other than 1x1 and 2x2 goes through row
  // transfer (chi^2 D^(2 Lx + 2) entries), planned when that stays below
  // 2^28 doubles per buffer
  const bool square12 = (x.Lx == 1 && x.Ly == 1) || (x.Lx == 2 && x.Ly == 2);
  const double rows_need = (double)c2 * std::pow((double)D2, (double)x.Lx + 1);
  O.rows_ok = !square12 && rows_need <= (double)(1ull << 28);
  if (O.rows_ok) big = std::max(big, (size_t)rows_need);
  O.big = big;
  O.t0 = ar.take<double>(big); O.t1 = ar.take<double>(big);
  O.t2 = ar.take<double>(big); O.t3 = ar.take<double>(big);
  // rho, then the raw contraction (complex tensors: a complex rho first)
  O.rho = ar.take<double>(d * d * d * d * (x.cfg.complex_tensors ? 3 : 2));
  O.red = ar.take<double>(256);
  O.vals = ar.take<double>(16);
}

// ---------------------------------------------------------------------------
// frames
// ---------------------------------------------------------------------------
// Number k of counter-clockwise quarter turns after which a move in direction
// `dir` (ctm_dir) is a left move: left 0, up 1, right 2, down 3.
int frame_of_dir(int dir) {
  static const int k[4] = {0, 2, 1, 3};  // CTM_LEFT, CTM_RIGHT, CTM_UP, CTM_DOWN
  return k[dir & 3];
}

void frame_dims(int k, int Lx, int Ly, int& lx, int& ly) {
  if (k % 2 == 0) { lx = Lx; ly = Ly; } else { lx = Ly; ly = Lx; }
}
int pmod(int a, int m) { int r = a % m; return r < 0 ? r + m : r; }

// Site (x, y) shown at (xp, yp) after k counter-clockwise quarter turns; one
// turn maps (x, y) to (y, -x), so undoing it maps (xp, yp) to (-yp, xp).
void frame_site(int k, int xp, int yp, int Lx, int Ly, int& x, int& y) {
  int lx, ly;
  frame_dims(k, Lx, Ly, lx, ly);
  xp = pmod(xp, lx);
  yp = pmod(yp, ly);
  for (int j = k % 4; j > 0; --j) {
    int ax, ay;
    frame_dims(j - 1, Lx, Ly, ax, ay);
    int nx = pmod(-yp, ax), ny = pmod(xp, ay);
    xp = nx;
    yp = ny;
  }
  x = pmod(xp, Lx);
  y = pmod(yp, Ly);
}

// frame coordinates of site (x, y) after k turns
void to_frame(int k, int x, int y, int Lx, int Ly, int& xp, int& yp) {
  for (int j = 0; j < k % 4; ++j) {
    int nx = y, ny = -x;
    x = nx;
    y = ny;
  }
  int lx, ly;
  frame_dims(k, Lx, Ly, lx, ly);
  xp = pmod(x, lx);
  yp = pmod(y, ly);
}

struct Roles {
  const ctm_ctx_s* x;
  Inst* I;
  int k;
  int pos(int xp, int yp) const {
    int sx, sy;
    frame_site(k, xp, yp, x->Lx, x->Ly, sx, sy);
    return sy * x->Lx + sx;
  }
  int tid(int xp, int yp) const { return x->pattern[pos(xp, yp)]; }
  double* C(int i, int xp, int yp) const { return I->C[(i + k) % 4][pos(xp, yp)]; }
  double* T(int i, int xp, int yp) const { return I->T[(i + k) % 4][pos(xp, yp)]; }
  void stale_C(int i, int xp, int yp) const { I->staleC[(i + k) % 4][pos(xp, yp)] = true; }
  void stale_T(int i, int xp, int yp) const { I->staleT[(i + k) % 4][pos(xp, yp)] = true; }
  void* Cw(int i, int xp, int yp) const { return I->Cw[(i + k) % 4][pos(xp, yp)]; }
  void* Tw(int i, int xp, int yp) const { return I->Tw[(i + k) % 4][pos(xp, yp)]; }
  void* TwP(int i, int xp, int yp) const { return I->TwP[(i + k) % 4][pos(xp, yp)]; }
  void* TwR(int i, int xp, int yp) const { return I->TwR[(i + k) % 4][pos(xp, yp)]; }
  void* bT(int xp, int yp, int r) const { return I->bT[tid(xp, yp)][(k + r) % 4]; }
  void* bTp(int xp, int yp, int r) const { return I->bTp[tid(xp, yp)][(k + r) % 4]; }
  // double layer of the site in this frame, additionally turned by r
  double* b64(int xp, int yp, int r) const { return I->b64[tid(xp, yp)][(k + r) % 4]; }
  void* bw(int xp, int yp, int r) const { return I->bw[tid(xp, yp)][(k + r) % 4]; }
  int cut(int xp, int yp) const { return pos(xp, yp); }
};

// ---------------------------------------------------------------------------
// GEMM helpers
// ---------------------------------------------------------------------------
struct G {
  std::vector<const void*> A, B;
  std::vector<void*> C;
  void add(const void* a, const void* b, void* c) {
    A.push_back(a); B.push_back(b); C.push_back(c);
  }
  int size() const { return (int)A.size(); }
  // problems j0 .. j0 + count - 1 as one launch group (count <= MAXG)
  GemmGroup group(int j0, int count) const {
    GemmGroup g{};
    for (int j = 0; j < count; ++j) { g.A[j] = A[j0 + j]; g.B[j] = B[j0 + j]; g.C[j] = C[j0 + j]; }
    return g;
  }
};

// every problem of `g` in launches of at most MAXG problems
ctm_status gemm_run(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va,
                    const View& vb, const View& vc, const G& g, double alpha = 1.0,
                    double beta = 0.0) {
  for (int j0 = 0; j0 < g.size(); j0 += MAXG) {
    int cnt = std::min(MAXG, g.size() - j0);
    HIPCHK(ctmk::gemm(s, ta, tc, M, N, K, alpha, va, vb, beta, vc, g.group(j0, cnt), cnt));
  }
  return CTM_OK;
}

// long contractions with few output columns go to the split-K kernel
ctm_status gemm_long(ctm_ctx_s& x, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va,
                     const View& vb, const View& vc, const G& g) {
  if (K < 1024 || !ts_gemm_supported(ta, tc, M, N, K, va, vb, vc))
    return gemm_run(x.stream, ta, tc, M, N, K, va, vb, vc, g);
  for (int j0 = 0; j0 < g.size(); j0 += MAXG) {
    int cnt = std::min(MAXG, g.size() - j0);
    HIPCHK(ts_gemm(x.stream, ta, tc, M, N, K, va, vb, vc, g.group(j0, cnt), cnt, x.ts_scratch, x.ts_bytes));
  }
  return CTM_OK;
}

// C = A B, (n x K)(K x N) float64 row-major, for every problem of g: the
// small-matrix kernel for K, N <= 64, the generic GEMM otherwise
ctm_status rmul_run(ctm_ctx_s& x, int64_t n, int K, int N, const G& g) {
  if (K > 64 || N > 64) return gemm_run(x.stream, F64, F64, n, N, K, rowmajor(K), rowmajor(N), rowmajor(N), g);
  for (int j0 = 0; j0 < g.size(); j0 += MAXP) {
    const int cnt = std::min(MAXP, g.size() - j0);
    CPtrSet a{}, b{};
    PtrSet c{};
    for (int i = 0; i < cnt; ++i) {
      a.p[i] = (const double*)g.A[j0 + i];
      b.p[i] = (const double*)g.B[j0 + i];
      c.p[i] = (double*)g.C[j0 + i];
    }
    HIPCHK(rmul_small(x.stream, n, K, N, a, b, c, cnt));
  }
  return CTM_OK;
}

ctm_status gemm_sk(ctm_ctx_s& x, int64_t M, int64_t N, int64_t K, const View& va, const View& vb,
                   const View& vc, const G& g) {
  for (int j0 = 0; j0 < g.size(); j0 += MAXG) {
    int cnt = std::min(MAXG, g.size() - j0);
    HIPCHK(ctmk::gemm_splitk(x.stream, M, N, K, 1.0, va, vb, 0.0, vc, g.group(j0, cnt), cnt, x.splitk,
                             x.splitk_elems));
  }
  return CTM_OK;
}

// grouped copies / conversions, in launches of at most MAXJ tensors
struct Xfer {
  std::vector<const void*> src;
  std::vector<void*> dst;
  std::vector<int64_t> n;
  void add(const void* a, void* b, int64_t cnt) { src.push_back(a); dst.push_back(b); n.push_back(cnt); }
};

ctm_status xfer_run(hipStream_t s, int tin, int tout, const Xfer& x) {
  for (size_t j0 = 0; j0 < x.src.size(); j0 += MAXJ) {
    int cnt = (int)std::min<size_t>(MAXJ, x.src.size() - j0);
    XferSet xs{};
    for (int j = 0; j < cnt; ++j) { xs.src[j] = x.src[j0 + j]; xs.dst[j] = x.dst[j0 + j]; xs.n[j] = x.n[j0 + j]; }
    HIPCHK(convert_group(s, tin, tout, xs, cnt));
  }
  return CTM_OK;
}

// p /= ||p||_F for every listed float64 tensor
ctm_status normalize_run(ctm_ctx_s& x, const std::vector<std::pair<double*, int64_t>>& t) {
  for (size_t j0 = 0; j0 < t.size(); j0 += MAXJ) {
    int cnt = (int)std::min<size_t>(MAXJ, t.size() - j0);
    NormSet ns{};
    for (int j = 0; j < cnt; ++j) { ns.p[j] = t[j0 + j].first; ns.n[j] = t[j0 + j].second; }
    HIPCHK(normalize_group(x.stream, ns, cnt, x.norm_part));
  }
  return CTM_OK;
}

ctm_status gemm1(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va,
                 const void* a, const View& vb, const void* b, const View& vc, void* c,
                 double alpha = 1.0, double beta = 0.0) {
  G g;
  g.add(a, b, c);
  return gemm_run(s, ta, tc, M, N, K, va, vb, vc, g, alpha, beta);
}

View view2(int64_t r_ext, int64_t r_ls, int64_t r_hs, int64_t c_ext, int64_t c_ls, int64_t c_hs) {
  return View{r_ext, r_ls, r_hs, c_ext, c_ls, c_hs};
}
const int64_t BIG = INT64_MAX / 4;

// ---------------------------------------------------------------------------
// enlarged corners: Q[(g,dn),(b,r)] = sum C[p,n] Tn[n,u,b] Tp[g,l,p] a[u,l,dn,r]
//   X[(g,l), n]     = Tp[(g,l), p] C[p, n]
//   Y[(g,l), (u,b)] = X[(g,l), n] Tn[n, (u,b)]
//   Q               = sum_{(l,u)} Y[(g,b),(l,u)] b[(l,u),(dn,r)], written to
//                     the row-major [W x N] matrix through a two-level view.
// One grouped launch per stage covers every corner of every row.
// ---------------------------------------------------------------------------
struct CornerJob {
  const void *C, *Tn, *Tp, *b;
  void *X, *Y, *Q;
  const void *TnP = nullptr, *bT = nullptr;  // bf16 path: permuted edge, transposed double layer
  const void* bTp = nullptr;                 // ... and the latter packed for the corner kernel
  const void* TnR = nullptr;                 // bf16 path: bf16 edge as [next][inner][prev]
  const void *Sk = nullptr, *Sb = nullptr;   // single-layer mode: ket and bra of the rotation
  const void *SkT = nullptr, *SbT = nullptr; // ... as operands of the bf16 corner kernel
};

struct Stage3Timer {
  std::vector<std::array<hipEvent_t, 2>>* pool = nullptr;
  size_t* used = nullptr;
};

ctm_status stage3_timed(hipStream_t s, const Stage3Timer* tm, const std::function<ctm_status()>& f) {
  const bool timed = tm && tm->pool && !dry_run();
  if (!timed) return f();
  if (*tm->used == tm->pool->size()) {
    std::array<hipEvent_t, 2> e{};
    for (auto& v : e) HIPCHK(hipEventCreate(&v));
    tm->pool->push_back(e);
  }
  const std::array<hipEvent_t, 2>& e = (*tm->pool)[*tm->used];
  HIPCHK(hipEventRecord(e[0], s));
  CHK(f());
  HIPCHK(hipEventRecord(e[1], s));
  *tm->used += 1;
  return CTM_OK;
}

// bf16: the double-layer stage (stage 3) takes bf16 operands (stage 2 writes
// Y in bf16, the double layer is the transposed bf16 copy) with fp32
// accumulation; stages 1 and 2 run in `tin`.
// ---------------------------------------------------------------------------
// Single-layer form of a double-layer product (Sec. II D: A and its conjugate
// absorbed one at a time).  With the fused legs ket-major (l = (l_k, l_b), ...)
// and a[(l,u),(dn,r)] = sum_s A[s,u_k,l_k,d_k,r_k] B[s,u_b,l_b,d_b,r_b],
//   P[(g,b),(dn,r)] = sum_(l,u) Y[(g,b),(l,u)] a[(l,u),(dn,r)]
// is taken as
//   Y' [(g,b,l_b,u_b),(l_k,u_k)]   = Y with its legs permuted
//   Z  [(g,b,l_b,u_b),(s,d_k,r_k)] = Y' Sk,  Sk[(l_k,u_k),(s,d_k,r_k)] = A
//   P' [(g,b,d_k,r_k),(d_b,r_b)]   = sum_(l_b,u_b,s) Z Sb,  Sb[(l_b,u_b,s),(d_b,r_b)] = B
//   P  = P' with its legs permuted into the consumer's layout,
// 4 c^2 d D^6 flop instead of 2 c^2 D^8 (c the extent of g and b).  Y is
// given by its 6-d storage dims and the permutation that orders them as
// (g, b, l_b, u_b, l_k, u_k); P' has dims (g, b, d_k, r_k, d_b, r_b) and
// out_perm orders them as the consumer stores them.  Sk and Sb are the
// tensors' [L'][U'][s][D'][R'] copies, read as D^2 x d D^2 and d D^2 x D^2
// matrices.  Jobs go in passes of as many as the scratch holds.
// ---------------------------------------------------------------------------
struct SlJob {
  const void *y, *sk, *sb;
  void* out;
};

ctm_status sl_product(ctm_ctx_s& x, int64_t c, int D, int d, const std::vector<SlJob>& jobs, const int64_t ydims[6],
                      const int yperm[6], const int out_perm[6], int tin, int tz, int tout) {
  // tin: type of Y; tz: operand type of both products (and of Z); P' is
  // float64 for float64 operands, else float32 (fp32 accumulation)
  hipStream_t s = x.stream;
  const int tp = tz == F64 ? F64 : F32;
  const int64_t D2 = (int64_t)D * D, M = c * c * D2;
  const size_t yb = (size_t)M * D2 * dtype_size(tz), zb = yb * (size_t)d, pb = (size_t)M * D2 * dtype_size(tp);
  if (!x.sl_y || yb == 0) return fail(CTM_E_STATE, "single-layer scratch missing");
  const size_t nb = std::max<size_t>(1, std::min<size_t>({(size_t)MAXG, x.sl_ybytes / std::max(yb, pb),
                                                          x.sl_zbytes / zb}));
  if (nb * std::max(yb, pb) > x.sl_ybytes || nb * zb > x.sl_zbytes)
    return fail(CTM_E_STATE, "single-layer scratch too small");
  const int64_t pdims[6] = {c, c, D, D, D, D};
  for (size_t j0 = 0; j0 < jobs.size(); j0 += nb) {
    const size_t j1 = std::min(jobs.size(), j0 + nb);
    G ga, gb;
    for (size_t j = j0; j < j1; ++j) {
      char* yj = (char*)x.sl_y + (j - j0) * yb;
      char* zj = (char*)x.sl_z + (j - j0) * zb;
      char* pj = (char*)x.sl_p + (j - j0) * pb;
      HIPCHK(permute(s, tin, jobs[j].y, tz, yj, 6, ydims, yperm));
      ga.add(yj, jobs[j].sk, zj);
      gb.add(zj, jobs[j].sb, pj);
    }
    CHK(gemm_run(s, tz, tz, M, (int64_t)d * D2, D2, rowmajor(D2), rowmajor((int64_t)d * D2),
                 rowmajor((int64_t)d * D2), ga));
    // Z read as rows (g,b | d_k,r_k) -> gb d D^4 + (d_k,r_k), columns (l_b,u_b,s) -> stride D^2
    CHK(gemm_run(s, tz, tp, M, D2, (int64_t)d * D2, view2(D2, 1, (int64_t)d * D2 * D2, BIG, D2, 0), rowmajor(D2),
                 rowmajor(D2), gb));
    for (size_t j = j0; j < j1; ++j)
      HIPCHK(permute(s, tp, (char*)x.sl_p + (j - j0) * pb, tout, jobs[j].out, 6, pdims, out_perm));
  }
  return CTM_OK;
}

// out[r][0 .. kp) = in[r][0 .. K) followed by zeros, bf16, r < rows
__global__ void pad_rows_kernel(const __bf16* __restrict__ in, int64_t rows, int K, int kp, __bf16* __restrict__ out) {
  const int64_t n = rows * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / kp;
    const int c = (int)(e - r * kp);
    out[e] = c < K ? in[r * K + c] : (__bf16)0.0f;
  }
}

hipError_t pad_rows_bf16(hipStream_t s, const void* in, int64_t rows, int K, int kp, void* out) {
  if (!span_ok(in, (size_t)rows * K * 2, "pad in") || !span_ok(out, (size_t)rows * kp * 2, "pad out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(4096, (rows * kp + 255) / 256);
  hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, s,
                     (const __bf16*)in, rows, K, kp, (__bf16*)out);
  return hipGetLastError();
}

// Y'[(g,b,l_b,u_b)][(l_k,u_k) padded to kp] from the enlarged corner's
// Y[g][l_k][l_b][u_k][u_b][b] (bf16); the padding is zero.  For fixed
// (g, l_b, u_b) this is the transpose of the D^2 x c matrix over ((l_k,u_k), b):
// a work-group takes 64 consecutive b, reads each (l_k,u_k) row along b and
// writes each b row along (l_k,u_k) through LDS.
__global__ void __launch_bounds__(256) sl_gather_kernel(const __bf16* __restrict__ Y, int c, int D, int kp,
                                                        __bf16* __restrict__ out) {
  __shared__ __bf16 tile[64][152 + 2];  // [b][(l_k,u_k)], D^2 <= 144 < 152
  const int D2 = D * D;
  const int nbt = (c + 63) / 64;
  const int64_t grp = blockIdx.x / nbt;  // (g, l_b, u_b)
  const int b0 = (int)(blockIdx.x % nbt) * 64;
  const int64_t g = grp / D2;
  const int lb = (int)((grp / D) % D), ub = (int)(grp % D);
  const int tid = threadIdx.x;
  // read: 64 b per (l_k,u_k) row, four rows per pass
  for (int e = tid; e < D2 * 64; e += 256) {
    const int col = e / 64, bb = e % 64, b = b0 + bb;
    const int lk = col / D, uk = col % D;
    tile[bb][col] = b < c ? Y[((((g * D + lk) * D + lb) * D + uk) * D + ub) * (int64_t)c + b] : (__bf16)0.0f;
  }
  __syncthreads();
  // write: kp consecutive entries per b row
  for (int e = tid; e < 64 * kp; e += 256) {
    const int bb = e / kp, col = e % kp, b = b0 + bb;
    if (b >= c) continue;
    const int64_t row = ((g * c + b) * D + lb) * D + ub;
    out[row * kp + col] = col < D2 ? tile[bb][col] : (__bf16)0.0f;
  }
}

// The single-layer product in the bf16 form on the bf16 corner kernel (see
// sl_product): Y' gathered with zero-padded rows; the first product taken
// transposed, Z^T[(d_k,r_k,s),(g,b,l_b,u_b)] = SkT Y'^T, written through the
// output view straight into Z[(g,b,d_k,r_k)][(l_b,u_b,s)] (four consecutive
// s per 8-byte store), the row-major A operand of the second product; P'
// float32, then permuted into the consumer's layout.
ctm_status sl_product_bf16(ctm_ctx_s& x, int64_t c, int D, int d, const std::vector<SlJob>& jobs,
                           const int out_perm[6], int tout) {
  hipStream_t s = x.stream;
  const int64_t D2 = (int64_t)D * D, M = c * c * D2, kp = (D2 + 7) / 8 * 8, N1 = (int64_t)d * D2;
  const size_t yb = (size_t)M * kp * 2, zb = (size_t)M * N1 * 2, pb = (size_t)M * D2 * 4;
  if (!x.sl_y || yb == 0) return fail(CTM_E_STATE, "single-layer scratch missing");
  if (D2 > 144) return fail(CTM_E_INVALID, "single-layer bf16 form: D <= 12");
  const size_t nb = std::max<size_t>(1, std::min<size_t>({(size_t)MAXG, x.sl_ybytes / std::max(yb, pb),
                                                          x.sl_zbytes / zb}));
  if (nb * std::max(yb, pb) > x.sl_ybytes || nb * zb > x.sl_zbytes)
    return fail(CTM_E_STATE, "single-layer scratch too small");
  const int64_t pdims[6] = {c, c, D, D, D, D};
  // Z element (row (dr_k, s), column (gb, lu_b)) at dr_k d D^2 + s + gb d D^4 + lu_b d
  const View vzt{d, 1, N1, D2, d, D2 * D2 * d};
  for (size_t j0 = 0; j0 < jobs.size(); j0 += nb) {
    const size_t j1 = std::min(jobs.size(), j0 + nb);
    G ga, gb;
    for (size_t j = j0; j < j1; ++j) {
      char* yj = (char*)x.sl_y + (j - j0) * yb;
      char* zj = (char*)x.sl_z + (j - j0) * zb;
      char* pj = (char*)x.sl_p + (j - j0) * pb;
      HIPCHK(spans({{jobs[j].y, (size_t)M * D2 * 2}, {yj, yb}}, "sl gather"));
      const int64_t blocks = c * D2 * ((c + 63) / 64);
      if (!dry_run())
        hipLaunchKernelGGL(sl_gather_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const __bf16*)jobs[j].y,
                           (int)c, D, (int)kp, (__bf16*)yj);
      HIPCHK(last_err());
      ga.add(jobs[j].sk, yj, zj);
      gb.add(zj, jobs[j].sb, pj);
    }
    HIPCHK(corner_bf16(s, N1, M, kp, vzt, ga.group(0, ga.size()), ga.size(), BF16));
    HIPCHK(corner_bf16(s, M, D2, N1, rowmajor(D2), gb.group(0, gb.size()), gb.size(), F32));
    for (size_t j = j0; j < j1; ++j)
      HIPCHK(permute(s, F32, (char*)x.sl_p + (j - j0) * pb, tout, jobs[j].out, 6, pdims, out_perm));
  }
  return CTM_OK;
}

ctm_status corner_chain(hipStream_t s, int tin, int tq, int chi, int D2, const std::vector<CornerJob>& jobs,
                        const Stage3Timer* tm, bool bf16, ctm_ctx_s* slx = nullptr, int D = 0, int d = 0) {
  const int64_t c = chi, n = (int64_t)chi * D2;
  const int64_t K4 = (int64_t)D2 * D2;
  const bool fast = bf16 && tq == F32 && !jobs.empty() && jobs[0].TnP && jobs[0].bT &&
                    corner_bf16_supported(c * c, K4, K4);
  const int ty = bf16 ? BF16 : tin;  // type of Y
  const bool fast2 = fast && jobs[0].TnR && corner_bf16_supported(n, n, c);
  bool packed = fast && corner_packed_b();
  for (const CornerJob& j : jobs) packed = packed && j.bTp;
  for (size_t j0 = 0; j0 < jobs.size(); j0 += MAXG) {
    size_t j1 = std::min(jobs.size(), j0 + MAXG);
    G g1, g2, g3;
    bool packed_a = false;
    if (fast) {
      // stage 2 writes Y as [(g,b)][(l,u)], so that stage 3 has both operands
      // contiguous in the contracted index; rows m = (g, l) -> g chi D^4 + l D^2,
      // cols (b, u) -> b D^4 + u
      View vy = view2(D2, D2, c * K4, D2, 1, K4);
      if (fast2) {
        // stage 2 on the bf16 kernel too: X in bf16 from stage 1, the edge as
        // [(b,u)][n] (its bf16 copy ordered [next][inner][prev])
        for (size_t j = j0; j < j1; ++j) {
          g1.add(jobs[j].Tp, jobs[j].C, jobs[j].X);
          g2.add(jobs[j].X, jobs[j].TnR, jobs[j].Y);
          g3.add(jobs[j].Y, packed ? jobs[j].bTp : jobs[j].bT, jobs[j].Q);
        }
        CHK(gemm_run(s, tin, BF16, n, c, c, rowmajor(c), rowmajor(c), rowmajor(c), g1));
        if (packed && corner_packed_a() && D2 % 4 == 0) {
          // taken transposed: the edge rows (b, u) times X rows (g, l)
          packed_a = true;
          G g2t;
          for (size_t j = j0; j < j1; ++j) g2t.add(jobs[j].TnR, jobs[j].X, jobs[j].Y);
          HIPCHK(corner_bf16_to_packed_a(s, n, n, c, c, D2, g2t.group(0, g2t.size()), g2t.size()));
        } else {
          HIPCHK(corner_bf16(s, n, n, c, vy, g2.group(0, g2.size()), g2.size(), BF16));
        }
      } else {
        // stage 2 reads the edge as [n][(b,u)]
        for (size_t j = j0; j < j1; ++j) {
          g1.add(jobs[j].Tp, jobs[j].C, jobs[j].X);
          g2.add(jobs[j].X, jobs[j].TnP, jobs[j].Y);
          g3.add(jobs[j].Y, packed ? jobs[j].bTp : jobs[j].bT, jobs[j].Q);
        }
        CHK(gemm_run(s, tin, tin, n, c, c, rowmajor(c), rowmajor(c), rowmajor(c), g1));
        CHK(gemm_run(s, tin, ty, n, n, c, rowmajor(c), rowmajor(n), vy, g2));
      }
      View vc = view2(c, D2, (int64_t)D2 * n, D2, 1, n);
      CHK(stage3_timed(s, tm, [&]() -> ctm_status {
        HIPCHK(corner_bf16(s, c * c, K4, K4, vc, g3.group(0, g3.size()), g3.size(), F32, 0, packed, packed_a));
        return CTM_OK;
      }));
      continue;
    }
    for (size_t j = j0; j < j1; ++j) {
      g1.add(jobs[j].Tp, jobs[j].C, jobs[j].X);
      g2.add(jobs[j].X, jobs[j].Tn, jobs[j].Y);
      g3.add(jobs[j].Y, bf16 ? jobs[j].bT : jobs[j].b, jobs[j].Q);
    }
    CHK(gemm_run(s, tin, tin, n, c, c, rowmajor(c), rowmajor(c), rowmajor(c), g1));
    CHK(gemm_run(s, tin, ty, n, n, c, rowmajor(c), rowmajor(n), rowmajor(n), g2));
    if (slx) {
      // Y[g][l_k][l_b][u_k][u_b][b] -> (g, b, l_b, u_b, l_k, u_k); P' (g, b, d_k, r_k, d_b, r_b)
      // -> Q[(g,dn),(b,r)] = [g][d_k][d_b][b][r_k][r_b]
      const int64_t ydims[6] = {c, D, D, D, D, c};
      const int yperm[6] = {0, 5, 2, 4, 1, 3};
      const int operm[6] = {0, 2, 4, 1, 3, 5};
      // bf16: both products on the bf16 MFMA (Y and Z in bf16, fp32
      // accumulation), on the corner kernel where its K % 8 == 0 holds
      const bool fast_sl = bf16 && jobs[0].SkT && ((int64_t)d * D * D) % 8 == 0 && d % 4 == 0 && D * D <= 144;
      std::vector<SlJob> sj;
      for (size_t j = j0; j < j1; ++j)
        sj.push_back(fast_sl ? SlJob{jobs[j].Y, jobs[j].SkT, jobs[j].SbT, jobs[j].Q}
                             : SlJob{jobs[j].Y, jobs[j].Sk, jobs[j].Sb, jobs[j].Q});
      CHK(stage3_timed(s, tm, [&]() {
        return fast_sl ? sl_product_bf16(*slx, c, D, d, sj, operm, tq)
                       : sl_product(*slx, c, D, d, sj, ydims, yperm, operm, ty, ty, tq);
      }));
      continue;
    }
    // A: rows m = (g, b): b low (extent chi, stride 1), g high (stride D2*D2*chi);
    //    cols k = (l, u): stride chi
    View va = view2(c, 1, (int64_t)D2 * D2 * c, BIG, c, 0);
    // B: the double layer [(l,u)][(dn,r)], or its transposed bf16 copy
    View vb = bf16 ? transposed(rowmajor(K4)) : rowmajor(K4);
    // C: rows m = (g, b) -> g*D2*n + b*D2; cols (dn, r) -> dn*n + r
    View vc = view2(c, D2, (int64_t)D2 * n, D2, 1, n);
    CHK(stage3_timed(s, tm, [&]() { return gemm_run(s, ty, tq, c * c, K4, K4, va, vb, vc, g3); }));
  }
  return CTM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------
namespace {

struct SolveRow {
  const void* Q[4];
  Row* R;
  double* Vkeep;
  SolveStatus* skeep;
  bool warm;
};

// out = op(N) in for all problems, with N = Q2^T Q1^T Q4^T Q3^T (transposeN =
// false) or N^T = Q3 Q4 Q1 Q2 (true).  `mid` receives the product after the
// first two factors (Lh^T in, or Uh in).  in/out/mid float64 n x k.  With
// nfac = 2 only mid is formed.
// in_cast false: the rows' float32 input (qin) already holds `in` rounded
// (written by the orthonormalisation that produced it).
ctm_status napply(ctm_ctx_s& x, int n, int k, const std::vector<SolveRow>& rows,
                  const std::vector<double*>& in, const std::vector<double*>& out,
                  const std::vector<double*>& mid, bool transposeN, int nfac = 4, bool in_cast = true) {
  hipStream_t s = x.stream;
  const int qt = x.qt;
  const View vq = transposeN ? rowmajor(n) : transposed(rowmajor(n));
  const View vb = rowmajor(k);
  // factor order
  const int ord_n[4] = {2, 3, 0, 1};   // Q3^T, Q4^T, Q1^T, Q2^T applied in turn
  const int ord_t[4] = {1, 0, 3, 2};   // Q2, Q1, Q4, Q3
  const int* ord = transposeN ? ord_t : ord_n;
  const size_t P = rows.size();
  if (qt == F64) {
    for (int f = 0; f < nfac; ++f) {
      G g;
      for (size_t r = 0; r < P; ++r) {
        Row* R = rows[r].R;
        const double* src = f == 0 ? in[r] : (f == 1 ? R->tmp : (f == 2 ? mid[r] : R->tmp));
        double* dst = f == 0 ? R->tmp : (f == 1 ? mid[r] : (f == 2 ? R->tmp : out[r]));
        g.add(rows[r].Q[ord[f]], src, dst);
      }
      CHK(gemm_long(x, F64, F64, n, k, n, vq, vb, vb, g));
    }
    return CTM_OK;
  }
  // reduced precision: cast in, apply in the Q type, mid and out in float64.
  // Where the float32 tall-skinny kernel takes the second product, its
  // reduction writes mid beside the float32 result; elsewhere a conversion.
  if (in_cast) {
    Xfer cv;
    for (size_t r = 0; r < P; ++r) cv.add(in[r], rows[r].R->qin, (int64_t)n * k);
    CHK(xfer_run(s, F64, qt, cv));
  }
  const bool ts_mid = qt == F32 && n >= 1024 && ts_gemm_supported(F32, F32, n, k, n, vq, vb, vb);
  for (int f = 0; f < nfac; ++f) {
    G g, gm;
    for (size_t r = 0; r < P; ++r) {
      Row* R = rows[r].R;
      const void* src = f == 0 ? R->qin : (f == 1 ? R->q1 : (f == 2 ? R->q2 : R->q1));
      void* dst = f == 0 ? R->q1 : (f == 1 ? R->q2 : (f == 2 ? R->q1 : (void*)out[r]));
      g.add(rows[r].Q[ord[f]], src, dst);
      gm.add(nullptr, nullptr, mid[r]);
    }
    if (f == 1 && ts_mid) {
      for (int j0 = 0; j0 < g.size(); j0 += MAXG) {
        const int cnt = std::min(MAXG, g.size() - j0);
        const GemmGroup g2 = gm.group(j0, cnt);
        HIPCHK(ts_gemm(s, F32, F32, n, k, n, vq, vb, vb, g.group(j0, cnt), cnt, x.ts_scratch, x.ts_bytes, &g2));
      }
      continue;
    }
    CHK(gemm_long(x, qt, f == 3 ? F64 : qt, n, k, n, vq, vb, vb, g));
    if (f == 1) {
      Xfer cv;
      for (size_t r = 0; r < P; ++r) cv.add(rows[r].R->q2, mid[r], (int64_t)n * k);
      CHK(xfer_run(s, qt, F64, cv));
    }
  }
  return CTM_OK;
}

// Y <- Y R^{-1} `passes` times with R from the shifted Cholesky factor of Y^T Y
// (Cholesky-QR with shifts; Fukaya et al., SIAM J. Sci. Comput. 2020); up to
// 64 columns by substitution with R, otherwise through R^{-1} and a product.
// With to_qin (k <= 64 only), the last pass also writes Y rounded to float32
// into each row's N-apply input (what napply's cast would write).  With Yin
// (k <= 64 only), the first pass starts from Yin instead of Y's contents
// (Yin is read, Y written).
ctm_status orthonormalize(ctm_ctx_s& x, int n, int k, const std::vector<SolveRow>& rows,
                          const std::vector<double*>& Y, int passes = 3, bool to_qin = false,
                          const std::vector<double*>* Yin = nullptr) {
  hipStream_t s = x.stream;
  const size_t P = rows.size();
  const double u = 1.1102230246251565e-16;
  if (Yin && k > CHOL_WAVE_MAX) {  // the product form works in place: copy first
    Xfer cp;
    for (size_t r = 0; r < P; ++r) cp.add((*Yin)[r], Y[r], (int64_t)n * k);
    CHK(xfer_run(s, F64, F64, cp));
    Yin = nullptr;
  }
  for (int pass = 0; pass < passes; ++pass) {
    double coef = pass == 0 ? 11.0 * ((double)n * k + (double)k * (k + 1)) * u : 4.0 * u;
    G gg;
    CPtrSet Gs{};
    PtrSet Ri{};
    StatSet st{};
    // the first pass reads Yin when given
    const bool from_in = Yin && pass == 0;
    for (size_t r = 0; r < P; ++r) {
      gg.add(Y[r], Y[r], rows[r].R->G);
      Gs.p[r] = rows[r].R->G;
      Ri.p[r] = rows[r].R->Rinv;
      st.p[r] = rows[r].R->st;
    }
    if (k <= 64) {
      CPtrSet Ys{};
      PtrSet Gp{};
      for (size_t r = 0; r < P; ++r) { Ys.p[r] = from_in ? (*Yin)[r] : Y[r]; Gp.p[r] = rows[r].R->G; }
      HIPCHK(gram_small(s, n, k, Ys, Gp, (int)P, x.splitk, x.splitk_elems));
    } else {
      CHK(gemm_sk(x, k, k, n, transposed(rowmajor(k)), rowmajor(k), rowmajor(k), gg));
    }
    if (k <= CHOL_WAVE_MAX) {
      // R itself, then Y <- Y R^{-1} by substitution in place
      HIPCHK(chol_shift_inv(s, k, coef, Gs, Ri, st, (int)P, false));
      PtrSet Ys{};
      CPtrSet Rs{};
      for (size_t r = 0; r < P; ++r) { Ys.p[r] = Y[r]; Rs.p[r] = rows[r].R->Rinv; }
      PtrSet q32{};
      CPtrSet yin{};
      for (size_t r = 0; r < P; ++r) {
        q32.p[r] = (double*)rows[r].R->qin;
        yin.p[r] = from_in ? (*Yin)[r] : nullptr;
      }
      HIPCHK(trsm_rows(s, n, k, Ys, Rs, (int)P, (to_qin && pass + 1 == passes) ? &q32 : nullptr,
                       from_in ? &yin : nullptr));
      continue;
    }
    HIPCHK(chol_shift_inv(s, k, coef, Gs, Ri, st, (int)P));
    G gm;
    for (size_t r = 0; r < P; ++r) gm.add(Y[r], rows[r].R->Rinv, rows[r].R->tmp);
    CHK(gemm_run(s, F64, F64, n, k, k, rowmajor(k), rowmajor(k), rowmajor(k), gm));
    Xfer cp;
    for (size_t r = 0; r < P; ++r) cp.add(rows[r].R->tmp, Y[r], (int64_t)n * k);
    CHK(xfer_run(s, F64, F64, cp));
  }
  return CTM_OK;
}

// Truncated SVD of N = (Lh Uh)^T by block subspace iteration with
// Rayleigh-Ritz, then the projectors
//   P1 = Lh^T V S^{-1/2},   P2^T = Uh U S^{-1/2}   (kept columns only).
ctm_status solve_projectors(ctm_ctx_s& x, Inst& I, std::vector<SolveRow>& rows, uint64_t key) {
  hipStream_t s = x.stream;
  const int n = I.n, k = I.k_act, chi = I.chi;
  const size_t P = rows.size();
  const ctm_config& c = x.cfg;
  // start block: kept columns of the previous solve on this cut, then normals
  {
    PtrSet V0{};
    CPtrSet Vp{};
    StatSet pr{};
    StatSet st{};
    for (size_t r = 0; r < P; ++r) {
      V0.p[r] = rows[r].R->V;
      Vp.p[r] = rows[r].warm ? rows[r].Vkeep : nullptr;
      pr.p[r] = rows[r].warm ? rows[r].skeep : nullptr;
      st.p[r] = rows[r].R->st;
    }
    // the random columns of the start block depend only on the cut group
    // (direction, column, launch), not on how often it was solved, so a
    // captured sweep replays exactly what the eager sweep computes
    HIPCHK(warm_start(s, n, I.n_cap, k, I.k, V0, Vp, pr, c.seed + 0x9E3779B97F4A7C15ull * (key + 1), (int)P));
    HIPCHK(reset_status(s, st, (int)P));
  }
  std::vector<double*> V(P), Yb(P), Qb(P), Z(P), LV(P), UU(P), Ub(P), Vpv(P);
  for (size_t r = 0; r < P; ++r) {
    Row* R = rows[r].R;
    V[r] = R->V; Yb[r] = R->Yb; Qb[r] = R->Qb; Z[r] = R->Z; LV[r] = R->LV; UU[r] = R->UU;
    Ub[r] = R->Ub; Vpv[r] = R->Vp;
  }
  const int maxit = std::max(1, c.svd_max_iters);
  const bool adaptive = c.svd_resid_tol > 0;
  // full Cholesky-QR3 for the bases that enter Rayleigh-Ritz in float64; in
  // the fixed-count (reduced-precision) mode the shifted pass and one more
  // leave an orthogonality error well below that of the fp32 products
  const int ortho_passes = adaptive ? 3 : 2;
  // the start block (kept orthonormal columns and independent normals) is
  // well conditioned: Cholesky-QR twice orthonormalises it to rounding level.
  // The fixed-count iteration only takes its span (the first application of
  // N is orthonormalised afresh), so one pass is enough there
  // the orthonormalisations that feed an N-application write its float32
  // input themselves (k <= 64, float32 Q), and that application skips its cast
  const bool q32 = x.qt == F32 && k <= CHOL_WAVE_MAX;
  CHK(orthonormalize(x, n, k, rows, V, adaptive ? 2 : 1, q32));
  std::vector<SolveStatus> hst(P);
  auto copy_blocks = [&](std::vector<double*>& dst, const std::vector<double*>& src) -> ctm_status {
    Xfer cp;
    for (size_t r = 0; r < P; ++r) cp.add(src[r], dst[r], (int64_t)n * k);
    return xfer_run(s, F64, F64, cp);
  };
  // One Rayleigh-Ritz iteration: Y = N V = Q R, R = U_R S W_R^T, then the
  // left vectors U = Q U_R, right vectors V' = V W_R, Z = N^T U and the
  // residuals |Z_i - S_i V'_i|.
  auto rr_iteration = [&](bool want_resid) -> ctm_status {
    CHK(napply(x, n, k, rows, V, Yb, LV, false, 4, !q32));  // Y = N V, LV = Lh^T V
    CHK(orthonormalize(x, n, k, rows, Qb, ortho_passes, false, &Yb));  // Q = orth(Y), Y kept
    if (k <= 48) {
      CPtrSet Qs{}, Ys{};
      PtrSet Rs{};
      for (size_t r = 0; r < P; ++r) { Qs.p[r] = Qb[r]; Ys.p[r] = Yb[r]; Rs.p[r] = rows[r].R->Rm; }
      HIPCHK(gram_cross_small(s, n, k, Qs, Ys, Rs, (int)P, x.splitk, x.splitk_elems));
    } else {
      G g;
      for (size_t r = 0; r < P; ++r) g.add(Qb[r], Yb[r], rows[r].R->Rm);
      CHK(gemm_sk(x, k, k, n, transposed(rowmajor(k)), rowmajor(k), rowmajor(k), g));
    }
    {
      CPtrSet M{};
      PtrSet U{}, S{}, W{}, J{};
      // R is upper triangular with a graded diagonal: rotating its rows (the
      // columns of R^T) converges in a few sweeps (preconditioned Jacobi,
      // Drmac & Veselic 2008).  R^T W = X S gives R = W S X^T, so U_R = W
      // and W_R = X.
      StatSet stj{};
      for (size_t r = 0; r < P; ++r) {
        Row* R = rows[r].R;
        M.p[r] = R->Rm; U.p[r] = R->WR; S.p[r] = R->S; W.p[r] = R->UR; J.p[r] = R->jw;
        stj.p[r] = R->st;
      }
      // directions 100x below the cutoff can never be kept.  With reduced-
      // precision contractions and a fixed iteration count the rotations
      // stop at a column cosine of 1e-8, far below the contractions' own
      // rounding, instead of float64 orthogonality (about one sweep less)
      const double rot_rel = (x.qt != F64 && !adaptive) ? 1e-8 : 0.0;
      HIPCHK(jacobi_svd(s, k, M, U, S, W, J, (int)P, true, true, &stj, 1e-2 * c.svd_cutoff, rot_rel));
    }
    {
      // three products of one shape per row, one grouped launch; the small
      // kernel (k <= 64) may write in place, so Lh^T V' replaces Lh^T V there
      const bool in_place = k <= 64;
      G gq;
      for (size_t r = 0; r < P; ++r) {
        Row* R = rows[r].R;
        gq.add(Qb[r], R->UR, Ub[r]);   // U  = Q U_R
        gq.add(V[r], R->WR, Vpv[r]);   // V' = V W_R
        gq.add(LV[r], R->WR, in_place ? (void*)LV[r] : R->tmp);  // Lh^T V' = (Lh^T V) W_R
      }
      CHK(rmul_run(x, n, k, k, gq));
      if (!in_place) {
        Xfer cp;
        for (size_t r = 0; r < P; ++r) cp.add(rows[r].R->tmp, LV[r], (int64_t)n * k);
        CHK(xfer_run(s, F64, F64, cp));
      }
    }
    // UU = Uh U (the projector's factor), and Z = N^T U for the residuals
    CHK(napply(x, n, k, rows, Ub, Z, UU, true, want_resid ? 4 : 2));
    {
      CPtrSet Zs{}, Vs{}, Ss{};
      StatSet st{};
      for (size_t r = 0; r < P; ++r) {
        Zs.p[r] = want_resid ? Z[r] : nullptr; Vs.p[r] = Vpv[r]; Ss.p[r] = rows[r].R->S; st.p[r] = rows[r].R->st;
      }
      HIPCHK(residual_status(s, n, k, chi, c.svd_cutoff, c.svd_resid_tol > 0 ? c.svd_resid_tol : 0.0,
                             Zs, Vs, Ss, st, (int)P, x.splitk, x.splitk_elems));
    }
    return CTM_OK;
  };
  if (adaptive) {
    // Rayleigh-Ritz every iteration; stop when all kept residuals are small
    for (int it = 0; it < maxit; ++it) {
      CHK(rr_iteration(true));
      if (it + 1 >= maxit) break;
      bool all = true;
      for (size_t r = 0; r < P; ++r) HIPCHK(d2h(&hst[r], rows[r].R->st, sizeof(SolveStatus), s));
      HIPCHK(ssync(s));
      for (size_t r = 0; r < P; ++r) all = all && hst[r].converged;
      if (all) break;
      CHK(copy_blocks(V, Z));
      CHK(orthonormalize(x, n, k, rows, V, 3, q32));
    }
  } else {
    // fixed count: plain subspace iterations V <- orth(N^T orth(N V)), then
    // one Rayleigh-Ritz step.  The inner basis only carries the span to
    // N^T: the shifted Cholesky-QR pass alone leaves it conditioned well
    // enough for that step.  The residuals steer nothing
    // here; they are formed on the last column step of a sweep (and of every
    // single move) as the accuracy record of the solver.
    for (int it = 0; it + 1 < maxit; ++it) {
      CHK(napply(x, n, k, rows, V, Yb, LV, false, 4, !q32));
      CHK(orthonormalize(x, n, k, rows, Yb, 1, q32));
      // V is not read again before it is replaced: N^T orth(N V) goes there
      CHK(napply(x, n, k, rows, Yb, V, UU, true, 4, !q32));
      CHK(orthonormalize(x, n, k, rows, V, ortho_passes, q32));
    }
    CHK(rr_iteration(x.resid_step));
  }
  // projectors
  {
    // LV already holds Lh^T V' (rotated); Wp and Up = the diag-scaled
    // selector, problems (row r, copy j) at j P + r, in as few launches as fit
    for (size_t r0 = 0; r0 < 2 * P; r0 += MAXP) {
      const size_t r1 = std::min(2 * P, r0 + MAXP);
      CPtrSet Sv{}, Id{};
      PtrSet Wu{};
      StatSet st{};
      for (size_t q = r0; q < r1; ++q) {
        Row* R = rows[q % P].R;
        Sv.p[q - r0] = R->S; Id.p[q - r0] = nullptr; Wu.p[q - r0] = q < P ? R->Wp : R->Up; st.p[q - r0] = R->st;
      }
      HIPCHK(scale_kept(s, k, chi, Id, Sv, Wu, st, (int)(r1 - r0)));
    }
    G gp;
    for (size_t r = 0; r < P; ++r) {
      Row* R = rows[r].R;
      gp.add(LV[r], R->Wp, R->P1);
      gp.add(UU[r], R->Up, R->P2T);
    }
    CHK(rmul_run(x, n, k, chi, gp));
    // keep the right vectors and status for the next solve on the same cut
    static_assert(sizeof(SolveStatus) % 8 == 0, "status copied as 8-byte words");
    Xfer cp;
    for (size_t r = 0; r < P; ++r) {
      cp.add(Vpv[r], rows[r].Vkeep, (int64_t)n * k);
      cp.add(rows[r].R->st, rows[r].skeep, (int64_t)(sizeof(SolveStatus) / 8));
    }
    CHK(xfer_run(s, F64, F64, cp));
  }
  return CTM_OK;
}

// ---------------------------------------------------------------------------
// absorption, every row of every instance of a class together (frame roles):
//   C1'  = P1[y-1]^T (C1 T1)
//   T4'  = P1[y]^T-contracted ( (T4 P2[y-1]^T) b )
//   C4'  = (T3 C4) P2[y]^T-contracted
// then every new tensor divided by its Frobenius norm and stored.
// ---------------------------------------------------------------------------
ctm_status absorb_rows(ctm_ctx_s& x, const std::vector<Inst*>& insts, int k, int xp) {
  hipStream_t s = x.stream;
  const int at = x.wt;
  const Inst& I0 = *insts[0];
  const int64_t c = I0.chi, D2 = I0.D2, n = I0.n;
  int lx, ly;
  frame_dims(k, x.Lx, x.Ly, lx, ly);
  G g1, g2, g3, g4, g5, g6, g7;
  for (Inst* I : insts) {
    Roles ro{&x, I, k};
    for (int yp = 0; yp < ly; ++yp) {
      Row& R = I->rows[yp];
      Row& Rp = I->rows[pmod(yp - 1, ly)];
      g1.add(ro.Cw(0, xp, yp), ro.Tw(0, xp, yp), R.CT);
      g2.add(Rp.P1w, R.CT, R.nC1);
      g3.add(ro.Tw(3, xp, yp), Rp.P2Tw, R.W1);
      g4.add(R.W1, ro.bw(xp, yp, 0), R.W2);
      g5.add(R.P1w, R.W2, R.nT4);
      g6.add(ro.Tw(2, xp, yp), ro.Cw(3, xp, yp), R.X6);
      g7.add(R.X6, R.P2Tw, R.nC4);
    }
  }
  // C1' [b', r] = sum_(a,U) P1prev[(a,U), b'] CT[(a,U), r]
  CHK(gemm_run(s, at, at, c, D2 * c, c, rowmajor(c), rowmajor(D2 * c), rowmajor(D2 * c), g1));
  CHK(gemm_long(x, at, F64, c, c, n, transposed(rowmajor(c)), rowmajor(c), rowmajor(c), g2));
  // W1 = sum_p T4[(g,l),p] P2T_prev[(p,u), c2];  then
  // W2[(g,c2),(dn,R)] = sum_(l,u) W1[(g,c2),(l,u)] b[(l,u),(dn,R)] is the new
  // edge itself: rounding its operands to bf16 perturbs the fixed point
  // directly (~10x the energy error of bf16 enlarged corners, which only steer
  // the truncation).  In bf16 mode both are three-term products
  // hi.hi + hi.lo + lo.hi of bf16 splits (operand error ~2^-16) on the bf16
  // kernel (W1 is stored split and transposed to [(g,c2)][(l,u)]); otherwise
  // in the working type.
  const int64_t K4 = D2 * D2;
  // W2 is written transposed (W2t, below) by its own product in bf16 mode
  bool w2t_done = false;
  if (x.cfg.single_layer) {
    // the new edge itself: float32 (or float64) operands also in CTM_BF16
    CHK(gemm_run(s, at, at, c * D2, D2 * c, c, rowmajor(c), rowmajor(D2 * c), rowmajor(D2 * c), g3));
    // W1[g][l_k][l_b][u_k][u_b][c2] -> (g, c2, l_b, u_b, l_k, u_k); P' (g, c2, d_k, R_k, d_b, R_b)
    // -> W2[(g,c2)][(dn,R)], or straight into W2t[(g,dn)][(R,c2)] in float32
    const int64_t ydims[6] = {c, I0.D, I0.D, I0.D, I0.D, c};
    const int yperm[6] = {0, 5, 2, 4, 1, 3};
    const bool to_t = at == F32 && D2 >= 2 && I0.rows[0].W2t;
    const int operm_w2[6] = {0, 1, 2, 4, 3, 5};
    const int operm_w2t[6] = {0, 2, 4, 3, 5, 1};
    std::vector<SlJob> sj;
    for (Inst* I : insts) {
      Roles ro{&x, I, k};
      for (int yp = 0; yp < ly; ++yp) {
        Row& R = I->rows[yp];
        const int t = ro.tid(xp, yp);
        sj.push_back(SlJob{R.W1, I->Sk[t][k % 4], I->Sb[t][k % 4], to_t ? R.W2t : R.W2});
      }
    }
    CHK(sl_product(x, c, I0.D, I0.d, sj, ydims, yperm, to_t ? operm_w2t : operm_w2, at, at, at));
    w2t_done = to_t;
  } else if (x.prec == CTM_BF16 && I0.rows[0].A3 && corner_bf16_supported(c * c, K4, 3 * K4)) {
    bool a3_done = false;
    if (I0.rows[0].T3s && corner_bf16_supported(c * D2, D2 * c, 3 * c)) {
      // W1 as a three-term bf16 product too, split from the float64 masters:
      //   A side T4[(g,l), p], B side (P2T as [p][(u,c2)])^T with its rows
      //   taken in (c2, u) order.
      // The product stores its result directly as the split operand of the
      // next one, A3[(g,c2)][hi | hi | lo over (l,u)]: element ((g,l),(c2,u))
      // at (g c + c2) 3 K4 + l D2 + u, the copies K4 apart; with u the fast
      // output column, 16 lanes store 16 consecutive entries
      G g3b;
      std::vector<Split3Job> sj;
      for (Inst* I : insts) {
        Roles ro{&x, I, k};
        for (int yp = 0; yp < ly; ++yp) {
          Row& R = I->rows[yp];
          Row& Rp = I->rows[pmod(yp - 1, ly)];
          sj.push_back(Split3Job{ro.T(3, xp, yp), rowmajor(c), true, R.T3s});
          sj.push_back(Split3Job{Rp.P2T, view2(D2, c, 1, BIG, D2 * c, 0), false, R.P3s});
          g3b.add(R.T3s, R.P3s, R.A3);
        }
      }
      HIPCHK(split3_bf16_group(s, sj.data(), (int)sj.size(), c * D2, c));
      const View va3 = view2(D2, D2, c * 3 * K4, D2, 1, 3 * K4);
      for (int j0 = 0; j0 < g3b.size(); j0 += MAXG) {
        int cnt = std::min(MAXG, g3b.size() - j0);
        HIPCHK(corner_bf16(s, c * D2, D2 * c, 3 * c, va3, g3b.group(j0, cnt), cnt, BF16, K4));
      }
      a3_done = true;
    } else {
      CHK(gemm_run(s, at, at, c * D2, D2 * c, c, rowmajor(c), rowmajor(D2 * c), rowmajor(D2 * c), g3));
    }
    // W2[(g,c2), (dn,R)] stored as W2t[(g,dn)][(R,c2)] when the fp32 path
    // below reads it that way: element (m, n) at (m / c) K4 c + m % c + n c
    // (four consecutive c2 per 16-byte store)
    const bool to_t = at == F32 && D2 >= 2 && I0.rows[0].W2t;
    // the double layer's split in the packed fragment layout when every
    // instance of the class has it
    bool b3p = corner_packed_b();
    for (Inst* I : insts)
      for (int t = 0; t < MAXT; ++t) b3p = b3p && (I->bT3[t][0] == nullptr || I->bT3p[t][0] != nullptr);
    G g3x;
    for (Inst* I : insts) {
      Roles ro{&x, I, k};
      for (int yp = 0; yp < ly; ++yp) {
        Row& R = I->rows[yp];
        // W1 as c matrices [(l,u)][c2] -> A3[(g,c2)][hi | hi | lo over (l,u)]
        if (!a3_done) HIPCHK(split3_transpose_bf16(s, (const float*)R.W1, c, K4, c, true, R.A3));
        const int tt = ro.tid(xp, yp), rr = (k + 0) % 4;
        g3x.add(R.A3, b3p ? I->bT3p[tt][rr] : I->bT3[tt][rr], to_t ? R.W2t : R.W2);
      }
    }
    const View vw2 = to_t ? View{c, 1, K4 * c, INT64_MAX / 4, c, 0} : rowmajor(K4);
    for (int j0 = 0; j0 < g3x.size(); j0 += MAXG) {
      int cnt = std::min(MAXG, g3x.size() - j0);
      HIPCHK(corner_bf16(s, c * c, K4, 3 * K4, vw2, g3x.group(j0, cnt), cnt, F32, 0, b3p));
    }
    w2t_done = to_t;
  } else {
    CHK(gemm_run(s, at, at, c * D2, D2 * c, c, rowmajor(c), rowmajor(D2 * c), rowmajor(D2 * c), g3));
    CHK(gemm_run(s, at, at, c * c, K4, K4, view2(c, 1, D2 * D2 * c, BIG, c, 0), rowmajor(K4), rowmajor(K4), g4));
  }
  // T4'[c1, (R, c2)] = sum_(g,dn) P1[(g,dn), c1] W2[(g,dn), (R, c2)]
  //   B rows k = (g, dn): dn low (extent D2, stride D2), g high (stride chi*D2*D2)
  //   B cols n = (R, c2): c2 low (extent chi, stride D2*D2), R high (stride 1)
  if (at == F32 && D2 >= 2) {
    // W2 read through that view touches one element per cache line: use it
    // transposed (per g: [c2][(dn,R)] -> [(dn,R)][c2], i.e. W2t[(g,dn)][(R,c2)]),
    // as stored by the bf16 product or transposed here.
    // The product is then tall and skinny in transposed form,
    //   T4'^T[(R,c2), c1] = sum_(g,dn) W2t[(g,dn),(R,c2)] P1[(g,dn), c1],
    // with chi output columns and a contraction of length n (the freed W2,
    // chi^2 D2^2 floats >= chi^2 D2 doubles, holds it), transposed back into T4'.
    G g5t;
    for (Inst* I : insts)
      for (int yp = 0; yp < ly; ++yp) {
        Row& R = I->rows[yp];
        if (!w2t_done) HIPCHK(transpose_batched(s, (const float*)R.W2, c, c, K4, (float*)R.W2t));
        g5t.add(R.W2t, R.P1w, R.W2);
      }
    if (ts_gemm_supported(F32, F64, D2 * c, c, n, transposed(rowmajor(D2 * c)), rowmajor(c), rowmajor(c))) {
      for (int j0 = 0; j0 < g5t.size(); j0 += MAXG) {
        int cnt = std::min(MAXG, g5t.size() - j0);
        HIPCHK(ts_gemm(s, F32, F64, D2 * c, c, n, transposed(rowmajor(D2 * c)), rowmajor(c), rowmajor(c),
                       g5t.group(j0, cnt), cnt, x.ts_scratch, x.ts_bytes));
      }
    } else {
      CHK(gemm_run(s, F32, F64, D2 * c, c, n, transposed(rowmajor(D2 * c)), rowmajor(c), rowmajor(c), g5t));
    }
    const int64_t dims[2] = {D2 * c, c};
    const int perm[2] = {1, 0};
    for (Inst* I : insts)
      for (int yp = 0; yp < ly; ++yp) {
        Row& R = I->rows[yp];
        HIPCHK(permute(s, F64, R.W2, F64, R.nT4, 2, dims, perm));
      }
  } else {
    CHK(gemm_run(s, at, F64, c, D2 * c, n, transposed(rowmajor(c)), view2(D2, D2, c * D2 * D2, c, D2 * D2, 1),
                 rowmajor(D2 * c), g5));
  }
  // X6[z, (g, dn)] = sum_q T3[(z,dn), q] C4[q, g]  written as [z][g][dn]
  CHK(gemm_run(s, at, at, c * D2, c, c, rowmajor(c), rowmajor(c), view2(D2, 1, c * D2, BIG, D2, 0), g6));
  // C4'[z, c] = sum_(g,dn) X6[z,(g,dn)] P2T[(g,dn), c]
  CHK(gemm_long(x, at, F64, c, c, n, rowmajor(n), rowmajor(c), rowmajor(c), g7));
  // normalise, then store into the environment (all projectors of the column
  // step were computed before any tensor is replaced)
  std::vector<std::pair<double*, int64_t>> nt;
  Xfer st;
  for (Inst* I : insts) {
    Roles ro{&x, I, k};
    for (int yp = 0; yp < ly; ++yp) {
      Row& R = I->rows[yp];
      nt.push_back({R.nC1, c * c});
      nt.push_back({R.nT4, c * c * D2});
      nt.push_back({R.nC4, c * c});
      st.add(R.nC1, ro.C(0, xp + 1, yp), c * c);
      st.add(R.nT4, ro.T(3, xp + 1, yp), c * c * D2);
      st.add(R.nC4, ro.C(3, xp + 1, yp), c * c);
      ro.stale_C(0, xp + 1, yp);
      ro.stale_T(3, xp + 1, yp);
      ro.stale_C(3, xp + 1, yp);
    }
  }
  CHK(normalize_run(x, nt));
  CHK(xfer_run(s, F64, F64, st));
  return CTM_OK;
}

// working-precision copies of every corner and edge of the instances
ctm_status refresh_working(ctm_ctx_s& x, const std::vector<Inst*>& insts) {
  if (x.wt == F64) return CTM_OK;
  const int npos = x.Lx * x.Ly;
  Xfer cv;
  for (Inst* I : insts) {
    const int64_t c2 = (int64_t)I->chi * I->chi, t3 = c2 * I->D2;
    for (int c = 0; c < 4; ++c)
      for (int p = 0; p < npos; ++p) {
        if (I->staleC[c][p]) cv.add(I->C[c][p], I->Cw[c][p], c2);
        if (!I->staleT[c][p]) continue;
        cv.add(I->T[c][p], I->Tw[c][p], t3);
        if (I->TwP[c][p]) {
          int64_t dims[3] = {I->chi, I->D2, I->chi};
          int perm[3] = {0, 2, 1};
          HIPCHK(permute(x.stream, F64, I->T[c][p], x.wt, I->TwP[c][p], 3, dims, perm));
        }
        if (I->TwR[c][p]) {
          int64_t dims[3] = {I->chi, I->D2, I->chi};
          int perm[3] = {2, 1, 0};
          HIPCHK(permute(x.stream, F64, I->T[c][p], BF16, I->TwR[c][p], 3, dims, perm));
        }
      }
  }
  CHK(xfer_run(x.stream, F64, x.wt, cv));
  // only once the copies are enqueued (a failure above leaves them stale)
  for (Inst* I : insts)
    for (int c = 0; c < 4; ++c)
      for (int p = 0; p < npos; ++p) I->staleC[c][p] = I->staleT[c][p] = false;
  return CTM_OK;
}

// the record of the current column step (created on first use)
ctm_status timing_begin(ctm_ctx_s& x) {
  if (!x.timing || !x.phase_timing || dry_run() || x.tused < x.tpool.size()) return CTM_OK;
  std::array<hipEvent_t, 4> e{};
  for (auto& v : e) HIPCHK(hipEventCreate(&v));
  x.tpool.push_back(e);
  return CTM_OK;
}
void ev_record(ctm_ctx_s& x, int i) {
  if (x.timing && x.phase_timing && !dry_run()) (void)hipEventRecord(x.tpool[x.tused][i], x.stream);
}
double ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  (void)hipEventSynchronize(b);
  (void)hipEventElapsedTime(&ms, a, b);
  return ms * 1e-3;
}
// adds every pending record to the totals
void timing_flush(ctm_ctx_s& x) {
  for (size_t i = 0; i < x.tused; ++i) {
    const auto& e = x.tpool[i];
    x.t_corner += ev_ms(e[0], e[1]);
    x.t_solver += ev_ms(e[1], e[2]);
    x.t_absorb += ev_ms(e[2], e[3]);
  }
  for (size_t i = 0; i < x.sused; ++i) {
    x.t_stage3 += ev_ms(x.spool[i][0], x.spool[i][1]);
    x.stage3_launches += 1;
  }
  x.tused = x.sused = 0;
}

// One column step of the move in direction k at frame column xp, for every
// instance of one class (equal d, D, chi) in lock-step: each stage is one
// grouped launch over all rows of all of them.
ctm_status column_step(ctm_ctx_s& x, const std::vector<Inst*>& insts, int k, int xp) {
  hipStream_t s = x.stream;
  Inst& I0 = *insts[0];
  int lx, ly;
  frame_dims(k, x.Lx, x.Ly, lx, ly);
  CHK(refresh_working(x, insts));
  CHK(timing_begin(x));
  ev_record(x, 0);
  // enlarged corners of every plaquette (xp, yp)
  std::vector<CornerJob> jobs;
  for (Inst* I : insts) {
    Roles ro{&x, I, k};
    for (int yp = 0; yp < ly; ++yp) {
      Row& R = I->rows[yp];
      const int cx[4] = {xp, xp + 1, xp + 1, xp};
      const int cy[4] = {yp, yp, yp + 1, yp + 1};
      for (int q = 0; q < 4; ++q) {
        CornerJob j;
        j.C = ro.Cw(q, cx[q], cy[q]);
        j.Tn = ro.Tw(q, cx[q], cy[q]);
        j.Tp = ro.Tw((q + 3) % 4, cx[q], cy[q]);
        j.b = ro.bw(cx[q], cy[q], q);
        if (x.cfg.single_layer) {
          const int t = ro.tid(cx[q], cy[q]), r = (k + q) % 4;
          j.Sk = x.prec == CTM_BF16 ? I->Sk16[t][r] : I->Sk[t][r];
          j.Sb = x.prec == CTM_BF16 ? I->Sb16[t][r] : I->Sb[t][r];
          j.SkT = I->SkT16[t][r];
          j.SbT = I->SbT16[t][r];
        }
        j.X = R.X[q];
        j.Y = R.Y[q];
        j.Q = R.Q[q];
        if (x.prec == CTM_BF16) {
          j.TnR = ro.TwR(q, cx[q], cy[q]);
          j.TnP = ro.TwP(q, cx[q], cy[q]);
          j.bT = ro.bT(cx[q], cy[q], q);
          j.bTp = ro.bTp(cx[q], cy[q], q);
        }
        jobs.push_back(j);
      }
    }
  }
  Stage3Timer tm;
  if (x.timing) {
    tm.pool = &x.spool;
    tm.used = &x.sused;
    // algorithmic work of the (l,u)-contraction with the double layer:
    // 2 chi^2 D^8 flop per corner; single-layer: 4 chi^2 d D^6
    const double d8 = (double)I0.D2 * I0.D2 * I0.D2 * I0.D2;
    const double w = x.cfg.single_layer ? 4.0 * I0.d * d8 / I0.D2 : 2.0 * d8;
    x.stage3_flop += w * (double)I0.chi * I0.chi * (double)jobs.size();
    x.stage3_flop_nom += w * (double)I0.chi_cap * I0.chi_cap * (double)jobs.size();
    x.live_chi = I0.chi;
  }
  CHK(corner_chain(s, x.wt, x.qt, I0.chi, I0.D2, jobs, x.timing ? &tm : nullptr, x.prec == CTM_BF16,
                   x.cfg.single_layer ? &x : nullptr, I0.D, I0.d));
  x.corner_launches += 3 * ((jobs.size() + MAXG - 1) / MAXG);
  x.moves += 1;
  ev_record(x, 1);
  // projectors, all rows together (at most MAXP problems per launch)
  std::vector<SolveRow> rows;
  for (Inst* I : insts) {
    Roles ro{&x, I, k};
    for (int yp = 0; yp < ly; ++yp) {
      SolveRow sr;
      Row& R = I->rows[yp];
      for (int q = 0; q < 4; ++q) sr.Q[q] = R.Q[q];
      sr.R = &R;
      int cut = ro.cut(xp, yp);
      sr.Vkeep = I->Vkeep[k][cut];
      sr.skeep = I->skeep[k][cut];
      sr.warm = I->has_keep[k][cut];
      rows.push_back(sr);
    }
  }
  for (size_t r0 = 0; r0 < rows.size(); r0 += MAXP) {
    std::vector<SolveRow> part(rows.begin() + r0, rows.begin() + std::min(rows.size(), r0 + MAXP));
    CHK(solve_projectors(x, I0, part, ((uint64_t)k * MAXPOS + (uint64_t)xp) * 4096 + r0 / MAXP));
  }
  for (Inst* I : insts) {
    Roles ro{&x, I, k};
    for (int yp = 0; yp < ly; ++yp) I->has_keep[k][ro.cut(xp, yp)] = true;
  }
  if (x.wt != F64) {
    Xfer cv;
    for (Inst* I : insts)
      for (int yp = 0; yp < ly; ++yp) {
        Row& R = I->rows[yp];
        cv.add(R.P1, R.P1w, (int64_t)I->n * I->chi);
        cv.add(R.P2T, R.P2Tw, (int64_t)I->n * I->chi);
      }
    CHK(xfer_run(s, F64, x.wt, cv));
  }
  ev_record(x, 2);
  CHK(absorb_rows(x, insts, k, xp));
  ev_record(x, 3);
  if (x.timing && !dry_run()) {
    if (x.phase_timing) x.tused += 1;
    if (x.tused >= 1024 || x.sused >= 1024) timing_flush(x);  // bounded event pools
  }
  return CTM_OK;
}

// ---------------------------------------------------------------------------
// corner spectra and the convergence measure
// ---------------------------------------------------------------------------
struct SpecSet {
  double* spec_new[MAXP];
  double* spec_old[MAXP];
  double* delta[MAXP];
  int* flag[MAXP];             // [0] non-finite, [1] largest chi_eff of the last solves
  const SolveStatus* st[MAXP];  // the instance's kept-solve statuses, contiguous
};

// one block per instance; spec_new holds its ncorner spectra (descending,
// stride chi); entries from `live` on are the zero singular values of the
// zero-padded corner and are written as such
__global__ void spectra_delta_kernel(SpecSet ss, int chi, int live, int ncorner, int nstat, int first,
                                     int commit) {
  __shared__ double red[256];
  double* __restrict__ spec_new = ss.spec_new[blockIdx.x];
  double* __restrict__ spec_old = ss.spec_old[blockIdx.x];
  double dmax = 0.0;
  for (int c = 0; c < ncorner; ++c) {
    double tot = 0.0;
    for (int i = threadIdx.x; i < live; i += blockDim.x) tot += spec_new[c * chi + i];
    red[threadIdx.x] = tot;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    tot = red[0];
    __syncthreads();
    double d = 0.0;
    for (int i = threadIdx.x; i < chi; i += blockDim.x) {
      double v = i >= live ? 0.0 : (tot > 0 ? spec_new[c * chi + i] / tot : spec_new[c * chi + i]);
      if (!isfinite(v)) *ss.flag[blockIdx.x] = 1;
      spec_new[c * chi + i] = v;
      d += fabs(v - spec_old[c * chi + i]);
    }
    red[threadIdx.x] = d;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    dmax = fmax(dmax, red[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ss.delta[blockIdx.x] = first ? INFINITY : dmax;
    int ce = 0;
    for (int i = 0; i < nstat; ++i) ce = max(ce, ss.st[blockIdx.x][i].chi_eff);
    ss.flag[blockIdx.x][1] = ce;
  }
  if (commit) {
    __syncthreads();
    for (int i = threadIdx.x; i < ncorner * chi; i += blockDim.x) spec_old[i] = spec_new[i];
  }
}

// singular values of every corner of the instances (one class), normalised
// to unit sum; Delta = largest l1 change against the previous spectra
ctm_status corner_spectra(ctm_ctx_s& x, const std::vector<Inst*>& insts, bool first, bool commit) {
  hipStream_t s = x.stream;
  // corners are live-extent matrices; spectra are stored at the full chi
  const int npos = x.Lx * x.Ly, nc = 4 * npos, chi = insts[0]->chi, cs = insts[0]->chi_cap;
  const size_t c2 = (size_t)chi * chi;
  std::vector<std::pair<const double*, double*>> probs;  // (corner, output spectrum)
  for (Inst* I : insts)
    for (int c = 0; c < nc; ++c) probs.push_back({I->C[c % 4][c / 4], I->spec_new + (size_t)c * cs});
  for (size_t c0 = 0; c0 < probs.size(); c0 += MAXP) {
    int cnt = (int)std::min<size_t>(MAXP, probs.size() - c0);
    CPtrSet M{};
    PtrSet U{}, S{}, W{}, J{};
    for (int j = 0; j < cnt; ++j) {
      M.p[j] = probs[c0 + j].first;
      S.p[j] = probs[c0 + j].second;
      U.p[j] = x.spec_tmp_U + (size_t)j * c2;
      W.p[j] = x.spec_tmp_W + (size_t)j * c2;
      J.p[j] = x.spec_tmp_J + (size_t)j * 2 * chi * ((chi + 15) / 16 * 16);
    }
    // corner singular values far below the solver cutoff carry no information;
    // with reduced-precision contractions the rotations stop at a column
    // cosine of 1e-8, far below the spectra's own rounding (as in the
    // solver's Rayleigh-Ritz step)
    HIPCHK(jacobi_svd(s, chi, M, U, S, W, J, cnt, false, false, nullptr, 1e-2 * x.cfg.svd_cutoff,
                      x.qt != F64 ? 1e-8 : 0.0));
  }
  for (size_t i0 = 0; i0 < insts.size(); i0 += MAXP) {
    int cnt = (int)std::min<size_t>(MAXP, insts.size() - i0);
    SpecSet ss{};
    for (int j = 0; j < cnt; ++j) {
      Inst* I = insts[i0 + j];
      HIPCHK(spans({{I->spec_new, (size_t)nc * cs * 8}, {I->spec_old, (size_t)nc * cs * 8}, {I->delta, 8},
                    {I->flag, 8}, {I->skeep_all, (size_t)nc * sizeof(SolveStatus)}}, "spectra"));
      ss.spec_new[j] = I->spec_new;
      ss.spec_old[j] = I->spec_old;
      ss.delta[j] = I->delta;
      ss.flag[j] = I->flag;
      ss.st[j] = I->skeep_all;
    }
    if (!dry_run())
      hipLaunchKernelGGL(spectra_delta_kernel, dim3(cnt), dim3(256), 0, s, ss, cs, chi, nc, nc, first ? 1 : 0,
                         commit ? 1 : 0);
    HIPCHK(last_err());
  }
  return CTM_OK;
}

// ---------------------------------------------------------------------------
// environment initialisation
// ---------------------------------------------------------------------------
__global__ void init_env_kernel(double* C, double* T, int chi, int Dk, int Db, int diag,
                                const double* spec) {
  const int D2 = Dk * Db;
  const int64_t c2 = (int64_t)chi * chi, t3 = c2 * D2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < t3;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = e / ((int64_t)D2 * chi), rem = e % ((int64_t)D2 * chi);
    int U = (int)(rem / chi), b = (int)(rem % chi);
    int u = U / Db, uu = U % Db;
    double v = 0.0;
    if (u == uu) v = diag ? (a == b ? 1.0 : 0.0) : ((a == 0 && b == 0) ? 1.0 : 0.0);
    T[e] = v;
    if (e < c2) {
      int i = (int)(e / chi), j = (int)(e % chi);
      C[e] = diag ? (i == j ? spec[i] : 0.0) : ((i == 0 && j == 0) ? 1.0 : 0.0);
    }
  }
}

bool finite_host(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

ctm_status validate(const ctm_config* c) {
  if (!c) return fail(CTM_E_INVALID, "null config");
  if (c->n_inst < 1 || c->Lx < 1 || c->Ly < 1 || c->Lx > 4 || c->Ly > 4 || c->n_tensors < 1 ||
      c->n_tensors > MAXT)
    return fail(CTM_E_INVALID, "cell: need n_inst>=1, 1<=Lx,Ly<=4, 1<=n_tensors<=4");
  if (!c->pattern || !c->d || !c->D || !c->chi) return fail(CTM_E_INVALID, "null pattern/d/D/chi");
  for (int i = 0; i < c->Lx * c->Ly; ++i)
    if (c->pattern[i] < 0 || c->pattern[i] >= c->n_tensors) return fail(CTM_E_INVALID, "pattern entry out of range");
  if (c->prec < 0 || c->prec > 2) return fail(CTM_E_INVALID, "prec");
  if (c->complex_tensors != 0 && c->complex_tensors != 1) return fail(CTM_E_INVALID, "complex_tensors must be 0 or 1");
  if (c->complex_tensors && c->single_layer)
    return fail(CTM_E_INVALID, "complex tensors run on the real form of the double layer, not the single-layer route");
  for (int i = 0; i < c->n_inst; ++i) {
    int d = c->d[i], D = c->D[i], chi = c->chi[i];
    if (d < 1 || D < 1 || chi < 1 || d > 64 || D > 16) return fail(CTM_E_INVALID, "d in 1..64, D in 1..16, chi >= 1");
    int64_t n = (int64_t)chi * D * D;
    if (n * n > (int64_t)INT32_MAX * 4) return fail(CTM_E_INVALID, "chi*D^2 too large");
    int k = std::min<int64_t>(n, chi + std::max(0, c->svd_oversample));
    if (k > 176) return fail(CTM_E_INVALID, "chi + oversample must be <= 176");
    if (chi > 192) return fail(CTM_E_INVALID, "chi must be <= 192");
  }
  return CTM_OK;
}

ctm_status build_ctx(const ctm_config* cfg, ctm_ctx_s& x) {
  CHK(validate(cfg));
  x.cfg = *cfg;
  x.Lx = cfg->Lx;
  x.Ly = cfg->Ly;
  x.ntens = cfg->n_tensors;
  x.ninst = cfg->n_inst;
  x.pattern.assign(cfg->pattern, cfg->pattern + x.Lx * x.Ly);
  x.dv.assign(cfg->d, cfg->d + x.ninst);
  x.Dv.assign(cfg->D, cfg->D + x.ninst);
  x.chiv.assign(cfg->chi, cfg->chi + x.ninst);
  x.cfg.pattern = x.pattern.data();
  x.cfg.d = x.dv.data();
  x.cfg.D = x.Dv.data();
  x.cfg.chi = x.chiv.data();
  x.prec = cfg->prec;
  x.wt = wtype_of(cfg->prec);
  x.qt = qtype_of(cfg->prec);
  x.inst.assign(x.ninst, Inst());
  for (int i = 0; i < x.ninst; ++i) {
    Inst& I = x.inst[i];
    I.d = x.dv[i];
    I.D = x.Dv[i];
    I.D2 = I.D * I.D;
    I.chi_cap = I.chi = x.chiv[i];
    I.n_cap = I.n = I.chi * I.D2;
    I.k = subspace_dim(x.cfg, I.chi_cap, I.n_cap);
    I.k_act = I.k;
  }
  // classes of instances with equal (d, D, chi), in order of first appearance
  x.classes.clear();
  for (int i = 0; i < x.ninst; ++i) {
    bool placed = false;
    for (auto& cls : x.classes) {
      const Inst& J = x.inst[cls[0]];
      if (J.d == x.inst[i].d && J.D == x.inst[i].D && J.chi_cap == x.inst[i].chi_cap) {
        cls.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) x.classes.push_back({i});
  }
  Arena ar;
  plan(x, ar);
  x.ws_need = ar.off + 256;
  return CTM_OK;
}

ctm_status init_env(ctm_ctx_s& x, Inst& I, int inst_idx, int init, const double* spec_host) {
  hipStream_t s = x.stream;
  const int npos = x.Lx * x.Ly;
  int chimax = 0;
  for (int v : x.chiv) chimax = std::max(chimax, v);
  // a fresh environment is stored at the full extent
  I.chi = I.chi_cap;
  I.n = I.n_cap;
  I.k_act = I.k;
  double* dspec = nullptr;
  std::vector<double> hs;
  if (init == CTM_INIT_DIAG) {
    if (!spec_host) return fail(CTM_E_INVALID, "CTM_INIT_DIAG needs spectrum_host");
    // stage the spectra in spec_old temporarily (npos*4*chi)
    hs.resize((size_t)npos * 4 * I.chi);
    for (int p = 0; p < npos; ++p)
      for (int c = 0; c < 4; ++c)
        for (int j = 0; j < I.chi; ++j)
          hs[((size_t)p * 4 + c) * I.chi + j] =
              spec_host[(((size_t)inst_idx * npos + p) * 4 + c) * chimax + j];
    if (!finite_host(hs.data(), hs.size())) return fail(CTM_E_NONFINITE, "non-finite spectrum");
    HIPCHK(h2d(I.spec_old, hs.data(), hs.size() * 8, s));
    dspec = I.spec_old;
  }
  for (int p = 0; p < npos; ++p) {
    for (int c = 0; c < 4; ++c) {
      const double* sp = dspec ? dspec + ((size_t)p * 4 + c) * I.chi : nullptr;
      HIPCHK(spans({{I.C[c][p], (size_t)I.chi * I.chi * 8}, {I.T[c][p], (size_t)I.chi * I.chi * I.D2 * 8},
                    {sp, sp ? (size_t)I.chi * 8 : 0}}, "init env"));
      if (!dry_run())
        hipLaunchKernelGGL(init_env_kernel, dim3(256), dim3(256), 0, s, I.C[c][p], I.T[c][p], I.chi, I.D,
                           I.D, init == CTM_INIT_DIAG ? 1 : 0, sp);
      HIPCHK(last_err());
    }
  }
  if (init == CTM_INIT_DIAG) {
    std::vector<std::pair<double*, int64_t>> nt;
    for (int p = 0; p < npos; ++p)
      for (int c = 0; c < 4; ++c) {
        nt.push_back({I.C[c][p], (int64_t)I.chi * I.chi});
        nt.push_back({I.T[c][p], (int64_t)I.chi * I.chi * I.D2});
      }
    CHK(normalize_run(x, nt));
  }
  HIPCHK(dmemset(I.spec_old, 0, (size_t)npos * 4 * I.chi * 8, s));
  HIPCHK(dmemset(I.flag, 0, sizeof(int) * 4, s));
  HIPCHK(dmemset(I.skeep_all, 0, sizeof(SolveStatus) * 4 * npos, s));
  for (Row& R : I.rows) HIPCHK(dmemset(R.st, 0, sizeof(SolveStatus), s));
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < npos; ++p) I.staleC[c][p] = I.staleT[c][p] = true;
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < npos; ++p) I.has_keep[c][p] = false;
  for (int c = 0; c < 4; ++c) I.cursor[c] = 0;
  std::vector<Inst*> one{&I};
  CHK(corner_spectra(x, one, true, true));
  return CTM_OK;
}

// ---------------------------------------------------------------------------
// live extent
// ---------------------------------------------------------------------------
// Every kept projector column comes from a subspace of k_act columns, so at
// most min(chi_cap, k_act) leading indices of a corner or edge leg are
// nonzero; rounded up to a multiple of 8 (the bf16 kernels contract over chi
// in steps of 8; the extra indices are zero).
int live_extent(const Inst& I, int k_act) {
  const int r = (k_act + 7) / 8 * 8;
  return std::max(1, std::min(I.chi_cap, r));
}

// out[a][U][b] (extent cn) = in[a][U][b] (extent co) where a, b < co, else 0;
// with D2 = 1 the corner layout [a][b].
__global__ void repack_kernel(const double* __restrict__ in, double* __restrict__ out, int co, int cn, int D2) {
  const int64_t tot = (int64_t)cn * D2 * cn;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / ((int64_t)D2 * cn), rem = e % ((int64_t)D2 * cn);
    const int u = (int)(rem / cn), b = (int)(rem % cn);
    out[e] = (a < co && b < co) ? in[(a * D2 + u) * co + b] : 0.0;
  }
}

// Re-lays every corner and edge of I out at the live extent cn (indices
// dropped when shrinking are exact zeros; those added when growing are
// zero), through the row scratch of the absorption.
ctm_status set_live(ctm_ctx_s& x, Inst& I, int cn) {
  cn = std::max(1, std::min(cn, I.chi_cap));
  const int co = I.chi;
  if (cn == co) return CTM_OK;
  const int npos = x.Lx * x.Ly;
  double* tmp = I.rows[0].nT4;  // chi_cap^2 D^2 doubles
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < npos; ++p)
      for (int which = 0; which < 2; ++which) {
        double* t = which == 0 ? I.C[c][p] : I.T[c][p];
        const int D2 = which == 0 ? 1 : I.D2;
        const size_t nin = (size_t)co * D2 * co, nout = (size_t)cn * D2 * cn;
        HIPCHK(spans({{t, std::max(nin, nout) * 8}, {tmp, nout * 8}}, "repack"));
        if (!dry_run()) {
          const int blocks = (int)std::min<size_t>(1024, (nout + 255) / 256);
          hipLaunchKernelGGL(repack_kernel, dim3(blocks), dim3(256), 0, x.stream, t, tmp, co, cn, D2);
        }
        HIPCHK(last_err());
        HIPCHK(d2d(t, tmp, nout * 8, x.stream));
      }
  I.chi = cn;
  I.n = cn * I.D2;
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < npos; ++p) I.staleC[c][p] = I.staleT[c][p] = true;
  return CTM_OK;
}

// Subspace width of every instance of a class, and the live extent that
// follows from it.
ctm_status set_width(ctm_ctx_s& x, const std::vector<int>& cls, int kn) {
  for (int i : cls) {
    Inst& I = x.inst[i];
    I.k_act = std::max(1, std::min(I.k, kn));
    CHK(set_live(x, I, live_extent(I, I.k_act)));
  }
  return CTM_OK;
}

// Moves of ctm_move run outside the convergence loop: when a narrowed
// subspace of a class was filled by the last solves (the width, not chi or
// the cutoff, then set the truncation), the width grows by the oversampling.
ctm_status grow_if_capped(ctm_ctx_s& x, const std::vector<int>& cls) {
  Inst& J = x.inst[cls[0]];
  if (J.k_act >= J.k || x.width_pinned) return CTM_OK;
  int ce = 0;
  for (int i : cls) {
    Inst& I = x.inst[i];
    for (Row& R : I.rows) {
      SolveStatus st{};
      HIPCHK(d2h(&st, R.st, sizeof(SolveStatus), x.stream));
      HIPCHK(ssync(x.stream));
      ce = std::max(ce, (int)st.chi_eff);
    }
  }
  if (ce >= J.k_act) CHK(set_width(x, cls, J.k_act + std::max(1, x.cfg.svd_oversample)));
  return CTM_OK;
}

std::vector<Inst*> class_insts(ctm_ctx_s& x, const std::vector<int>& cls) {
  std::vector<Inst*> v;
  for (int i : cls) v.push_back(&x.inst[i]);
  return v;
}

ctm_status do_move(ctm_ctx_s& x, const std::vector<Inst*>& insts, int dir, int count) {
  int lx, ly;
  frame_dims(dir, x.Lx, x.Ly, lx, ly);
  for (int i = 0; i < count; ++i) {
    int xp = insts[0]->cursor[dir];
    CHK(column_step(x, insts, dir, xp));
    for (Inst* I : insts) I->cursor[dir] = (xp + 1) % lx;
  }
  return CTM_OK;
}

ctm_status do_sweep(ctm_ctx_s& x, const std::vector<Inst*>& insts) {
  const int order[4] = {frame_of_dir(CTM_LEFT), frame_of_dir(CTM_RIGHT), frame_of_dir(CTM_UP),
                        frame_of_dir(CTM_DOWN)};
  for (int o = 0; o < 4; ++o) {
    int lx, ly;
    frame_dims(order[o], x.Lx, x.Ly, lx, ly);
    if (o < 3) {
      x.resid_step = false;
      CHK(do_move(x, insts, order[o], lx));
    } else {
      x.resid_step = false;
      CHK(do_move(x, insts, order[o], lx - 1));
      x.resid_step = true;  // the sweep's last column step
      CHK(do_move(x, insts, order[o], 1));
    }
  }
  x.resid_step = true;
  return CTM_OK;
}

// The instances of each class that are still sweeping (live[i] != 0).
std::vector<Inst*> live_insts(ctm_ctx_s& x, const std::vector<int>& cls, const std::vector<char>& live) {
  std::vector<Inst*> v;
  for (int i : cls)
    if (live[i]) v.push_back(&x.inst[i]);
  return v;
}

// One sweep of every live instance followed by its corner spectra and Delta,
// captured once as a HIP graph and replayed (graph mode) until the live set or
// the subspace width changes.  The first capture follows an eager sweep, so
// that every cut has a kept subspace (the solver's warm start) and every GEMM
// shape has been tuned.
ctm_status capture_sweep(ctm_ctx_s& x, const std::vector<char>& live) {
  if (x.gexec) return CTM_OK;
  const bool conc = concurrent_classes(x);
  hipStream_t main = x.stream;
  if (conc && x.class_streams.empty()) {
    // default priority (no priority argument)
    x.class_streams.assign(x.classes.size(), nullptr);
    for (auto& cs : x.class_streams) HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    x.class_events.assign(x.classes.size() + 1, nullptr);
    for (auto& ev : x.class_events) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
  ctm_status st = CTM_OK;
  const int64_t moves0 = x.moves;
  hipError_t ef = conc ? hipEventRecord(x.class_events[0], main) : hipSuccess;
  std::vector<char> forked(x.classes.size(), 0);
  for (size_t ci = 0; ci < x.classes.size() && ef == hipSuccess; ++ci) {
    const auto& cls = x.classes[ci];
    std::vector<Inst*> insts = live_insts(x, cls, live);
    if (insts.empty()) continue;
    if (conc) {
      // a branch of its own: forked from the main stream, own scratch
      ef = hipStreamWaitEvent(x.class_streams[ci], x.class_events[0], 0);
      if (ef != hipSuccess) break;
      forked[ci] = 1;
      x.stream = x.class_streams[ci];
      use_scratch(x, ci);
    }
    st = do_sweep(x, insts);
    if (st == CTM_OK) st = corner_spectra(x, insts, false, true);
    if (conc) {
      ef = hipEventRecord(x.class_events[ci + 1], x.class_streams[ci]);
      x.stream = main;
      use_scratch(x, 0);
    }
    if (st != CTM_OK) break;
  }
  // join every branch back into the main stream (also after a failure, so
  // that the capture ends cleanly)
  for (size_t ci = 0; ci < x.classes.size(); ++ci)
    if (forked[ci]) (void)hipStreamWaitEvent(main, x.class_events[ci + 1], 0);
  x.stream = main;
  x.moves = moves0;
  hipError_t e = hipStreamEndCapture(x.stream, &g);
  if (st == CTM_OK && ef != hipSuccess) st = hip_fail(ef, "graph branch fork/join");
  if (st != CTM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  HIPCHK(e);
  e = hipGraphInstantiate(&x.gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) x.gexec = nullptr;
  HIPCHK(e);
  return CTM_OK;
}

void drop_graph(ctm_ctx_s& x) {
  if (x.gexec) {
    (void)hipGraphExecDestroy(x.gexec);
    x.gexec = nullptr;
  }
}

bool graph_usable(const ctm_ctx_s& x) {
  return x.cfg.use_graph && !(x.cfg.svd_resid_tol > 0) && !x.timing && !dry_run() && x.stream != nullptr;
}

}  // namespace

// ===========================================================================
// observables
// ===========================================================================
namespace {

__global__ void dot_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                           double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) acc += a[e] * b[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int np, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

ctm_status dot_dev(ctm_ctx_s& x, const double* a, const double* b, int64_t n, double* out) {
  int64_t blocks = std::min<int64_t>(256, std::max<int64_t>(1, (n + 255) / 256));
  HIPCHK(spans({{a, (size_t)n * 8}, {b, (size_t)n * 8}, {x.obs.red, (size_t)blocks * 8}, {out, 8}}, "dot"));
  if (dry_run()) return CTM_OK;
  hipLaunchKernelGGL(dot_kernel, dim3((unsigned)blocks), dim3(256), 0, x.stream, a, b, n, x.obs.red);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, x.stream, x.obs.red, (int)blocks, out);
  HIPCHK(last_err());
  return CTM_OK;
}

// Strip along the top of the frame-k window anchored at (xp0, yp0) with lx
// sites: out[a, U_0 .. U_{lx-1}, b] = C1 T1_0 .. T1_{lx-1} C2 (float64).
ctm_status top_strip(ctm_ctx_s& x, Inst& I, int k, int xp0, int yp0, int lxw, double* out,
                     double* w0, double* w1) {
  hipStream_t s = x.stream;
  Roles ro{&x, &I, k};
  const int64_t c = I.chi, D2 = I.D2;
  // cur [rows x chi] starting with C1 (rows = chi)
  const double* cur = ro.C(0, xp0, yp0);
  int64_t rows = c;
  double* bufs[2] = {w0, w1};
  int b = 0;
  for (int i = 0; i < lxw; ++i) {
    double* dst = bufs[b];
    CHK(gemm1(s, F64, F64, rows, D2 * c, c, rowmajor(c), cur, rowmajor(D2 * c), ro.T(0, xp0 + i, yp0),
              rowmajor(D2 * c), dst));
    cur = dst;
    rows *= D2;
    b ^= 1;
  }
  CHK(gemm1(s, F64, F64, rows, c, c, rowmajor(c), cur, rowmajor(c), ro.C(1, xp0 + lxw - 1, yp0),
            rowmajor(c), out));
  return CTM_OK;
}

// Z10 of the frame-k window anchored at (xp0, yp0) of lxw x lyw sites: the top
// strip joined directly to the bottom strip.  The bottom strip is the top strip
// of the picture turned by two more quarter turns; joining reverses all legs.
ctm_status z10(ctm_ctx_s& x, Inst& I, int k, int xp0, int yp0, int lxw, int lyw, double* out) {
  Obs& O = x.obs;
  const int64_t c = I.chi, D2 = I.D2;
  CHK(top_strip(x, I, k, xp0, yp0, lxw, O.t0, O.t2, O.t3));
  int lx, ly;
  frame_dims(k, x.Lx, x.Ly, lx, ly);
  // frame-(k+2) coordinates of the bottom-right site of the window
  int bx = xp0 + lxw - 1, by = yp0 + lyw - 1;
  int ax = pmod(-bx, lx), ay = pmod(-by, ly);
  CHK(top_strip(x, I, (k + 2) % 4, ax, ay, lxw, O.t1, O.t2, O.t3));
  int64_t dims[8];
  int perm[8];
  int nd = lxw + 2;
  dims[0] = c;
  for (int i = 0; i < lxw; ++i) dims[1 + i] = D2;
  dims[nd - 1] = c;
  for (int i = 0; i < nd; ++i) perm[i] = nd - 1 - i;
  HIPCHK(permute(x.stream, F64, O.t1, F64, O.t2, nd, dims, perm));
  int64_t tot = c * c;
  for (int i = 0; i < lxw; ++i) tot *= D2;
  return dot_dev(x, O.t0, O.t2, tot, out);
}

// Z00 = Tr(C1 C2 C3 C4) of the frame-0 window of the cell anchored at (0, 0).
ctm_status z00(ctm_ctx_s& x, Inst& I, double* out) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  Roles ro{&x, &I, 0};
  const int64_t c = I.chi;
  const int lx = x.Lx, ly = x.Ly;
  CHK(gemm1(s, F64, F64, c, c, c, rowmajor(c), ro.C(0, 0, 0), rowmajor(c), ro.C(1, lx - 1, 0), rowmajor(c), O.t0));
  // (C3 C4)^T written through a transposed output view
  CHK(gemm1(s, F64, F64, c, c, c, rowmajor(c), ro.C(2, lx - 1, ly - 1), rowmajor(c), ro.C(3, 0, ly - 1),
            colmajor(c), O.t1));
  return dot_dev(x, O.t0, O.t1, c * c, out);
}

// Left block of the frame-k site (xp, yp) with the double-layer matrix bq
// [(L,U) x (Dn,R)]:  out[e, R, z] = sum C1 T1 T4 a C4 T3 (legs: e = T1's
// C2-side, R = a's right leg, z = T3's C3-side).  G1/B1 are recomputed only
// when `prep` is true.
ctm_status left_block(ctm_ctx_s& x, Inst& I, int k, int xp, int yp, const double* bq, double* out,
                      bool prep) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  Roles ro{&x, &I, k};
  const int64_t c = I.chi, D2 = I.D2;
  if (prep) {
    // CT[p, (U, e)] = C1[p, n] T1[n, (U, e)]
    CHK(gemm1(s, F64, F64, c, D2 * c, c, rowmajor(c), ro.C(0, xp, yp), rowmajor(D2 * c), ro.T(0, xp, yp),
              rowmajor(D2 * c), O.CT));
    // G1[(g,L), (U,e)] = T4[(g,L), p] CT[p, (U,e)]
    CHK(gemm1(s, F64, F64, c * D2, D2 * c, c, rowmajor(c), ro.T(3, xp, yp), rowmajor(D2 * c), O.CT,
              rowmajor(D2 * c), O.G1));
    // B1[(z,Dn), g] = T3[(z,Dn), q] C4[q, g]
    CHK(gemm1(s, F64, F64, c * D2, c, c, rowmajor(c), ro.T(2, xp, yp), rowmajor(c), ro.C(3, xp, yp),
              rowmajor(c), O.B1));
  }
  // H[(g,e),(Dn,R)] = sum_(L,U) G1[g,L,U,e] bq[(L,U),(Dn,R)]
  {
    View va = view2(c, 1, D2 * D2 * c, BIG, c, 0);
    CHK(gemm1(s, F64, F64, c * c, D2 * D2, D2 * D2, va, O.G1, rowmajor(D2 * D2), bq, rowmajor(D2 * D2), O.H));
  }
  // out[(e,R), z] = sum_(g,Dn) H[(g,e),(Dn,R)] B1[(z,Dn), g]
  {
    View va = view2(D2, 1, D2 * D2, D2, D2, c * D2 * D2);
    View vb = view2(D2, c, 1, BIG, D2 * c, 0);
    CHK(gemm1(s, F64, F64, c * D2, c, c * D2, va, O.H, vb, O.B1, rowmajor(c), out));
  }
  return CTM_OK;
}

// Z11 of a 1x1 cell: left block (C1 T1 / T4 a / C4 T3) joined to C2 T2 C3.
ctm_status z11_1x1(ctm_ctx_s& x, Inst& I, double* out) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  Roles ro{&x, &I, 0};
  const int64_t c = I.chi, D2 = I.D2;
  CHK(left_block(x, I, 0, 0, 0, ro.b64(0, 0, 0), O.t0, true));
  // right part [e, R, z] = C2[e, b] T2[b, (R, t)] C3[t, z]
  CHK(gemm1(s, F64, F64, c, D2 * c, c, rowmajor(c), ro.C(1, 0, 0), rowmajor(D2 * c), ro.T(1, 0, 0),
            rowmajor(D2 * c), O.t1));
  CHK(gemm1(s, F64, F64, c * D2, c, c, rowmajor(c), O.t1, rowmajor(c), ro.C(2, 0, 0), rowmajor(c), O.t2));
  return dot_dev(x, O.t0, O.t2, c * D2 * c, out);
}

// Z11 of a 2x2 cell: Tr(Q1 Q2 Q3 Q4) of the frame-0 plaquette at (0, 0), float64.
ctm_status z11_2x2(ctm_ctx_s& x, Inst& I, double* out) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  Roles ro{&x, &I, 0};
  const int64_t n = I.n;
  std::vector<CornerJob> jobs;
  const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
  for (int q = 0; q < 4; ++q) {
    CornerJob j;
    j.C = ro.C(q, cx[q], cy[q]);
    j.Tn = ro.T(q, cx[q], cy[q]);
    j.Tp = ro.T((q + 3) % 4, cx[q], cy[q]);
    j.b = ro.b64(cx[q], cy[q], q);
    j.X = O.X;
    j.Y = O.Y;
    j.Q = O.Q[q];
    std::vector<CornerJob> one{j};
    CHK(corner_chain(s, F64, F64, I.chi, I.D2, one, nullptr, false));
  }
  CHK(gemm1(s, F64, F64, n, n, n, rowmajor(n), O.Q[0], rowmajor(n), O.Q[1], rowmajor(n), O.Uh));
  CHK(gemm1(s, F64, F64, n, n, n, rowmajor(n), O.Q[2], rowmajor(n), O.Q[3], colmajor(n), O.LhT));
  return dot_dev(x, O.Uh, O.LhT, n * n, out);
}

// Z11 of a general Lx x Ly cell by row transfer: the top strip
// [a, U_0 .. U_{Lx-1}, b] absorbs, row by row, the left edge T4, the double
// layers of the row and the right edge T2; the result is joined to the
// bottom strip (as in z10).  The largest intermediate holds chi^2 D^(2 Lx + 2)
// entries, so this serves cells whose observables scratch was sized for it.
ctm_status z11_rows(ctm_ctx_s& x, Inst& I, double* out) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  Roles ro{&x, &I, 0};
  const int64_t c = I.chi, D2 = I.D2, D4 = D2 * D2;
  const int Lx = x.Lx, Ly = x.Ly;
  int64_t need = c * c * D2;
  for (int i = 0; i < Lx; ++i) need *= D2;
  if ((size_t)need > O.big || !O.rows_ok)
    return fail(CTM_E_INVALID, "norm per site of this cell needs more observables scratch than was planned");
  double* cur = O.t0;
  double* nxt = O.t1;
  CHK(top_strip(x, I, 0, 0, 0, Lx, cur, O.t2, O.t3));  // [a, U_0.., b]
  int64_t Pw = 1;                                      // D2^Lx
  for (int i = 0; i < Lx; ++i) Pw *= D2;
  for (int y = 0; y < Ly; ++y) {
    // [g, L, U_0.., b] = T4[(g, L), a] v[a, (U.., b)]
    CHK(gemm1(s, F64, F64, c * D2, Pw * c, c, rowmajor(c), ro.T(3, 0, y), rowmajor(Pw * c), cur,
              rowmajor(Pw * c), nxt));
    std::swap(cur, nxt);
    int64_t P = c, Q = Pw / D2 * c;  // prefix (g, Dn_0..Dn_{x-1}), suffix (U_{x+1}.., b)
    for (int sx = 0; sx < Lx; ++sx) {
      // out[p, (Dn, R), q] = sum_(L,U) v[p, (L, U_x), q] a[(L, U), (Dn, R)]
      View va = view2(Q, 1, D4 * Q, BIG, Q, 0);
      View vc = view2(Q, 1, D4 * Q, BIG, Q, 0);
      CHK(gemm1(s, F64, F64, P * Q, D4, D4, va, cur, rowmajor(D4), ro.b64(sx, y, 0), vc, nxt));
      std::swap(cur, nxt);
      P *= D2;
      Q /= D2;
    }
    // [g, Dn.., b'] = sum_(R, b) v[(g, Dn..), (R, b)] T2[b, R, b']
    View vb = view2(c, D2 * c, c, BIG, 1, 0);
    CHK(gemm1(s, F64, F64, c * Pw, c, D2 * c, rowmajor(D2 * c), cur, vb, ro.T(1, Lx - 1, y), rowmajor(c), nxt));
    std::swap(cur, nxt);
  }
  // bottom strip: the top strip two turns on, legs reversed (as in z10)
  double* bot = nxt;
  int lx, ly;
  frame_dims(2, x.Lx, x.Ly, lx, ly);
  const int ax = pmod(-(Lx - 1), lx), ay = pmod(-(Ly - 1), ly);
  CHK(top_strip(x, I, 2, ax, ay, Lx, O.t2, bot, O.t3));
  int64_t dims[8];
  int perm[8];
  const int nd = Lx + 2;
  dims[0] = c;
  for (int i = 0; i < Lx; ++i) dims[1 + i] = D2;
  dims[nd - 1] = c;
  for (int i = 0; i < nd; ++i) perm[i] = nd - 1 - i;
  HIPCHK(permute(x.stream, F64, O.t2, F64, bot, nd, dims, perm));
  return dot_dev(x, cur, bot, c * c * Pw, out);
}

ctm_status kappa(ctm_ctx_s& x, Inst& I, double* kap) {
  Obs& O = x.obs;
  double* v = O.vals;
  if (x.Lx == 1 && x.Ly == 1) {
    CHK(z11_1x1(x, I, v + 0));
  } else if (x.Lx == 2 && x.Ly == 2) {
    CHK(z11_2x2(x, I, v + 0));
  } else {
    CHK(z11_rows(x, I, v + 0));
  }
  CHK(z00(x, I, v + 1));
  CHK(z10(x, I, 0, 0, 0, x.Lx, x.Ly, v + 2));
  // Z01: the left strip is the top strip of the picture turned by three
  // quarter turns, anchored at the frame coordinates of site (0, Ly-1)
  int ax, ay;
  to_frame(3, 0, x.Ly - 1, x.Lx, x.Ly, ax, ay);
  CHK(z10(x, I, 3, ax, ay, x.Ly, x.Lx, v + 3));
  double h[4];
  HIPCHK(d2h(h, v, 4 * sizeof(double), x.stream));
  HIPCHK(ssync(x.stream));
  double kc = h[0] * h[1] / (h[2] * h[3]);
  int ns = x.Lx * x.Ly;
  if (ns > 1) kc = (kc < 0 ? -1.0 : 1.0) * std::pow(std::fabs(kc), 1.0 / ns);
  *kap = kc;
  return CTM_OK;
}

__global__ void rdm_finalize_kernel(const double* __restrict__ raw, int d1, int d2, double* __restrict__ rho,
                                    const double* __restrict__ h, double* __restrict__ out3) {
  // raw[(s1,s1'),(s2,s2')] -> rho[(s1,s2),(s1',s2')] / trace; out3 = {herm defect, tr(rho h), trace}
  __shared__ double red[256];
  __shared__ double s_tr;
  const int m = d1 * d2;
  double tr = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    int s1 = i / d2, s2 = i % d2;
    tr += raw[(s1 * d1 + s1) * (d2 * d2) + s2 * d2 + s2];
  }
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) s_tr = red[0];
  __syncthreads();
  const double t = s_tr;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    int r = e / m, cc = e % m;
    int s1 = r / d2, s2 = r % d2, p1 = cc / d2, p2 = cc % d2;
    rho[e] = raw[(s1 * d1 + p1) * (d2 * d2) + s2 * d2 + p2] / t;
  }
  __syncthreads();
  double num = 0.0, den = 0.0, ev = 0.0;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    int r = e / m, cc = e % m;
    double a = rho[e], b = rho[cc * m + r];
    num += (a - b) * (a - b);
    den += a * a;
    if (h) ev += a * h[cc * m + r];
  }
  double vals[3] = {num, den, ev};
  for (int q = 0; q < 3; ++q) {
    __syncthreads();
    red[threadIdx.x] = vals[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    vals[q] = red[0];
  }
  if (threadIdx.x == 0) {
    out3[0] = sqrt(vals[0] / vals[1]);
    out3[1] = vals[2];
    out3[2] = t;
  }
}

// Complex kets: raw[sigma1, sigma2] is the contraction in the real basis V of
// the physical pairs (slot (x, x) <- e_(x,x); for x < x' slot (x, x') <-
// (e_(x,x') + e_(x',x)) / sqrt 2 and slot (x', x) <- i (e_(x,x') - e_(x',x)) /
// sqrt 2).  The pair p = (s, s') comes back as sum over sigma of
// conj(V[sigma, p]) raw[sigma, .]:  x < x': raw[upper] / sqrt 2 - i raw[lower] /
// sqrt 2;  x > x': raw[upper] / sqrt 2 + i raw[lower] / sqrt 2.
// rho[(s1,s2),(s1',s2')] (complex, interleaved) = R[(s1,s1'),(s2,s2')] / trace;
// out3 = {hermiticity defect ||rho - rho^H|| / ||rho||, Re tr(rho h), trace}.
__device__ __forceinline__ int back_terms(int x, int xp, int d, int* slot, double* cr, double* ci) {
  const double h = 0.70710678118654752440;
  if (x == xp) { slot[0] = x * d + x; cr[0] = 1.0; ci[0] = 0.0; return 1; }
  const int lo = x < xp ? x : xp, hi = x < xp ? xp : x;
  slot[0] = lo * d + hi; cr[0] = h; ci[0] = 0.0;          // upper slot
  slot[1] = hi * d + lo; cr[1] = 0.0; ci[1] = x < xp ? -h : h;  // lower slot
  return 2;
}

__global__ void rdm_cplx_finalize_kernel(const double* __restrict__ raw, int d, double* __restrict__ rho,
                                         const double* __restrict__ h, double* __restrict__ out3) {
  __shared__ double red[256];
  __shared__ double s_tr;
  const int m = d * d, m2 = m * m;
  double tr = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int s1 = i / d, s2 = i % d;
    tr += raw[(s1 * d + s1) * m + s2 * d + s2];
  }
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) s_tr = red[0];
  __syncthreads();
  const double t = s_tr;
  for (int e = threadIdx.x; e < m2; e += blockDim.x) {
    const int r = e / m, cc = e % m;
    const int s1 = r / d, s2 = r % d, p1 = cc / d, p2 = cc % d;
    int sa[2], sb[2];
    double ar[2], ai[2], br[2], bi[2];
    const int na = back_terms(s1, p1, d, sa, ar, ai), nb = back_terms(s2, p2, d, sb, br, bi);
    double vr = 0.0, vi = 0.0;
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < nb; ++j) {
        const double w = raw[(int64_t)sa[i] * m + sb[j]];
        const double cr = ar[i] * br[j] - ai[i] * bi[j], ci = ar[i] * bi[j] + ai[i] * br[j];
        vr += cr * w;
        vi += ci * w;
      }
    rho[2 * e] = vr / t;
    rho[2 * e + 1] = vi / t;
  }
  __syncthreads();
  double num = 0.0, den = 0.0, ev = 0.0;
  for (int e = threadIdx.x; e < m2; e += blockDim.x) {
    const int r = e / m, cc = e % m;
    const double xr = rho[2 * e], xi = rho[2 * e + 1];
    const double yr = rho[2 * (cc * m + r)], yi = -rho[2 * (cc * m + r) + 1];  // (rho^H)[r][cc]
    num += (xr - yr) * (xr - yr) + (xi - yi) * (xi - yi);
    den += xr * xr + xi * xi;
    if (h) ev += xr * h[cc * m + r];
  }
  double vals[3] = {num, den, ev};
  for (int q = 0; q < 3; ++q) {
    __syncthreads();
    red[threadIdx.x] = vals[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    vals[q] = red[0];
  }
  if (threadIdx.x == 0) {
    out3[0] = vals[1] > 0 ? sqrt(vals[0] / vals[1]) : 0.0;
    out3[1] = vals[2];
    out3[2] = t;
  }
}

// Two-site density matrix of the bond from (x, y) to the right (vertical = 0)
// or lower neighbour, left in O.rho (d^2 x d^2) with O.vals[4..6] = {herm
// defect, tr(rho h), trace}.  Built from left blocks with open physical legs:
// for every (s, s') the double layer A_s (x) B_s' replaces a.
ctm_status rdm(ctm_ctx_s& x, Inst& I, int sx, int sy, int vertical, const double* hdev) {
  hipStream_t s = x.stream;
  Obs& O = x.obs;
  const int k = vertical ? 1 : 0;
  int xp, yp;
  to_frame(k, sx, sy, x.Lx, x.Ly, xp, yp);
  // right site in frame k is (xp+1, yp); its block is a left block two turns on
  int rx, ry;
  {
    int ox, oy;
    frame_site(k, xp + 1, yp, x.Lx, x.Ly, ox, oy);
    to_frame((k + 2) % 4, ox, oy, x.Lx, x.Ly, rx, ry);
  }
  const int64_t c = I.chi, D2 = I.D2, a8 = D2 * D2 * D2 * D2;
  const int D = I.D, d = I.d;
  const int64_t t5s = (int64_t)D * D * D * D;  // one physical slice of A
  const int64_t blk = c * D2 * c;
  const bool cplx = x.cfg.complex_tensors != 0;
  const int64_t d4 = (int64_t)d * d * d * d;
  double* raw = O.rho + (cplx ? 2 : 1) * d4;
  for (int side = 0; side < 2; ++side) {
    int kk = side == 0 ? k : (k + 2) % 4;
    int px = side == 0 ? xp : rx, py = side == 0 ? yp : ry;
    Roles ro{&x, &I, kk};
    int t = ro.tid(px, py);
    double* dst = side == 0 ? O.Lall : O.Rall;
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2) {
        double* outs[4] = {O.ab, O.ab + a8, O.ab + 2 * a8, O.ab + 3 * a8};
        // complex kets: the real open double layer of physical slot (s1, s2)
        if (cplx) HIPCHK(double_layer_cplx(s, I.Ac[t], d, D, s1 * d + s2, outs));
        else HIPCHK(double_layer(s, I.A[t] + s1 * t5s, I.B[t] + s2 * t5s, 1, D, outs, 0));
        CHK(left_block(x, I, kk, px, py, O.ab + (kk % 4) * a8, dst + (int64_t)(s1 * d + s2) * blk,
                       s1 == 0 && s2 == 0));
      }
  }
  // Rp[(s2,s2')][e][R][z] = Rall[(s2,s2')][z][R][e]
  {
    int64_t dims[4] = {(int64_t)d * d, c, D2, c};
    int perm[4] = {0, 3, 2, 1};
    HIPCHK(permute(s, F64, O.Rall, F64, O.Rp, 4, dims, perm));
  }
  // raw[(s1,s1'),(s2,s2')] = Lall . Rp^T
  CHK(gemm1(s, F64, F64, (int64_t)d * d, (int64_t)d * d, blk, rowmajor(blk), O.Lall, transposed(rowmajor(blk)),
            O.Rp, rowmajor((int64_t)d * d), raw));
  HIPCHK(spans({{O.rho, (size_t)(cplx ? 3 : 2) * d4 * 8}, {hdev, hdev ? (size_t)d4 * 8 : 0},
                {O.vals + 4, 3 * 8}}, "rdm finalize"));
  if (!dry_run()) {
    if (cplx)
      hipLaunchKernelGGL(rdm_cplx_finalize_kernel, dim3(1), dim3(256), 0, s, raw, d, O.rho, hdev, O.vals + 4);
    else
      hipLaunchKernelGGL(rdm_finalize_kernel, dim3(1), dim3(256), 0, s, raw, d, d, O.rho, hdev, O.vals + 4);
  }
  HIPCHK(last_err());
  return CTM_OK;
}

// One JSON line per instance that swept since the last check: the change of
// the corner spectra, the subspace width and live extent, and per cut (keyed
// by the move direction, indexed by the site that owns the cut) the kept
// count, the weight of the subspace's singular values beyond it
// (sum_{i >= chi_eff} s_i^2 / sum_i s_i^2 over the k computed values) and the
// largest kept residual; with flag 1 also the norm per site.
ctm_status write_metrics(ctm_ctx_s& x, int sweep, const std::vector<char>& live, const std::vector<double>& delta,
                         double ms_per_sweep) {
  const int npos = x.Lx * x.Ly;
  std::vector<SolveStatus> st((size_t)4 * npos);
  static const char* names[4] = {"L", "R", "U", "D"};
  static const int dirs[4] = {CTM_LEFT, CTM_RIGHT, CTM_UP, CTM_DOWN};
  for (int i = 0; i < x.ninst; ++i) {
    if (!live[i]) continue;
    Inst& I = x.inst[i];
    HIPCHK(d2h(st.data(), I.skeep_all, st.size() * sizeof(SolveStatus), x.stream));
    HIPCHK(ssync(x.stream));
    double kap = NAN;
    const bool want_kappa = (x.metrics_flags & 1) != 0;
    if (want_kappa && kappa(x, I, &kap) != CTM_OK) kap = NAN;
    std::string line = "{\"inst\": " + std::to_string(i) + ", \"sweep\": " + std::to_string(sweep);
    char buf[64];
    auto num = [&](double v) -> std::string {
      if (!std::isfinite(v)) return "null";
      std::snprintf(buf, sizeof buf, "%.6e", v);
      return buf;
    };
    line += ", \"delta\": " + num(delta[i]);
    line += ", \"width\": " + std::to_string(I.k_act) + ", \"live_chi\": " + std::to_string(I.chi);
    line += ", \"ms_per_sweep\": " + num(ms_per_sweep);
    if (want_kappa) line += ", \"kappa\": " + num(kap);
    const char* fields[3] = {"chi_eff", "discarded", "max_resid"};
    for (int f = 0; f < 3; ++f) {
      line += std::string(", \"") + fields[f] + "\": {";
      for (int o = 0; o < 4; ++o) {
        const int k = frame_of_dir(dirs[o]);
        line += std::string(o ? ", " : "") + "\"" + names[o] + "\": [";
        for (int q = 0; q < npos; ++q) {
          const SolveStatus& t = st[(size_t)k * npos + q];
          if (q) line += ", ";
          if (f == 0) line += std::to_string(t.chi_eff);
          else if (f == 1) line += num(t.discarded);
          else line += num(t.max_resid);
        }
        line += "]";
      }
      line += "}";
    }
    line += "}\n";
    std::fputs(line.c_str(), x.metrics);
  }
  std::fflush(x.metrics);
  return CTM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void ctm_config_default(ctm_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n_inst = 1;
  c->Lx = 1;
  c->Ly = 1;
  c->n_tensors = 1;
  c->prec = CTM_FP64;
  c->svd_oversample = 16;
  c->svd_max_iters = 30;
  c->svd_resid_tol = 1e-13;
  c->svd_cutoff = 1e-12;
  c->seed = 12345;
  c->use_graph = 0;
  c->autotune = 1;
  c->concurrent_classes = 1;
}

ctm_status ctm_workspace_size(const ctm_config* cfg, size_t* bytes) {
  if (!bytes) return fail(CTM_E_INVALID, "null bytes");
  ctm_ctx_s x;
  CHK(build_ctx(cfg, x));
  *bytes = x.ws_need;
  return CTM_OK;
}

static std::once_flag g_table_once;

static ctm_status init_impl(const ctm_config* cfg, const double* const* A_dev, const double* const* B_dev,
                            void* ws_dev, size_t ws_bytes, void* stream, int32_t init,
                            const double* spectrum_host, ctm_ctx* out) {
  if (!out) return fail(CTM_E_INVALID, "null out");
  // a tile table named by CTM_TILE_TABLE is loaded at the first ctm_init
  ctm_status tst = CTM_OK;
  std::call_once(g_table_once, [&] {
    const char* t = std::getenv("CTM_TILE_TABLE");
    if (t && t[0]) tst = ctm_tile_table_load(t, nullptr);
  });
  if (tst != CTM_OK) return tst;
  *out = nullptr;
  if (!A_dev) return fail(CTM_E_INVALID, "null tensors");
  if (init != CTM_INIT_TRIVIAL && init != CTM_INIT_DIAG) return fail(CTM_E_INVALID, "init kind");
  ctm_ctx_s* x = new ctm_ctx_s();
  ctm_status st = build_ctx(cfg, *x);
  if (st != CTM_OK) { delete x; return st; }
  if (!ws_dev || ws_bytes < x->ws_need) {
    size_t need = x->ws_need;
    delete x;
    return fail(CTM_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  if (((uintptr_t)ws_dev) & 255) { delete x; return fail(CTM_E_INVALID, "workspace must be 256-byte aligned"); }
  x->stream = (hipStream_t)stream;
  const char* dr = std::getenv("CTM_DRY_RUN");
  x->reg.dry = dr && dr[0] == '1';
  x->reg.lo = (uintptr_t)ws_dev;
  x->reg.hi = (uintptr_t)ws_dev + x->ws_need;
  Arena ar;
  ar.base = (char*)ws_dev;
  ar.reg = &x->reg;
  plan(*x, ar);
  std::sort(x->reg.allocs.begin(), x->reg.allocs.end());
  RegGuard guard(&x->reg);
  auto cleanup = [&](ctm_status s) { delete x; return s; };
  // copy tensors and check them
  for (int i = 0; i < x->ninst; ++i) {
    Inst& I = x->inst[i];
    const size_t t5 = (size_t)I.d * I.D2 * I.D2;
    const bool cplx = x->cfg.complex_tensors != 0;
    for (int t = 0; t < x->ntens; ++t) {
      const double* a = A_dev[i * x->ntens + t];
      const double* b = B_dev ? B_dev[i * x->ntens + t] : a;
      if (!a || !b) return cleanup(fail(CTM_E_INVALID, "null tensor pointer"));
      if (cplx) {
        // the bra of a complex ket is its conjugate
        if (b != a) return cleanup(fail(CTM_E_INVALID, "complex tensors: pass no bra tensors (the bra is the conjugate)"));
        if (d2d(I.Ac[t], a, 2 * t5 * 8, x->stream) != hipSuccess) return cleanup(fail(CTM_E_HIP, "tensor copy failed"));
        continue;
      }
      if (d2d(I.A[t], a, t5 * 8, x->stream) != hipSuccess ||
          d2d(I.B[t], b, t5 * 8, x->stream) != hipSuccess)
        return cleanup(fail(CTM_E_HIP, "tensor copy failed"));
    }
    if (dmemset(I.flag, 0, 16, x->stream) != hipSuccess) return cleanup(fail(CTM_E_HIP, "memset"));
    for (int t = 0; t < x->ntens; ++t) {
      if (cplx ? nonfinite(x->stream, I.Ac[t], (int64_t)(2 * t5), I.flag) != hipSuccess
               : (nonfinite(x->stream, I.A[t], (int64_t)t5, I.flag) != hipSuccess ||
                  nonfinite(x->stream, I.B[t], (int64_t)t5, I.flag) != hipSuccess))
        return cleanup(fail(CTM_E_HIP, "nonfinite check"));
    }
    int hflag = 0;
    if (d2h(&hflag, I.flag, sizeof(int), x->stream) != hipSuccess ||
        ssync(x->stream) != hipSuccess)
      return cleanup(fail(CTM_E_HIP, "flag readback"));
    if (hflag) return cleanup(fail(CTM_E_NONFINITE, "non-finite entry in a PEPS tensor"));
    for (int t = 0; t < x->ntens; ++t) {
      if ((cplx ? double_layer_cplx(x->stream, I.Ac[t], I.d, I.D, -1, I.b64[t])
                : double_layer(x->stream, I.A[t], I.B[t], I.d, I.D, I.b64[t], 0)) != hipSuccess)
        return cleanup(fail(CTM_E_HIP, "double layer"));
      if (x->wt != F64 && !x->cfg.single_layer)
        for (int r = 0; r < 4; ++r)
          if (convert(x->stream, F64, I.b64[t][r], x->wt, I.bw[t][r], (int64_t)I.D2 * I.D2 * I.D2 * I.D2) !=
              hipSuccess)
            return cleanup(fail(CTM_E_HIP, "convert"));
      if (x->cfg.single_layer)
        for (int r = 0; r < 4; ++r) {
          // rotation r of the frame: A[s][u][l][d][r] -> [L'][U'][s][D'][R'], with
          // the legs relabelled as in the rotated double layer
          static const int perm[4][5] = {{2, 1, 0, 3, 4}, {1, 4, 0, 2, 3}, {4, 3, 0, 1, 2}, {3, 2, 0, 4, 1}};
          const int64_t dims[5] = {I.d, I.D, I.D, I.D, I.D};
          if (permute(x->stream, F64, I.A[t], x->wt, I.Sk[t][r], 5, dims, perm[r]) != hipSuccess ||
              permute(x->stream, F64, I.B[t], x->wt, I.Sb[t][r], 5, dims, perm[r]) != hipSuccess)
            return cleanup(fail(CTM_E_HIP, "single-layer tensors"));
          if (x->prec == CTM_BF16 &&
              (permute(x->stream, F64, I.A[t], BF16, I.Sk16[t][r], 5, dims, perm[r]) != hipSuccess ||
               permute(x->stream, F64, I.B[t], BF16, I.Sb16[t][r], 5, dims, perm[r]) != hipSuccess))
            return cleanup(fail(CTM_E_HIP, "single-layer tensors"));
          if (x->prec == CTM_BF16) {
            // [L'][U'][s][D'][R'] -> [D'][R'][s][L'][U'] (through the single-layer
            // scratch), rows padded to a multiple of 8; and -> [D'][R'][L'][U'][s]
            const int64_t sdims[5] = {I.D, I.D, I.d, I.D, I.D};
            const int pk[5] = {3, 4, 2, 0, 1}, pb[5] = {3, 4, 0, 1, 2};
            const int64_t kp = ((int64_t)I.D2 + 7) / 8 * 8;
            if (permute(x->stream, BF16, I.Sk16[t][r], BF16, x->sl_y, 5, sdims, pk) != hipSuccess ||
                pad_rows_bf16(x->stream, x->sl_y, (int64_t)I.d * I.D2, I.D2, kp, I.SkT16[t][r]) != hipSuccess ||
                permute(x->stream, BF16, I.Sb16[t][r], BF16, I.SbT16[t][r], 5, sdims, pb) != hipSuccess)
              return cleanup(fail(CTM_E_HIP, "single-layer bf16 operands"));
          }
        }
      if (x->prec == CTM_BF16 && !x->cfg.single_layer)
        for (int r = 0; r < 4; ++r) {
          int64_t dims[2] = {(int64_t)I.D2 * I.D2, (int64_t)I.D2 * I.D2};
          int perm[2] = {1, 0};
          if (permute(x->stream, F64, I.b64[t][r], BF16, I.bT[t][r], 2, dims, perm) != hipSuccess)
            return cleanup(fail(CTM_E_HIP, "transpose double layer"));
          if (I.bTp[t][r] && corner_bf16_pack_b(x->stream, I.bT[t][r], dims[0], dims[1], I.bTp[t][r]) != hipSuccess)
            return cleanup(fail(CTM_E_HIP, "pack double layer"));
          // B side of the three-term product: rows (dn,R), columns (l,u)
          const int64_t K4 = (int64_t)I.D2 * I.D2;
          if (split3_bf16(x->stream, F64, I.b64[t][r], transposed(rowmajor(K4)), K4, K4, false, I.bT3[t][r]) !=
              hipSuccess)
            return cleanup(fail(CTM_E_HIP, "split double layer"));
          if (I.bT3p[t][r] && corner_bf16_pack_b(x->stream, I.bT3[t][r], K4, 3 * K4, I.bT3p[t][r]) != hipSuccess)
            return cleanup(fail(CTM_E_HIP, "pack split double layer"));
        }
    }
    st = init_env(*x, I, i, init, spectrum_host);
    if (st != CTM_OK) return cleanup(st);
  }
  *out = x;
  return CTM_OK;
}

ctm_status ctm_init(const ctm_config* cfg, const double* const* A_dev, const double* const* B_dev,
                    void* ws_dev, size_t ws_bytes, void* stream, int32_t init,
                    const double* spectrum_host, ctm_ctx* out) {
  return init_impl(cfg, A_dev, B_dev, ws_dev, ws_bytes, stream, init, spectrum_host, out);
}

ctm_status ctm_move(ctm_ctx x, int32_t dir, int32_t count) {
  if (!x) return fail(CTM_E_INVALID, "null ctx");
  RegGuard guard(&x->reg);
  TuneGuard tg(x->cfg.autotune != 0);
  if (count < 0 || dir < 0 || dir > CTM_SWEEP) return fail(CTM_E_INVALID, "dir/count");
  for (auto& cls : x->classes) {
    std::vector<Inst*> insts = class_insts(*x, cls);
    if (dir == CTM_SWEEP) {
      for (int i = 0; i < count; ++i) {
        CHK(do_sweep(*x, insts));
        CHK(grow_if_capped(*x, cls));
      }
    } else {
      x->resid_step = true;
      for (int i = 0; i < count; ++i) {
        CHK(do_move(*x, insts, frame_of_dir(dir), 1));
        CHK(grow_if_capped(*x, cls));
      }
    }
  }
  return CTM_OK;
}

ctm_status ctm_converge(ctm_ctx x, double tol, int32_t max_sweeps, int32_t check_every,
                        int32_t* sweeps_out, double* delta_out) {
  if (!x) return fail(CTM_E_INVALID, "null ctx");
  RegGuard guard(&x->reg);
  TuneGuard tg(x->cfg.autotune != 0);
  if (max_sweeps < 0 || !(tol >= 0)) return fail(CTM_E_INVALID, "tol/max_sweeps");
  if (check_every < 1) check_every = 1;
  const int ni = x->ninst;
  // every instance sweeps until its own change is below tol; instances of a
  // class that are still sweeping move together
  std::vector<int> done(ni, 0), conv(ni, 0);
  std::vector<char> live(ni, 1);
  std::vector<double> dl(ni, INFINITY);
  std::vector<double> hd(ni);
  std::vector<int> hf(4 * ni);
  bool bad = false;
  bool cursors0 = true;
  for (const Inst& I : x->inst)
    for (int c = 0; c < 4; ++c) cursors0 = cursors0 && I.cursor[c] == 0;
  const bool graph = graph_usable(*x) && cursors0;
  drop_graph(*x);
  int sweep = 0, last_check = 0;
  auto t_check = std::chrono::steady_clock::now();
  bool eager_next = true;  // an eager sweep tunes new GEMM shapes before a capture
  while (sweep < max_sweeps) {
    const bool use_graph = graph && !eager_next;
    eager_next = false;
    if (use_graph) {
      CHK(capture_sweep(*x, live));
      HIPCHK(hipGraphLaunch(x->gexec, x->stream));
      int nl = 0;
      for (int i = 0; i < ni; ++i) nl += live[i];
      x->moves += (int64_t)(2 * x->Lx + 2 * x->Ly) * nl;
    } else {
      for (auto& cls : x->classes) {
        std::vector<Inst*> insts = live_insts(*x, cls, live);
        if (insts.empty()) continue;
        CHK(do_sweep(*x, insts));
        CHK(corner_spectra(*x, insts, false, true));
      }
    }
    ++sweep;
    const bool check = (sweep % check_every == 0) || sweep == max_sweeps;
    if (!check) continue;
    HIPCHK(d2h(hd.data(), x->delta_all, (size_t)ni * 8, x->stream));
    HIPCHK(d2h(hf.data(), x->flag_all, (size_t)ni * 16, x->stream));
    HIPCHK(ssync(x->stream));
    if (x->metrics) {
      const auto now = std::chrono::steady_clock::now();
      const double ms = std::chrono::duration<double, std::milli>(now - t_check).count() / (sweep - last_check);
      CHK(write_metrics(*x, sweep, live, hd, ms));
      t_check = std::chrono::steady_clock::now();
      last_check = sweep;
    }
    // the subspace follows the number of kept singular values: chi_eff + p
    // columns suffice, and chi_eff can grow by p per column step.  After a
    // full sweep every corner and edge was produced by one of the solves
    // whose kept counts are read here, so none extends past the largest of
    // them, and the live extent can follow the new width.  A kept count
    // equal to the width means the width, not chi or the cutoff, set the
    // truncation: the subspace grows and that check cannot end the run.
    std::vector<char> capped(ni, 0);
    for (auto& cls : x->classes) {
      int ce = 0;
      for (int i : cls)
        if (live[i]) ce = std::max(ce, hf[4 * i + 1]);
      Inst& J = x->inst[cls[0]];
      const bool cap = ce > 0 && ce >= J.k_act && J.k_act < J.k && !x->width_pinned;
      if (cap)
        for (int i : cls) capped[i] = 1;
      const int p = std::max(0, x->cfg.svd_oversample);
      int kw = ce + p;
      // fixed-count mode: up to 4 of the p extra columns are dropped when
      // that saves a partial 16-column tile of the half-system products
      if (!(x->cfg.svd_resid_tol > 0) && p >= 8 && kw / 16 * 16 >= ce + p - 4) kw = kw / 16 * 16;
      if (cap) kw = std::max(kw, J.k_act + std::max(1, p));
      const int kn = std::max(1, std::min(J.k, kw));
      if (ce > 0 && kn != J.k_act && !x->width_pinned) {
        CHK(set_width(*x, cls, kn));
        eager_next = true;
        drop_graph(*x);
      }
    }
    bool all = true;
    for (int i = 0; i < ni; ++i) {
      if (!live[i]) continue;
      done[i] = sweep;
      dl[i] = hd[i];
      if (hf[4 * i] || !std::isfinite(hd[i])) bad = true;
      else if (hd[i] < tol && !capped[i]) {
        conv[i] = 1;
        live[i] = 0;
        drop_graph(*x);  // the live set changed
      }
      all = all && conv[i];
    }
    if (bad || all) break;
  }
  drop_graph(*x);
  bool all_ok = true;
  for (int i = 0; i < ni; ++i) {
    if (sweeps_out) sweeps_out[i] = done[i];
    if (delta_out) delta_out[i] = dl[i];
    all_ok = all_ok && conv[i];
  }
  if (bad) return fail(CTM_E_NONFINITE, "non-finite corner spectrum");
  if (!all_ok) return fail(CTM_E_NOCONV, "not converged within max_sweeps");
  return CTM_OK;
}

ctm_status ctm_set_metrics(ctm_ctx x, const char* path, int32_t flags) {
  if (!x) return fail(CTM_E_INVALID, "null ctx");
  if (x->metrics && x->metrics_own) std::fclose(x->metrics);
  x->metrics = nullptr;
  x->metrics_own = false;
  x->metrics_flags = flags;
  if (!path) return CTM_OK;
  if (std::strcmp(path, "-") == 0) {
    x->metrics = stderr;
    return CTM_OK;
  }
  x->metrics = std::fopen(path, "a");
  if (!x->metrics) return fail(CTM_E_INVALID, std::string("cannot open ") + path);
  x->metrics_own = true;
  return CTM_OK;
}

ctm_status ctm_spectra(ctm_ctx x, int32_t inst, double* out) {
  if (!x || !out || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  CHK(corner_spectra(*x, std::vector<Inst*>{&I}, false, false));
  HIPCHK(d2h(out, I.spec_new, (size_t)x->Lx * x->Ly * 4 * I.chi_cap * 8, x->stream));
  HIPCHK(ssync(x->stream));
  return CTM_OK;
}

}  // extern "C"

namespace {
// U[:, j] *= s[j] for the k x k row-major U of every problem
__global__ void scale_cols_kernel(PtrSet U, CPtrSet S, int k) {
  double* u = U.p[blockIdx.y];
  const double* sv = S.p[blockIdx.y];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) u[e] *= sv[e % k];
}
}  // namespace

extern "C" {

ctm_status ctm_set_corner_spectra(ctm_ctx x, int32_t inst, const double* spec_host) {
  if (!x || !spec_host || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  hipStream_t s = x->stream;
  const int npos = x->Lx * x->Ly, nc = 4 * npos, cl = I.chi, cc = I.chi_cap;
  const size_t c2 = (size_t)cl * cl, n16 = (size_t)2 * cl * ((cl + 15) / 16 * 16);
  for (size_t i = 0; i < (size_t)nc * cc; ++i)
    if (!std::isfinite(spec_host[i]) || spec_host[i] < 0) return fail(CTM_E_INVALID, "spectrum must be finite and >= 0");
  // the new values, staged in spec_new (recomputed below)
  HIPCHK(h2d(I.spec_new, spec_host, (size_t)nc * cc * 8, s));
  for (int c0 = 0; c0 < nc; c0 += MAXP) {
    const int cnt = std::min(MAXP, nc - c0);
    CPtrSet M{}, Sn{};
    PtrSet U{}, S{}, W{}, J{};
    G g;
    for (int j = 0; j < cnt; ++j) {
      const int c = c0 + j;
      double* C = I.C[c % 4][c / 4];
      M.p[j] = C;
      U.p[j] = x->spec_tmp_U + (size_t)j * c2;
      W.p[j] = x->spec_tmp_W + (size_t)j * c2;
      S.p[j] = x->spec_tmp_S + (size_t)j * cl;
      J.p[j] = x->spec_tmp_J + (size_t)j * n16;
      Sn.p[j] = I.spec_new + (size_t)c * cc;
      g.add(U.p[j], W.p[j], C);
    }
    // C = U S W^T, then C <- U diag(s_new) W^T (directions of zero singular
    // value have no left vector and stay zero)
    HIPCHK(jacobi_svd(s, cl, M, U, S, W, J, cnt, true, false));
    HIPCHK(spans({{U.p[0], c2 * cnt * 8}}, "scale cols"));
    if (!dry_run()) hipLaunchKernelGGL(scale_cols_kernel, dim3(std::max(1, (int)std::min<size_t>(64, (c2 + 255) / 256)), cnt),
                                       dim3(256), 0, s, U, Sn, cl);
    HIPCHK(last_err());
    CHK(gemm_run(s, F64, F64, cl, cl, cl, rowmajor(cl), transposed(rowmajor(cl)), rowmajor(cl), g));
  }
  std::vector<std::pair<double*, int64_t>> nt;
  for (int c = 0; c < nc; ++c) nt.push_back({I.C[c % 4][c / 4], (int64_t)c2});
  CHK(normalize_run(*x, nt));
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < npos; ++p) I.staleC[c][p] = true;
  // the convergence measure restarts from the new spectra
  CHK(corner_spectra(*x, std::vector<Inst*>{&I}, true, true));
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_norm(ctm_ctx x, int32_t inst, double* kap) {
  if (!x || !kap || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  RegGuard guard(&x->reg);
  return kappa(*x, x->inst[inst], kap);
}

ctm_status ctm_rdm(ctm_ctx x, int32_t inst, int32_t sx, int32_t sy, int32_t vertical, double* rho_host,
                   double* herm) {
  if (!x || !rho_host || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  if (x->cfg.complex_tensors) return fail(CTM_E_INVALID, "complex tensors: the density matrix is complex (ctm_rdm_complex)");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  CHK(rdm(*x, I, pmod(sx, x->Lx), pmod(sy, x->Ly), vertical ? 1 : 0, nullptr));
  const int m = I.d * I.d;
  double v3[3];
  HIPCHK(d2h(rho_host, x->obs.rho, (size_t)m * m * 8, x->stream));
  HIPCHK(d2h(v3, x->obs.vals + 4, 3 * 8, x->stream));
  HIPCHK(ssync(x->stream));
  if (herm) *herm = v3[0];
  return CTM_OK;
}

ctm_status ctm_rdm_complex(ctm_ctx x, int32_t inst, int32_t sx, int32_t sy, int32_t vertical, double* rho_host,
                           double* herm) {
  if (!x || !rho_host || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  if (!x->cfg.complex_tensors) return fail(CTM_E_INVALID, "real tensors: use ctm_rdm");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  CHK(rdm(*x, I, pmod(sx, x->Lx), pmod(sy, x->Ly), vertical ? 1 : 0, nullptr));
  const int m = I.d * I.d;
  double v3[3];
  HIPCHK(d2h(rho_host, x->obs.rho, (size_t)m * m * 16, x->stream));
  HIPCHK(d2h(v3, x->obs.vals + 4, 3 * 8, x->stream));
  HIPCHK(ssync(x->stream));
  if (herm) *herm = v3[0];
  return CTM_OK;
}

ctm_status ctm_expect(ctm_ctx x, int32_t inst, int32_t sx, int32_t sy, int32_t vertical, const double* h_host,
                      double* value) {
  if (!x || !h_host || !value || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  const int m = I.d * I.d;
  if (!finite_host(h_host, (size_t)m * m)) return fail(CTM_E_NONFINITE, "operator");
  double* hdev = x->obs.t3;  // staging (m*m doubles fit in the scratch)
  HIPCHK(h2d(hdev, h_host, (size_t)m * m * 8, x->stream));
  CHK(rdm(*x, I, pmod(sx, x->Lx), pmod(sy, x->Ly), vertical ? 1 : 0, hdev));
  double v3[3];
  HIPCHK(d2h(v3, x->obs.vals + 4, 3 * 8, x->stream));
  HIPCHK(ssync(x->stream));
  *value = v3[1];
  return CTM_OK;
}

size_t ctm_env_bytes(ctm_ctx x, int32_t inst) {
  if (!x || inst < 0 || inst >= x->ninst) return 0;
  Inst& I = x->inst[inst];
  const size_t npos = (size_t)x->Lx * x->Ly, c2 = (size_t)I.chi_cap * I.chi_cap;
  return npos * 4 * (c2 + c2 * I.D2) * 8;
}

ctm_status ctm_env_export(ctm_ctx x, int32_t inst, void* buf, size_t bytes) {
  if (!x || !buf || bytes != ctm_env_bytes(x, inst)) return fail(CTM_E_INVALID, "args/bytes");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  const int npos = x->Lx * x->Ly;
  const size_t cl = I.chi, cc = I.chi_cap, D2 = I.D2;
  // device tensors are stored at the live extent; the buffer holds them
  // zero-padded to chi
  std::vector<double> t((size_t)cl * cl * D2);
  std::memset(buf, 0, bytes);
  double* p = (double*)buf;
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      HIPCHK(d2h(t.data(), I.C[c][q], cl * cl * 8, x->stream));
      HIPCHK(ssync(x->stream));
      for (size_t a = 0; a < cl; ++a) std::memcpy(p + a * cc, t.data() + a * cl, cl * 8);
      p += cc * cc;
    }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      HIPCHK(d2h(t.data(), I.T[c][q], cl * cl * D2 * 8, x->stream));
      HIPCHK(ssync(x->stream));
      for (size_t a = 0; a < cl; ++a)
        for (size_t u = 0; u < D2; ++u) std::memcpy(p + (a * D2 + u) * cc, t.data() + (a * D2 + u) * cl, cl * 8);
      p += cc * cc * D2;
    }
  return CTM_OK;
}

ctm_status ctm_env_import(ctm_ctx x, int32_t inst, const void* buf, size_t bytes) {
  if (!x || !buf || bytes != ctm_env_bytes(x, inst)) return fail(CTM_E_INVALID, "args/bytes");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  const int npos = x->Lx * x->Ly;
  const size_t c2 = (size_t)I.chi_cap * I.chi_cap, t3 = c2 * I.D2;
  if (!finite_host((const double*)buf, bytes / 8)) return fail(CTM_E_NONFINITE, "non-finite environment");
  // an imported environment may use every index up to chi: full extent and
  // subspace width, no kept subspaces
  I.chi = I.chi_cap;
  I.n = I.n_cap;
  I.k_act = I.k;
  const char* p = (const char*)buf;
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(h2d(I.C[c][q], p, c2 * 8, x->stream)); p += c2 * 8; }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(h2d(I.T[c][q], p, t3 * 8, x->stream)); p += t3 * 8; }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      I.has_keep[c][q] = false;
      I.staleC[c][q] = I.staleT[c][q] = true;
    }
  HIPCHK(dmemset(I.skeep_all, 0, sizeof(SolveStatus) * 4 * npos, x->stream));
  for (Row& R : I.rows) HIPCHK(dmemset(R.st, 0, sizeof(SolveStatus), x->stream));
  CHK(corner_spectra(*x, std::vector<Inst*>{&I}, true, true));
  HIPCHK(ssync(x->stream));
  return CTM_OK;
}

// Resumable state: a header, the corners and edges at the live extent, the
// previous spectra, and every kept subspace with its status.
namespace {
struct CkptHeader {
  int64_t magic, version, chi_cap, D, d, chi, k, k_act, npos, n_cap;
  int64_t cursor[4];
  int64_t has_keep[4 * MAXPOS];
};
constexpr int64_t CKPT_MAGIC = 0x43544d434b505431ll;  // "CTMCKPT1"
// version 2: solver statuses carry the discarded weight (56 bytes each)
constexpr int64_t CKPT_VERSION = 2;
size_t ckpt_bytes(const ctm_ctx_s& x, const Inst& I) {
  const size_t npos = (size_t)x.Lx * x.Ly, cc = I.chi_cap;
  return sizeof(CkptHeader) + npos * 4 * (cc * cc + cc * cc * I.D2) * 8 + npos * 4 * cc * 8 +
         npos * 4 * sizeof(SolveStatus) + npos * 4 * (size_t)I.n_cap * I.k * 8;
}
}  // namespace

size_t ctm_checkpoint_bytes(ctm_ctx x, int32_t inst) {
  if (!x || inst < 0 || inst >= x->ninst) return 0;
  return ckpt_bytes(*x, x->inst[inst]);
}

ctm_status ctm_checkpoint_save(ctm_ctx x, int32_t inst, void* buf, size_t bytes) {
  if (!x || !buf || inst < 0 || inst >= x->ninst || bytes != ckpt_bytes(*x, x->inst[inst]))
    return fail(CTM_E_INVALID, "args/bytes");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  const int npos = x->Lx * x->Ly;
  CkptHeader h{};
  h.magic = CKPT_MAGIC;
  h.version = CKPT_VERSION;
  h.chi_cap = I.chi_cap; h.D = I.D; h.d = I.d; h.chi = I.chi; h.k = I.k; h.k_act = I.k_act;
  h.npos = npos; h.n_cap = I.n_cap;
  for (int c = 0; c < 4; ++c) h.cursor[c] = I.cursor[c];
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) h.has_keep[c * MAXPOS + q] = I.has_keep[c][q] ? 1 : 0;
  char* p = (char*)buf;
  std::memset(buf, 0, bytes);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t cc = I.chi_cap, c2 = (size_t)I.chi * I.chi, t3 = c2 * I.D2;
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(d2h(p, I.C[c][q], c2 * 8, x->stream)); p += cc * cc * 8; }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(d2h(p, I.T[c][q], t3 * 8, x->stream)); p += cc * cc * I.D2 * 8; }
  HIPCHK(d2h(p, I.spec_old, (size_t)npos * 4 * cc * 8, x->stream));
  p += (size_t)npos * 4 * cc * 8;
  HIPCHK(d2h(p, I.skeep_all, (size_t)npos * 4 * sizeof(SolveStatus), x->stream));
  p += (size_t)npos * 4 * sizeof(SolveStatus);
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      HIPCHK(d2h(p, I.Vkeep[c][q], (size_t)I.n_cap * I.k * 8, x->stream));
      p += (size_t)I.n_cap * I.k * 8;
    }
  HIPCHK(ssync(x->stream));
  return CTM_OK;
}

ctm_status ctm_checkpoint_load(ctm_ctx x, int32_t inst, const void* buf, size_t bytes) {
  if (!x || !buf || inst < 0 || inst >= x->ninst || bytes != ckpt_bytes(*x, x->inst[inst]))
    return fail(CTM_E_INVALID, "args/bytes");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[inst];
  const int npos = x->Lx * x->Ly;
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != CKPT_MAGIC || h.version != CKPT_VERSION || h.chi_cap != I.chi_cap || h.D != I.D || h.d != I.d ||
      h.k != I.k || h.npos != npos || h.n_cap != I.n_cap || h.chi < 1 || h.chi > I.chi_cap || h.k_act < 1 ||
      h.k_act > I.k)
    return fail(CTM_E_INVALID, "checkpoint does not match this context");
  for (int c = 0; c < 4; ++c)
    if (h.cursor[c] < 0 || h.cursor[c] >= std::max(x->Lx, x->Ly)) return fail(CTM_E_INVALID, "checkpoint cursor");
  const char* p = (const char*)buf + sizeof(h);
  const size_t cc = I.chi_cap, cl = (size_t)h.chi, c2 = cl * cl, t3 = c2 * I.D2;
  if (!finite_host((const double*)p, npos * 4 * (cc * cc + cc * cc * I.D2 + cc)))
    return fail(CTM_E_NONFINITE, "non-finite checkpoint");
  I.chi = (int)h.chi;
  I.n = I.chi * I.D2;
  I.k_act = (int)h.k_act;
  for (int c = 0; c < 4; ++c) I.cursor[c] = (int)h.cursor[c];
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      I.has_keep[c][q] = h.has_keep[c * MAXPOS + q] != 0;
      I.staleC[c][q] = I.staleT[c][q] = true;
    }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(h2d(I.C[c][q], p, c2 * 8, x->stream)); p += cc * cc * 8; }
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) { HIPCHK(h2d(I.T[c][q], p, t3 * 8, x->stream)); p += cc * cc * I.D2 * 8; }
  HIPCHK(h2d(I.spec_old, p, (size_t)npos * 4 * cc * 8, x->stream));
  p += (size_t)npos * 4 * cc * 8;
  HIPCHK(h2d(I.skeep_all, p, (size_t)npos * 4 * sizeof(SolveStatus), x->stream));
  p += (size_t)npos * 4 * sizeof(SolveStatus);
  for (int c = 0; c < 4; ++c)
    for (int q = 0; q < npos; ++q) {
      HIPCHK(h2d(I.Vkeep[c][q], p, (size_t)I.n_cap * I.k * 8, x->stream));
      p += (size_t)I.n_cap * I.k * 8;
    }
  HIPCHK(ssync(x->stream));
  return CTM_OK;
}

ctm_status ctm_set_timing(ctm_ctx x, int32_t enable) {
  if (!x) return fail(CTM_E_INVALID, "null ctx");
  if (x->tused || x->sused) (void)hipStreamSynchronize(x->stream);  // pending records are dropped
  if (enable < 0 || enable > 2) return fail(CTM_E_INVALID, "enable must be 0, 1 or 2");
  x->tused = x->sused = 0;
  x->timing = enable != 0;
  x->phase_timing = enable == 1;
  x->t_corner = x->t_solver = x->t_absorb = x->t_stage3 = x->stage3_flop = x->stage3_flop_nom = 0;
  x->live_chi = 0;
  x->corner_launches = x->stage3_launches = x->moves = 0;
  return CTM_OK;
}

ctm_status ctm_get_timing(ctm_ctx x, double* v) {
  if (!x || !v) return fail(CTM_E_INVALID, "args");
  timing_flush(*x);
  v[0] = x->t_corner;
  v[1] = x->t_solver;
  v[2] = x->t_absorb;
  v[3] = x->t_stage3;
  v[4] = (double)x->stage3_launches;
  v[5] = x->stage3_flop;
  v[6] = (double)x->corner_launches;
  v[7] = (double)x->moves;
  v[8] = x->stage3_flop_nom;
  v[9] = (double)x->live_chi;
  return CTM_OK;
}

void ctm_destroy(ctm_ctx x) {
  if (!x) return;
  if (x->metrics && x->metrics_own) std::fclose(x->metrics);
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  for (hipStream_t cs : x->class_streams) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  for (hipEvent_t ev : x->class_events) (void)hipEventDestroy(ev);
  if (x->tused || x->sused) (void)hipStreamSynchronize(x->stream);
  for (auto& r : x->tpool)
    for (hipEvent_t e : r) (void)hipEventDestroy(e);
  for (auto& r : x->spool)
    for (hipEvent_t e : r) (void)hipEventDestroy(e);
  delete x;
}

const char* ctm_last_error(void) { return g_err.c_str(); }

ctm_status ctm_fidelity(const ctm_config* cfg, const double* const* A_dev, const double* const* B_dev,
                        void* ws_dev, size_t ws_bytes, void* stream, double tol, int32_t max_sweeps,
                        double* d_out, double* ln_d_out, int32_t* sweeps_out) {
  if (!cfg || !A_dev || !B_dev || !d_out) return fail(CTM_E_INVALID, "args");
  if (cfg->n_inst != 1) return fail(CTM_E_INVALID, "fidelity needs n_inst == 1");
  // the mixed network <B|A> of complex states has no real form
  if (cfg->complex_tensors) return fail(CTM_E_INVALID, "fidelity needs real tensors");
  double kap[3];
  const double* const* kets[3] = {A_dev, B_dev, A_dev};
  const double* const* bras[3] = {A_dev, B_dev, B_dev};
  bool all_conv = true;
  for (int r = 0; r < 3; ++r) {
    ctm_ctx x = nullptr;
    CHK(ctm_init(cfg, kets[r], bras[r], ws_dev, ws_bytes, stream, CTM_INIT_TRIVIAL, nullptr, &x));
    int32_t sw = 0;
    double dl = 0;
    ctm_status s = ctm_converge(x, tol, max_sweeps, 1, &sw, &dl);
    if (sweeps_out) sweeps_out[r] = sw;
    if (s != CTM_OK && s != CTM_E_NOCONV) { ctm_destroy(x); return s; }
    all_conv = all_conv && s == CTM_OK;
    s = ctm_norm(x, 0, &kap[r]);
    ctm_destroy(x);
    if (s != CTM_OK) return s;
  }
  double dv = std::fabs(kap[2]) / std::sqrt(std::fabs(kap[0] * kap[1]));
  *d_out = dv;
  if (ln_d_out) *ln_d_out = std::log(dv);
  if (!all_conv) return fail(CTM_E_NOCONV, "a CTM run of the fidelity did not converge within max_sweeps");
  return CTM_OK;
}

}  // extern "C"

// ===========================================================================
// fidelity without allocation: the workspace is a file-scope device array
// ===========================================================================
namespace {

constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;
// Host code never uses this name as an address (it is a host-side stand-in):
// the device address of each GPU's copy comes from hipGetSymbolAddress.
__device__ __align__(256) char scratch[STATIC_WS_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on the current device, looked up once per
// device with that device current
ctm_status scratch_ptr(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CTM_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> l(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CTM_E_HIP, "no device address for the static workspace");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CTM_OK;
}

}  // namespace

extern "C" {

size_t ctm_fidelity_noalloc_max_bytes(void) { return STATIC_WS_BYTES; }

ctm_status ctm_fidelity_noalloc(const ctm_config* cfg, const double* const* A_dev, const double* const* B_dev,
                                void* stream, double tol, int32_t max_sweeps, double* d_out, double* ln_d_out,
                                int32_t* sweeps_out) {
  if (!cfg || !A_dev || !B_dev || !d_out) return fail(CTM_E_INVALID, "args");
  if (cfg->complex_tensors) return fail(CTM_E_INVALID, "fidelity needs real tensors");
  // no graph instantiation and no tile timing (both create runtime objects)
  ctm_config c = *cfg;
  c.use_graph = 0;
  c.autotune = 0;
  c.concurrent_classes = 0;
  size_t need = 0;
  CHK(ctm_workspace_size(&c, &need));
  if (need > STATIC_WS_BYTES)
    return fail(CTM_E_NOMEM, "configuration needs " + std::to_string(need) +
                                 " bytes of workspace; the static workspace holds " +
                                 std::to_string(STATIC_WS_BYTES));
  void* ws = nullptr;
  CHK(scratch_ptr(&ws));
  return ctm_fidelity(&c, A_dev, B_dev, ws, STATIC_WS_BYTES, stream, tol, max_sweeps, d_out, ln_d_out,
                      sweeps_out);
}

}  // extern "C"

// ===========================================================================
// unit-test entry points (include/ctm_debug.h)
// ===========================================================================
extern "C" {

ctm_status ctm_debug_gemm(int32_t ta, int32_t tc, int64_t M, int64_t N, int64_t K, const void* A,
                          int32_t transA, const void* B, int32_t transB, void* C, void* stream) {
  if (M <= 0 || N <= 0 || K <= 0 || ta < 0 || ta > 2 || tc < 0 || tc > 2)
    return fail(CTM_E_INVALID, "sizes/types");
  hipStream_t s = (hipStream_t)stream;
  View va = transA ? transposed(rowmajor(M)) : rowmajor(K);
  View vb = transB ? transposed(rowmajor(K)) : rowmajor(N);
  GemmGroup g{};
  g.A[0] = A;
  g.B[0] = B;
  g.C[0] = C;
  hipError_t e = ctmk::gemm(s, ta, tc, M, N, K, 1.0, va, vb, 0.0, rowmajor(N), g, 1);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "unsupported type pair");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_tsgemm(int32_t ta, int32_t tc, int64_t M, int64_t N, int64_t K, const void* A,
                            int32_t transA, const void* B, void* C, void* scratch, int64_t scratch_bytes,
                            void* stream) {
  hipStream_t s = (hipStream_t)stream;
  View va = transA ? transposed(rowmajor(M)) : rowmajor(K);
  if (!ts_gemm_supported(ta, tc, M, N, K, va, rowmajor(N), rowmajor(N)) || !A || !B || !C || !scratch)
    return fail(CTM_E_INVALID, "sizes/types");
  GemmGroup g{};
  g.A[0] = A;
  g.B[0] = B;
  g.C[0] = C;
  hipError_t e = ts_gemm(s, ta, tc, M, N, K, va, rowmajor(N), rowmajor(N), g, 1, scratch, scratch_bytes);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "scratch too small");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_corner_bf16(int64_t M, int64_t N, int64_t K, const void* A, const void* Bt, void* C,
                                 void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!corner_bf16_supported(M, N, K) || !A || !Bt || !C) return fail(CTM_E_INVALID, "sizes");
  GemmGroup g{};
  g.A[0] = A;
  g.B[0] = Bt;
  g.C[0] = C;
  hipError_t e = corner_bf16(s, M, N, K, rowmajor(N), g, 1);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "alignment");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

size_t ctm_debug_corner_bf16_packed_bytes(int64_t N, int64_t K) {
  return (size_t)corner_bf16_packed_b_elems(N, K) * 2;
}

ctm_status ctm_debug_corner_bf16_packed(int64_t M, int64_t N, int64_t K, const void* A, const void* Bt, void* packed,
                                        void* C, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!corner_bf16_supported(M, N, K) || !A || !Bt || !packed || !C) return fail(CTM_E_INVALID, "sizes");
  HIPCHK(corner_bf16_pack_b(s, Bt, N, K, packed));
  GemmGroup g{};
  g.A[0] = A;
  g.B[0] = packed;
  g.C[0] = C;
  hipError_t e = corner_bf16(s, M, N, K, rowmajor(N), g, 1, F32, 0, true);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "alignment");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_tsgemm_dual(int64_t M, int64_t N, int64_t K, const float* A, int32_t transA, const float* B,
                                 float* C, double* C2, void* scratch, int64_t scratch_bytes, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  View va = transA ? transposed(rowmajor(M)) : rowmajor(K);
  if (!ts_gemm_supported(F32, F32, M, N, K, va, rowmajor(N), rowmajor(N)) || !A || !B || !C || !C2 || !scratch)
    return fail(CTM_E_INVALID, "sizes");
  GemmGroup g{}, g2{};
  g.A[0] = A;
  g.B[0] = B;
  g.C[0] = C;
  g2.C[0] = C2;
  hipError_t e = ts_gemm(s, F32, F32, M, N, K, va, rowmajor(N), rowmajor(N), g, 1, scratch, scratch_bytes, &g2);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "scratch too small");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_rmul(int64_t n, int32_t K, int32_t N, const double* A, const double* B, double* C, void* stream) {
  if (n < 1 || K < 1 || K > 64 || N < 1 || N > 64 || !A || !B || !C) return fail(CTM_E_INVALID, "args");
  hipStream_t s = (hipStream_t)stream;
  CPtrSet a{}, b{};
  PtrSet c{};
  a.p[0] = A;
  b.p[0] = B;
  c.p[0] = C;
  HIPCHK(rmul_small(s, n, K, N, a, b, c, 1));
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_gram(int64_t n, int32_t k, const double* X, const double* Y, double* G, double* part,
                          int64_t part_elems, void* stream) {
  if (n < 1 || k < 1 || k > (X ? 48 : 64) || !Y || !G || !part) return fail(CTM_E_INVALID, "args");
  hipStream_t s = (hipStream_t)stream;
  CPtrSet x{}, y{};
  PtrSet g{};
  x.p[0] = X;
  y.p[0] = Y;
  g.p[0] = G;
  hipError_t e = X ? gram_cross_small(s, n, k, x, y, g, 1, part, part_elems) : gram_small(s, n, k, y, g, 1, part, part_elems);
  if (e == hipErrorInvalidValue) return fail(CTM_E_INVALID, "scratch too small");
  HIPCHK(e);
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_chol(int32_t k, double shift_coef, const double* G, double* R, void* work, int32_t* fail_out,
                          void* stream) {
  if (k < 1 || k > CHOL_WAVE_MAX || !G || !R || !work || !fail_out) return fail(CTM_E_INVALID, "args");
  hipStream_t s = (hipStream_t)stream;
  CPtrSet g{};
  PtrSet r{};
  StatSet st{};
  g.p[0] = G;
  r.p[0] = R;
  st.p[0] = (SolveStatus*)work;
  HIPCHK(hipMemsetAsync(work, 0, sizeof(SolveStatus), s));
  HIPCHK(chol_shift_inv(s, k, shift_coef, g, r, st, 1, false));
  SolveStatus h{};
  HIPCHK(hipMemcpyAsync(&h, work, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(ssync(s));
  *fail_out = h.chol_fail;
  return CTM_OK;
}

ctm_status ctm_debug_svd(int32_t k, const double* M, double* U, double* S, double* W, double* work,
                         void* stream) {
  if (k < 1 || k > 192) return fail(CTM_E_INVALID, "k");
  hipStream_t s = (hipStream_t)stream;
  CPtrSet m{};
  PtrSet u{}, sv{}, w{}, j{};
  m.p[0] = M; u.p[0] = U; sv.p[0] = S; w.p[0] = W; j.p[0] = work;
  HIPCHK(jacobi_svd(s, k, m, u, sv, w, j, 1));
  HIPCHK(ssync(s));
  return CTM_OK;
}

ctm_status ctm_debug_dump(ctm_ctx x, int32_t what, int32_t index, void* buf, size_t bytes) {
  if (!x || !buf) return fail(CTM_E_INVALID, "args");
  RegGuard guard(&x->reg);
  Inst& I = x->inst[0];
  const int rows = std::max(x->Lx, x->Ly);
  const size_t n = I.n, chi = I.chi;
  const void* src = nullptr;
  size_t need = 0;
  if (what == 0) {
    if (index < 0 || index >= 4 * rows) return fail(CTM_E_INVALID, "index");
    src = I.rows[index / 4].Q[index % 4];
    need = n * n * dtype_size(x->qt);
  } else if (what == 1 || what == 2) {
    if (index < 0 || index >= rows) return fail(CTM_E_INVALID, "index");
    src = what == 1 ? I.rows[index].P1 : I.rows[index].P2T;
    need = n * chi * 8;
  } else if (what == 3) {
    if (index < 0 || index >= rows) return fail(CTM_E_INVALID, "index");
    src = I.rows[index].st;
    need = sizeof(SolveStatus);
  } else {
    return fail(CTM_E_INVALID, "what");
  }
  if (bytes != need) return fail(CTM_E_INVALID, "bytes must be " + std::to_string(need));
  HIPCHK(d2h(buf, src, bytes, x->stream));
  HIPCHK(ssync(x->stream));
  return CTM_OK;
}

ctm_status ctm_tile_table_load(const char* path, int32_t* entries_out) {
  if (!path) return fail(CTM_E_INVALID, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(CTM_E_INVALID, std::string("cannot open ") + path);
  static const char* names[TILE_KINDS] = {"gemm", "ts", "splitk", "corner"};
  char line[1024];
  int n = 0;
  auto num = [](const char* l, const char* key, int64_t* out) -> bool {
    const char* p = std::strstr(l, key);
    if (!p) return false;
    p = std::strchr(p + std::strlen(key), ':');
    if (!p) return false;
    char* end = nullptr;
    *out = std::strtoll(p + 1, &end, 10);
    return end != p + 1;
  };
  while (std::fgets(line, sizeof line, f)) {
    const char* kp = std::strstr(line, "\"kernel\"");
    if (!kp) continue;
    int kern = -1;
    for (int k = 0; k < TILE_KINDS; ++k) {
      std::string q = std::string("\"") + names[k] + "\"";
      const char* v = std::strstr(kp + 8, q.c_str());
      if (v) { kern = k; break; }
    }
    int64_t v[9];
    const char* keys[9] = {"\"ta\"", "\"tc\"", "\"ak\"", "\"bk\"", "\"groups\"", "\"M\"", "\"N\"", "\"K\"",
                           "\"variant\""};
    bool ok = kern >= 0;
    for (int i = 0; i < 9 && ok; ++i) ok = num(line, keys[i], &v[i]);
    if (!ok || v[8] < 0 || v[8] >= TILE_VARIANTS[kern]) {
      std::fclose(f);
      return fail(CTM_E_INVALID, std::string("malformed tile table entry: ") + line);
    }
    tile_set(TileKey{kern, (int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], v[5], v[6], v[7]}, (int)v[8]);
    ++n;
  }
  std::fclose(f);
  if (entries_out) *entries_out = n;
  return CTM_OK;
}

ctm_status ctm_tile_table_save(const char* path, int32_t* entries_out) {
  if (!path) return fail(CTM_E_INVALID, "null path");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(CTM_E_INVALID, std::string("cannot write ") + path);
  static const char* names[TILE_KINDS] = {"gemm", "ts", "splitk", "corner"};
  auto ent = tile_entries();
  std::fprintf(f, "[\n");
  for (size_t i = 0; i < ent.size(); ++i) {
    const TileKey& k = ent[i].first;
    std::fprintf(f,
                 "{\"kernel\": \"%s\", \"ta\": %d, \"tc\": %d, \"ak\": %d, \"bk\": %d, \"groups\": %d, "
                 "\"M\": %lld, \"N\": %lld, \"K\": %lld, \"variant\": %d}%s\n",
                 names[k.kernel], k.ta, k.tc, k.ak, k.bk, k.groups, (long long)k.M, (long long)k.N, (long long)k.K,
                 ent[i].second, i + 1 < ent.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
  if (entries_out) *entries_out = (int32_t)ent.size();
  return CTM_OK;
}

ctm_status ctm_tile_table_tune(int32_t on) {
  tile_tuning(on != 0);
  return CTM_OK;
}

ctm_status ctm_tile_table_clear(void) {
  tile_clear();
  return CTM_OK;
}

ctm_status ctm_debug_set_width(ctm_ctx x, int32_t width, int32_t* live_out) {
  if (!x) return fail(CTM_E_INVALID, "null ctx");
  RegGuard guard(&x->reg);
  x->width_pinned = width > 0;
  if (width > 0)
    for (auto& cls : x->classes) CHK(set_width(*x, cls, width));
  if (live_out) *live_out = x->inst[0].chi;
  return CTM_OK;
}

}  // extern "C"

// error reporting for the other C entry points of the library
ctm_status ctm_internal_fail(ctm_status s, const char* msg) { return fail(s, msg); }

ctm_status ctm_internal_edge_ring(ctm_ctx x, int inst, int column, CtmEdgeRing* out) {
  if (!x || !out || inst < 0 || inst >= x->ninst) return fail(CTM_E_INVALID, "args");
  // the boundary operators act on the ket and bra bond indices separately;
  // with complex kets the edges hold them in the real pair basis
  if (x->cfg.complex_tensors) return fail(CTM_E_INVALID, "the boundary operator needs real tensors");
  Inst& I = x->inst[inst];
  out->stream = x->stream;
  out->chi = I.chi;
  out->D = I.D;
  out->Ly = x->Ly;
  out->dry = x->reg.dry;
  const int xl = pmod(column, x->Lx), xr = pmod(column - 1, x->Lx);
  for (int y = 0; y < x->Ly; ++y) {
    out->T4[y] = I.T[3][y * x->Lx + xl];
    out->T2[y] = I.T[1][y * x->Lx + xr];
  }
  return CTM_OK;
}
