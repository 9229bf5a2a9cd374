// gfx950 kernels of the CTM library: generic MFMA GEMM with two-level
// (layout-fusing) operand views, permutation, conversion, double layer,
// reductions and the counter-based normal generator.
#include "kernels.h"

#include <hip/hip_bf16.h>
#include <algorithm>
#include <cmath>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

namespace ctmk {

thread_local Registry* g_reg = nullptr;

bool span_ok(const void* p, size_t bytes, const char* what) {
  if (!g_reg || bytes == 0) return true;
  uintptr_t a = (uintptr_t)p, b = a + bytes;
  if (b <= g_reg->lo || a >= g_reg->hi) return true;  // not workspace memory
  auto& v = g_reg->allocs;
  size_t lo = 0, hi = v.size();
  while (hi - lo > 1) {
    size_t mid = (lo + hi) / 2;
    if (v[mid].first <= a) lo = mid; else hi = mid;
  }
  if (!v.empty() && v[lo].first <= a && b <= v[lo].first + v[lo].second) return true;
  g_reg->violations++;
  g_reg->last = what;
  return false;
}

static int64_t dim_max(int64_t ext, int64_t ls, int64_t hs, int64_t R) {
  if (R <= 0) return 0;
  if (ext >= R) return (R - 1) * ls;
  int64_t q = R / ext, rem = R % ext;
  int64_t m = (q - 1) * hs + (ext - 1) * ls;
  if (rem > 0) m = std::max(m, q * hs + (rem - 1) * ls);
  return m;
}

int64_t view_max(const View& v, int64_t R, int64_t C) {
  return dim_max(v.r_ext, v.r_ls, v.r_hs, R) + dim_max(v.c_ext, v.c_ls, v.c_hs, C);
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// element access through a two-level view
// ---------------------------------------------------------------------------
struct DevView {
  int32_t r_ext, c_ext;
  int64_t r_ls, r_hs, c_ls, c_hs;
};

static DevView dev_view(const View& v, int64_t rows, int64_t cols) {
  DevView d;
  d.r_ext = (int32_t)(v.r_ext > rows ? (rows > 0 ? rows : 1) : v.r_ext);
  d.c_ext = (int32_t)(v.c_ext > cols ? (cols > 0 ? cols : 1) : v.c_ext);
  d.r_ls = v.r_ls;
  d.r_hs = v.r_hs;
  d.c_ls = v.c_ls;
  d.c_hs = v.c_hs;
  // when the extent covers the whole dimension the high part is always 0
  return d;
}

__device__ __forceinline__ int64_t row_off(const DevView& v, int32_t r) {
  int32_t h = r / v.r_ext;
  int32_t l = r - h * v.r_ext;
  return (int64_t)h * v.r_hs + (int64_t)l * v.r_ls;
}
__device__ __forceinline__ int64_t col_off(const DevView& v, int32_t c) {
  int32_t h = c / v.c_ext;
  int32_t l = c - h * v.c_ext;
  return (int64_t)h * v.c_hs + (int64_t)l * v.c_ls;
}

template <typename T> struct Acc;
template <> struct Acc<double> { typedef double type; };
template <> struct Acc<float> { typedef float type; };
template <> struct Acc<__bf16> { typedef float type; };

template <typename T> __device__ __forceinline__ T from_double(double x);
template <> __device__ __forceinline__ double from_double<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_double<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ __bf16 from_double<__bf16>(double x) { return (__bf16)(float)x; }

template <typename T> __device__ __forceinline__ double to_double(T x) { return (double)x; }
template <> __device__ __forceinline__ double to_double<__bf16>(__bf16 x) { return (double)(float)x; }

// ---------------------------------------------------------------------------
// Generic GEMM.  256 threads = 4 waves in a 2x2 grid; each wave computes a
// (BM/2) x (BN/2) block from 16x16 MFMA tiles.  Both operand tiles are staged
// in LDS with k contiguous per row (A) / per column (B).
//   f64: v_mfma_f64_16x16x4f64   lane l: A[l%16][k0 + l/16], B[k0 + l/16][l%16]
//   f32: v_mfma_f32_16x16x4f32   same operand layout
//   bf16: v_mfma_f32_16x16x32_bf16 lane l: A[l%16][8(l/16) .. +7], same for B
// result: acc[j] = C[4 (l/16) + j][l % 16] (f32, bf16) or C[l/16 + 4 j][l % 16] (f64).
// ---------------------------------------------------------------------------
template <typename TI> struct MfmaCfg;
template <> struct MfmaCfg<double> { static constexpr int KS = 4, BK = 16, PAD = 1; };
template <> struct MfmaCfg<float> { static constexpr int KS = 4, BK = 16, PAD = 1; };
template <> struct MfmaCfg<__bf16> { static constexpr int KS = 32, BK = 32, PAD = 8; };

template <typename TI, typename TO, int BM, int BN, bool A_KFAST, bool B_KFAST>
__global__ void __launch_bounds__(256)
gemm_kernel(int32_t M, int32_t N, int32_t K, double alpha, double beta,
            DevView va, DevView vb, DevView vc, GemmGroup g, int32_t ksplit) {
  typedef typename Acc<TI>::type TA;
  constexpr int BK = MfmaCfg<TI>::BK;
  constexpr int KS = MfmaCfg<TI>::KS;
  constexpr int LDK = BK + MfmaCfg<TI>::PAD;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ TI As[BM * LDK];
  __shared__ TI Bs[BN * LDK];

  // blockIdx.z = problem * ksplit + slice; with ksplit > 1 each slice sums a
  // contiguous K range into its own row-major M x N partial behind g.C[problem]
  const int gi = blockIdx.z / ksplit;
  const int sp = blockIdx.z - gi * ksplit;
  const TI* __restrict__ A = (const TI*)g.A[gi];
  const TI* __restrict__ B = (const TI*)g.B[gi];
  TO* __restrict__ C = (TO*)g.C[gi];
  int kbeg = 0, kend = K;
  if (ksplit > 1) {
    const int kc = (((K + ksplit - 1) / ksplit) + BK - 1) / BK * BK;
    kbeg = sp * kc;
    kend = min(K, kbeg + kc);
    C += (int64_t)sp * M * N;
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;

  // load slots: A tile BM x BK, B tile BN x BK (as B^T)
  constexpr int AE = (BM * BK) / 256;
  constexpr int BE = (BN * BK) / 256;
  int a_r[AE], a_k[AE];
  int64_t a_roff[AE];
  bool a_rok[AE];
#pragma unroll
  for (int j = 0; j < AE; ++j) {
    int e = tid + 256 * j;
    if (A_KFAST) { a_r[j] = e / BK; a_k[j] = e % BK; }
    else { a_r[j] = e % BM; a_k[j] = e / BM; }
    int r = m0 + a_r[j];
    a_rok[j] = r < M;
    a_roff[j] = a_rok[j] ? row_off(va, r) : 0;
  }
  int b_c[BE], b_k[BE];
  int64_t b_coff[BE];
  bool b_cok[BE];
#pragma unroll
  for (int j = 0; j < BE; ++j) {
    int e = tid + 256 * j;
    if (B_KFAST) { b_c[j] = e / BK; b_k[j] = e % BK; }
    else { b_c[j] = e % BN; b_k[j] = e / BN; }
    int c = n0 + b_c[j];
    b_cok[j] = c < N;
    b_coff[j] = b_cok[j] ? col_off(vb, c) : 0;
  }

  typedef typename std::conditional<std::is_same<TA, double>::value, v4d, v4f>::type VACC;
  VACC acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    TI ra[AE], rb[BE];
#pragma unroll
    for (int j = 0; j < AE; ++j) {
      int k = k0 + a_k[j];
      ra[j] = (a_rok[j] && k < kend) ? A[a_roff[j] + col_off(va, k)] : from_double<TI>(0.0);
    }
#pragma unroll
    for (int j = 0; j < BE; ++j) {
      int k = k0 + b_k[j];
      rb[j] = (b_cok[j] && k < kend) ? B[b_coff[j] + row_off(vb, k)] : from_double<TI>(0.0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < AE; ++j) As[a_r[j] * LDK + a_k[j]] = ra[j];
#pragma unroll
    for (int j = 0; j < BE; ++j) Bs[b_c[j] * LDK + b_k[j]] = rb[j];
    __syncthreads();

    const int lr = lane & 15;
    const int lk = lane >> 4;
    if constexpr (std::is_same<TI, __bf16>::value) {
      v8bf av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const TI* p = &As[(wm0 + i * 16 + lr) * LDK + lk * 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) av[i][q] = p[q];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const TI* p = &Bs[(wn0 + j * 16 + lr) * LDK + lk * 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) bv[j][q] = p[q];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += KS) {
        TI av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = As[(wm0 + i * 16 + lr) * LDK + ks + lk];
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = Bs[(wn0 + j * 16 + lr) * LDK + ks + lk];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (std::is_same<TI, double>::value)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
          }
      }
    }
  }

  // epilogue.  Result layout: f32/bf16 16x16 variants hold rows 4(l/16)+q,
  // the f64 variant holds rows (l/16)+4q, column l%16 in both.
  const int lc = lane & 15;
  constexpr bool F64OUT = std::is_same<TI, double>::value;
  const int rbase = F64OUT ? (lane >> 4) : (lane >> 4) * 4;
  const int rstep = F64OUT ? 4 : 1;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int c = n0 + wn0 + j * 16 + lc;
    if (c >= N) continue;
    int64_t coff = col_off(vc, c);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r = m0 + wm0 + i * 16 + rbase + rstep * q;
        if (r >= M) continue;
        int64_t off = row_off(vc, r) + coff;
        double v = alpha * (double)acc[i][j][q];
        if (beta != 0.0) v += beta * to_double<TO>(C[off]);
        C[off] = from_double<TO>(v);
      }
    }
  }
}

// Tile variants (BM x BN) of the generic GEMM; the autotuner picks one per shape.
constexpr int NTILE = 4;
constexpr int TILE_BM[NTILE] = {64, 32, 128, 128};
constexpr int TILE_BN[NTILE] = {64, 32, 64, 128};

template <typename TI, typename TO, bool AK, bool BK_, int BM, int BN>
static hipError_t launch_gemm_tile(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha,
                                   const DevView& da, const DevView& db, double beta,
                                   const DevView& dc, const GemmGroup& g, int groups) {
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)groups);
  hipLaunchKernelGGL((gemm_kernel<TI, TO, BM, BN, AK, BK_>), grid, dim3(256), 0, s,
                     (int32_t)M, (int32_t)N, (int32_t)K, alpha, beta, da, db, dc, g, 1);
  return hipGetLastError();
}

template <typename TI, typename TO, bool AK, bool BK_>
static hipError_t launch_gemm_t(hipStream_t s, int tile, int64_t M, int64_t N, int64_t K, double alpha,
                                const DevView& da, const DevView& db, double beta,
                                const DevView& dc, const GemmGroup& g, int groups) {
  switch (tile) {
    case 1: return launch_gemm_tile<TI, TO, AK, BK_, 32, 32>(s, M, N, K, alpha, da, db, beta, dc, g, groups);
    case 2: return launch_gemm_tile<TI, TO, AK, BK_, 128, 64>(s, M, N, K, alpha, da, db, beta, dc, g, groups);
    case 3: return launch_gemm_tile<TI, TO, AK, BK_, 128, 128>(s, M, N, K, alpha, da, db, beta, dc, g, groups);
    default: return launch_gemm_tile<TI, TO, AK, BK_, 64, 64>(s, M, N, K, alpha, da, db, beta, dc, g, groups);
  }
}

// ---------------------------------------------------------------------------
// split-K float64 GEMM for short-and-wide products (k x n times n x k): every
// K slice writes a partial product, then one kernel sums the slices in a
// fixed order (deterministic) and applies alpha, beta and the output view.
// ---------------------------------------------------------------------------
// Sum of the ksplit partials of every output element: 8 lanes per element,
// lane t adding partials t, t+8, ... in order, then a fixed xor tree over the
// 8 lanes (deterministic, and 8x fewer dependent loads per lane).
__global__ void splitk_reduce_kernel(const double* __restrict__ part, int ksplit, int32_t M, int32_t N,
                                     double alpha, double beta, DevView vc, GemmGroup g) {
  const int gi = blockIdx.y;
  const double* p = part + (int64_t)gi * ksplit * M * N;
  double* C = (double*)g.C[gi];
  const int t = threadIdx.x & 7;
  const int64_t MN = (int64_t)M * N;
  const int64_t per = (int64_t)gridDim.x * (blockDim.x >> 3);
  for (int64_t e0 = (int64_t)blockIdx.x * (blockDim.x >> 3); e0 < MN; e0 += per) {
    const int64_t e = e0 + (threadIdx.x >> 3);  // uniform trip count over the block: all lanes shuffle
    double acc = (e < MN && t < ksplit) ? ordered_sum(p + (int64_t)t * MN + e, (ksplit - t + 7) / 8, 8 * MN)
                                         : 0.0;
    acc += __shfl_xor(acc, 1, 8);
    acc += __shfl_xor(acc, 2, 8);
    acc += __shfl_xor(acc, 4, 8);
    if (e < MN && t == 0) {
      int r = (int)(e / N), c = (int)(e % N);
      int64_t off = row_off(vc, r) + col_off(vc, c);
      double v = alpha * acc;
      if (beta != 0.0) v += beta * C[off];
      C[off] = v;
    }
  }
}

static hipError_t gemm_splitk_v(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const View& va,
                                const View& vb, double beta, const View& vc, const GemmGroup& g, int groups,
                                double* scratch, int64_t scratch_elems, int64_t target);

hipError_t gemm_splitk(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const View& va,
                       const View& vb, double beta, const View& vc, const GemmGroup& g, int groups,
                       double* scratch, int64_t scratch_elems) {
  if (M <= 0 || N <= 0 || groups <= 0) return hipSuccess;
  // work-group target from the tile table (512 by default)
  const TileKey key{TK_SPLITK, F64, F64, va.c_ls == 1, vb.r_ls == 1, groups, M, N, K};
  int v = tile_lookup(key, -1);
  if (v < 0 && tile_tuning_on() && beta == 0.0 && !dry_run()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        float best_ms = 1e30f;
        int best = 2;
        for (int t = 0; t < TILE_VARIANTS[TK_SPLITK]; ++t) {
          float ms_min = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess ||
                gemm_splitk_v(s, M, N, K, alpha, va, vb, beta, vc, g, groups, scratch, scratch_elems,
                              (int64_t)128 << t) != hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
              break;
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms_min = std::min(ms_min, ms);
          }
          if (ms_min < best_ms) { best_ms = ms_min; best = t; }
        }
        tile_set(key, best);
        v = best;
      }
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  }
  if (v < 0 || v >= TILE_VARIANTS[TK_SPLITK]) v = 2;
  return gemm_splitk_v(s, M, N, K, alpha, va, vb, beta, vc, g, groups, scratch, scratch_elems, (int64_t)128 << v);
}

static hipError_t gemm_splitk_v(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const View& va,
                                const View& vb, double beta, const View& vc, const GemmGroup& g, int groups,
                                double* scratch, int64_t scratch_elems, int64_t target) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64) * groups;
  int64_t ksplit = std::max<int64_t>(1, std::min<int64_t>(target / std::max<int64_t>(tiles, 1), K / 64));
  while (ksplit > 1 && ksplit * M * N * groups > scratch_elems) ksplit /= 2;
  if (ksplit <= 1) return gemm(s, F64, F64, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX || groups > MAXG) return hipErrorInvalidValue;
  const size_t sa = (size_t)(view_max(va, M, K) + 1) * 8, sb = (size_t)(view_max(vb, K, N) + 1) * 8,
               sc = (size_t)(view_max(vc, M, N) + 1) * 8;
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], sa, "splitk A") || !span_ok(g.B[i], sb, "splitk B") || !span_ok(g.C[i], sc, "splitk C"))
      return hipErrorInvalidValue;
  if (!span_ok(scratch, (size_t)ksplit * M * N * groups * 8, "splitk scratch")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  GemmGroup gp = g;
  for (int i = 0; i < groups; ++i) gp.C[i] = scratch + (int64_t)i * ksplit * M * N;
  DevView da = dev_view(va, M, K), db = dev_view(vb, K, N), dc = dev_view(rowmajor(N), M, N);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)(groups * ksplit));
  bool ak = (va.c_ls == 1), bk = (vb.r_ls == 1);
  if (ak && bk)
    hipLaunchKernelGGL((gemm_kernel<double, double, 64, 64, true, true>), grid, dim3(256), 0, s, (int32_t)M,
                       (int32_t)N, (int32_t)K, 1.0, 0.0, da, db, dc, gp, (int32_t)ksplit);
  else if (ak)
    hipLaunchKernelGGL((gemm_kernel<double, double, 64, 64, true, false>), grid, dim3(256), 0, s, (int32_t)M,
                       (int32_t)N, (int32_t)K, 1.0, 0.0, da, db, dc, gp, (int32_t)ksplit);
  else if (bk)
    hipLaunchKernelGGL((gemm_kernel<double, double, 64, 64, false, true>), grid, dim3(256), 0, s, (int32_t)M,
                       (int32_t)N, (int32_t)K, 1.0, 0.0, da, db, dc, gp, (int32_t)ksplit);
  else
    hipLaunchKernelGGL((gemm_kernel<double, double, 64, 64, false, false>), grid, dim3(256), 0, s, (int32_t)M,
                       (int32_t)N, (int32_t)K, 1.0, 0.0, da, db, dc, gp, (int32_t)ksplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DevView dvc = dev_view(vc, M, N);
  // 32 elements per block of 256 (8 lanes each)
  int64_t blocks = std::min<int64_t>(2048, (M * N + 31) / 32);
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)blocks, groups), dim3(256), 0, s, scratch, (int)ksplit,
                     (int32_t)M, (int32_t)N, alpha, beta, dvc, g);
  return hipGetLastError();
}

template <typename TI, typename TO>
static hipError_t launch_gemm_ab(hipStream_t s, int tile, int64_t M, int64_t N, int64_t K, double alpha,
                                 const View& va, const View& vb, double beta, const View& vc,
                                 const GemmGroup& g, int groups) {
  DevView da = dev_view(va, M, K), db = dev_view(vb, K, N), dc = dev_view(vc, M, N);
  // A is "k fast" when its column (k) stride is 1; B is "k fast" when its row (k) stride is 1
  bool ak = (va.c_ls == 1);
  bool bk = (vb.r_ls == 1);
  if (ak && bk) return launch_gemm_t<TI, TO, true, true>(s, tile, M, N, K, alpha, da, db, beta, dc, g, groups);
  if (ak && !bk) return launch_gemm_t<TI, TO, true, false>(s, tile, M, N, K, alpha, da, db, beta, dc, g, groups);
  if (!ak && bk) return launch_gemm_t<TI, TO, false, true>(s, tile, M, N, K, alpha, da, db, beta, dc, g, groups);
  return launch_gemm_t<TI, TO, false, false>(s, tile, M, N, K, alpha, da, db, beta, dc, g, groups);
}

static hipError_t launch_typed(hipStream_t s, int tile, int ta, int tc, int64_t M, int64_t N, int64_t K,
                               double alpha, const View& va, const View& vb, double beta, const View& vc,
                               const GemmGroup& g, int groups) {
  if (ta == F64 && tc == F64) return launch_gemm_ab<double, double>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == F32 && tc == F32) return launch_gemm_ab<float, float>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == F32 && tc == F64) return launch_gemm_ab<float, double>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == BF16 && tc == F32) return launch_gemm_ab<__bf16, float>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == BF16 && tc == F64) return launch_gemm_ab<__bf16, double>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == BF16 && tc == BF16) return launch_gemm_ab<__bf16, __bf16>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  if (ta == F32 && tc == BF16) return launch_gemm_ab<float, __bf16>(s, tile, M, N, K, alpha, va, vb, beta, vc, g, groups);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// autotuner: process-wide cache of the fastest tile per GEMM shape
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int dev, ta, tc, ak, bk, groups;
  int64_t M, N, K;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, ta, tc, ak, bk, groups, M, N, K) <
           std::tie(o.dev, o.ta, o.tc, o.ak, o.bk, o.groups, o.M, o.N, o.K);
  }
};
std::map<TuneKey, int> g_tune;
std::mutex g_tune_mu;
thread_local bool g_tune_on = false;
}  // namespace

void set_tuning(bool on) { g_tune_on = on; }

namespace {
std::map<TileKey, int> g_tiles;
std::mutex g_tiles_mu;
std::atomic<bool> g_tile_tuning{false};
}  // namespace

bool TileKey::operator<(const TileKey& o) const {
  return std::tie(kernel, ta, tc, ak, bk, groups, M, N, K) <
         std::tie(o.kernel, o.ta, o.tc, o.ak, o.bk, o.groups, o.M, o.N, o.K);
}
int tile_lookup(const TileKey& k, int dflt) {
  std::lock_guard<std::mutex> l(g_tiles_mu);
  auto it = g_tiles.find(k);
  return it == g_tiles.end() ? dflt : it->second;
}
void tile_set(const TileKey& k, int variant) {
  std::lock_guard<std::mutex> l(g_tiles_mu);
  g_tiles[k] = variant;
}
void tile_clear() {
  std::lock_guard<std::mutex> l(g_tiles_mu);
  g_tiles.clear();
}
std::vector<std::pair<TileKey, int>> tile_entries() {
  std::lock_guard<std::mutex> l(g_tiles_mu);
  return std::vector<std::pair<TileKey, int>>(g_tiles.begin(), g_tiles.end());
}
void tile_tuning(bool on) { g_tile_tuning = on; }
bool tile_tuning_on() { return g_tile_tuning; }
int tuned_entries() {
  std::lock_guard<std::mutex> l(g_tune_mu);
  return (int)g_tune.size();
}

static int pick_tile(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, double alpha,
                     const View& va, const View& vb, double beta, const View& vc, const GemmGroup& g,
                     int groups) {
  // one choice per shape, whatever the number of problems in the launch
  TuneKey key{0, ta, tc, va.c_ls == 1, vb.r_ls == 1, 0, M, N, K};
  (void)hipGetDevice(&key.dev);
  const TileKey tk{TK_GEMM, ta, tc, va.c_ls == 1, vb.r_ls == 1, 0, M, N, K};
  {
    const int v = tile_lookup(tk, -1);
    if (v >= 0 && v < NTILE) return v;
  }
  {
    std::lock_guard<std::mutex> l(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  if (!g_tune_on || beta != 0.0) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return 0;
  }
  int best = 0;
  float best_ms = 1e30f;
  for (int t = 0; t < NTILE; ++t) {
    float ms_min = 1e30f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {
      ok = hipEventRecord(e0, s) == hipSuccess &&
           launch_typed(s, t, ta, tc, M, N, K, alpha, va, vb, beta, vc, g, groups) == hipSuccess &&
           hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0;
      if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms_min = std::min(ms_min, ms);
    }
    if (ok && ms_min < best_ms) { best_ms = ms_min; best = t; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tile_set(tk, best);
  std::lock_guard<std::mutex> l(g_tune_mu);
  g_tune[key] = best;
  return best;
}

hipError_t gemm(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, double alpha,
                const View& va, const View& vb, double beta, const View& vc,
                const GemmGroup& g, int groups) {
  if (M <= 0 || N <= 0 || groups <= 0) return hipSuccess;
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX || groups > MAXG) return hipErrorInvalidValue;
  {
    const size_t ea = dtype_size(ta), ec = dtype_size(tc);
    const size_t sa = (size_t)(view_max(va, M, K) + 1) * ea, sb = (size_t)(view_max(vb, K, N) + 1) * ea,
                 sc = (size_t)(view_max(vc, M, N) + 1) * ec;
    for (int i = 0; i < groups; ++i)
      if (!span_ok(g.A[i], K > 0 ? sa : 0, "gemm A") || !span_ok(g.B[i], K > 0 ? sb : 0, "gemm B") ||
          !span_ok(g.C[i], sc, "gemm C"))
        return hipErrorInvalidValue;
    if (dry_run()) return hipSuccess;
  }
  const int tile = pick_tile(s, ta, tc, M, N, K, alpha, va, vb, beta, vc, g, groups);
  return launch_typed(s, tile, ta, tc, M, N, K, alpha, va, vb, beta, vc, g, groups);
}

// ---------------------------------------------------------------------------
// permutation with conversion
// ---------------------------------------------------------------------------
struct PermArgs {
  int ndim;
  int64_t out_dims[8];
  int64_t in_stride_of_out[8];
};

template <typename TI, typename TO>
__global__ void permute_kernel(const TI* __restrict__ in, TO* __restrict__ out, int64_t n, PermArgs p) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, off = 0;
    for (int i = p.ndim - 1; i >= 0; --i) {
      int64_t q = rem / p.out_dims[i];
      int64_t idx = rem - q * p.out_dims[i];
      rem = q;
      off += idx * p.in_stride_of_out[i];
    }
    out[e] = from_double<TO>(to_double<TI>(in[off]));
  }
}

// The same when the innermost output index is also the innermost input
// index (stride 1): each thread copies four consecutive elements of a row of
// L, with the row's offset decoded once (ndim - 1 outer indices).
template <typename TI, typename TO>
__global__ void permute_run_kernel(const TI* __restrict__ in, TO* __restrict__ out, int64_t rows, PermArgs p) {
  const int nd = p.ndim - 1;
  const int64_t L = p.out_dims[nd], nq = (L + 3) / 4;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * nq;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / nq, j0 = (t - row * nq) * 4;
    int64_t rem = row, off = 0;
    for (int i = nd - 1; i >= 0; --i) {
      const int64_t q = rem / p.out_dims[i];
      off += (rem - q * p.out_dims[i]) * p.in_stride_of_out[i];
      rem = q;
    }
    const TI* src = in + off + j0;
    TO* dst = out + row * L + j0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j0 + j < L) dst[j] = from_double<TO>(to_double<TI>(src[j]));
  }
}

template <typename TI, typename TO>
static hipError_t launch_perm(hipStream_t s, const void* in, void* out, int64_t n, const PermArgs& p) {
  if (n == 0) return hipSuccess;
  const int64_t L = p.out_dims[p.ndim - 1];
  if (p.ndim >= 2 && p.in_stride_of_out[p.ndim - 1] == 1 && L >= 4) {
    const int64_t rows = n / L, work = rows * ((L + 3) / 4);
    const int64_t blocks = std::min<int64_t>(65536, (work + 255) / 256);
    hipLaunchKernelGGL((permute_run_kernel<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, s, (const TI*)in,
                       (TO*)out, rows, p);
    return hipGetLastError();
  }
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((permute_kernel<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const TI*)in, (TO*)out, n, p);
  return hipGetLastError();
}

template <typename TI>
static hipError_t perm_to(hipStream_t s, const void* in, int tout, void* out, int64_t n, const PermArgs& p) {
  if (tout == F64) return launch_perm<TI, double>(s, in, out, n, p);
  if (tout == F32) return launch_perm<TI, float>(s, in, out, n, p);
  if (tout == BF16) return launch_perm<TI, __bf16>(s, in, out, n, p);
  return hipErrorInvalidValue;
}

hipError_t permute(hipStream_t s, int tin, const void* in, int tout, void* out, int ndim,
                   const int64_t* in_dims, const int* perm) {
  if (ndim < 1 || ndim > 8) return hipErrorInvalidValue;
  PermArgs p;
  p.ndim = ndim;
  int64_t stride[8];
  int64_t acc = 1;
  for (int i = ndim - 1; i >= 0; --i) { stride[i] = acc; acc *= in_dims[i]; }
  for (int i = 0; i < ndim; ++i) {
    p.out_dims[i] = in_dims[perm[i]];
    p.in_stride_of_out[i] = stride[perm[i]];
  }
  int64_t n = acc;
  if (!span_ok(in, n * dtype_size(tin), "permute in") || !span_ok(out, n * dtype_size(tout), "permute out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (tin == F64) return perm_to<double>(s, in, tout, out, n, p);
  if (tin == F32) return perm_to<float>(s, in, tout, out, n, p);
  if (tin == BF16) return perm_to<__bf16>(s, in, tout, out, n, p);
  return hipErrorInvalidValue;
}

hipError_t convert(hipStream_t s, int tin, const void* in, int tout, void* out, int64_t n) {
  int64_t dims[1] = {n};
  int perm[1] = {0};
  return permute(s, tin, in, tout, out, 1, dims, perm);
}

// ---------------------------------------------------------------------------
// double layer: for rotation k, out_k[L'][U'][D'][R'] = rot_k(a)[U',L',D',R'],
// a[U,L,Dn,R] = sum_s A[s,u,l,d,r] B[s,u',l',d',r'], U = u*D + u'.
// Rotation k = 0..3 counter-clockwise quarter turns:
//   k=1: U=L', L=D', Dn=R', R=U';  k=2: U=D', L=R', Dn=U', R=L';
//   k=3: U=R', L=U', Dn=L', R=D'.
// out_layout != 0 additionally writes the plain a[U][L][Dn][R] to out_rot[...]
// (handled by the caller through rotation 0 with a transpose).
// ---------------------------------------------------------------------------
__global__ void double_layer_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                    int d, int D, double* o0, double* o1, double* o2, double* o3) {
  const int D2 = D * D;
  const int64_t n = (int64_t)D2 * D2 * D2 * D2;
  const int k = blockIdx.y;
  double* out = k == 0 ? o0 : (k == 1 ? o1 : (k == 2 ? o2 : o3));
  // strides of A[s][u][l][d][r] (d x D x D x D x D, row-major)
  const int64_t sR = 1, sDn = D, sL = (int64_t)D * D, sU = (int64_t)D * D * D,
                sS = (int64_t)D * D * D * D;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e;
    int Rp = rem % D2; rem /= D2;
    int Dp = rem % D2; rem /= D2;
    int Up = rem % D2; rem /= D2;
    int Lp = (int)rem;
    int U, L, Dn, R;
    if (k == 0) { U = Up; L = Lp; Dn = Dp; R = Rp; }
    else if (k == 1) { U = Lp; L = Dp; Dn = Rp; R = Up; }
    else if (k == 2) { U = Dp; L = Rp; Dn = Up; R = Lp; }
    else { U = Rp; L = Up; Dn = Lp; R = Dp; }
    int u = U / D, uu = U % D, l = L / D, ll = L % D, dd = Dn / D, ddd = Dn % D, r = R / D, rr = R % D;
    int64_t oa = u * sU + l * sL + dd * sDn + r * sR;
    int64_t ob = uu * sU + ll * sL + ddd * sDn + rr * sR;
    double acc = 0.0;
    for (int s = 0; s < d; ++s) acc += A[s * sS + oa] * B[s * sS + ob];
    out[e] = acc;
  }
}

hipError_t double_layer(hipStream_t s, const double* A, const double* B, int d, int D,
                        double* out_rot[4], int64_t) {
  int64_t n = (int64_t)D * D * D * D * D * D * D * D;
  const size_t t5 = (size_t)d * D * D * D * D * 8;
  if (!span_ok(A, t5, "double layer A") || !span_ok(B, t5, "double layer B")) return hipErrorInvalidValue;
  for (int r = 0; r < 4; ++r)
    if (!span_ok(out_rot[r], n * 8, "double layer out")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(double_layer_kernel, dim3((unsigned)blocks, 4), dim3(256), 0, s, A, B, d, D,
                     out_rot[0], out_rot[1], out_rot[2], out_rot[3]);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Real form of the double layer of a complex ket (bra = its conjugate).
// a = sum_s A_s (x) conj(A_s) satisfies conj(a) = S a S, S swapping ket and
// bra on every leg.  On each doubled leg (x, x') the unitary basis change V
//   slot (x, x)            <- e_(x,x)
//   slot (x, x'), x < x'   <- (e_(x,x') + e_(x',x)) / sqrt 2
//   slot (x', x), x < x'   <- i (e_(x,x') - e_(x',x)) / sqrt 2
// (V-bar: the conjugate coefficients) maps such tensors to real ones.  The
// right and down legs take V, the left and up legs V-bar: a bond pairs a V
// leg with a V-bar leg and V^T V-bar = 1, so every contraction of the network
// keeps its value and the whole CTM runs on real tensors.
//   sigma < 0: out = real part of (V-bar_u V-bar_l V_d V_r) a (the imaginary
//              part vanishes up to rounding);
//   sigma >= 0: the open double layer of physical slot sigma for the density
//              matrices: sum over the physical pairs (s, s') of slot sigma
//              (basis V on the physical pair) of A_s (x) conj(A_s'), legs
//              transformed as above (real as well).
// Ac is [d][D][D][D][D] complex (real, imaginary interleaved).  Rotations as
// in double_layer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double A_cr(const double* Ac, int64_t i) { return Ac[2 * i]; }
__device__ __forceinline__ double A_ci(const double* Ac, int64_t i) { return Ac[2 * i + 1]; }

struct PairTerms {
  int n;
  int k[2], b[2];      // ket and bra index of each term
  double cr[2], ci[2];  // complex coefficient
};

__device__ __forceinline__ PairTerms pair_terms(int slot, int D, bool conj_basis) {
  const double h = 0.70710678118654752440;
  const int p = slot / D, q = slot - p * D;
  PairTerms t;
  if (p == q) {
    t.n = 1; t.k[0] = p; t.b[0] = p; t.cr[0] = 1.0; t.ci[0] = 0.0;
  } else if (p < q) {
    t.n = 2;
    t.k[0] = p; t.b[0] = q; t.cr[0] = h; t.ci[0] = 0.0;
    t.k[1] = q; t.b[1] = p; t.cr[1] = h; t.ci[1] = 0.0;
  } else {
    // lower slot of the pair (q, p), q < p: i (e_(q,p) - e_(p,q)) / sqrt 2
    const double sg = conj_basis ? -1.0 : 1.0;
    t.n = 2;
    t.k[0] = q; t.b[0] = p; t.cr[0] = 0.0; t.ci[0] = sg * h;
    t.k[1] = p; t.b[1] = q; t.cr[1] = 0.0; t.ci[1] = -sg * h;
  }
  return t;
}

__global__ void double_layer_cplx_kernel(const double* __restrict__ Ac, int d, int D, int sigma, double* o0,
                                         double* o1, double* o2, double* o3) {
  const int D2 = D * D;
  const int64_t n = (int64_t)D2 * D2 * D2 * D2;
  const int k = blockIdx.y;
  double* out = k == 0 ? o0 : (k == 1 ? o1 : (k == 2 ? o2 : o3));
  const int64_t sR = 1, sDn = D, sL = (int64_t)D * D, sU = (int64_t)D * D * D, sS = (int64_t)D * D * D * D;
  PairTerms ph;
  if (sigma >= 0) ph = pair_terms(sigma, d, false);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e;
    const int Rp = rem % D2; rem /= D2;
    const int Dp = rem % D2; rem /= D2;
    const int Up = rem % D2; rem /= D2;
    const int Lp = (int)rem;
    int U, L, Dn, R;
    if (k == 0) { U = Up; L = Lp; Dn = Dp; R = Rp; }
    else if (k == 1) { U = Lp; L = Dp; Dn = Rp; R = Up; }
    else if (k == 2) { U = Dp; L = Rp; Dn = Up; R = Lp; }
    else { U = Rp; L = Up; Dn = Lp; R = Dp; }
    const PairTerms tu = pair_terms(U, D, true), tl = pair_terms(L, D, true);
    const PairTerms td = pair_terms(Dn, D, false), tr = pair_terms(R, D, false);
    double ar = 0.0, ai = 0.0;
    for (int a0 = 0; a0 < tu.n; ++a0)
      for (int a1 = 0; a1 < tl.n; ++a1)
        for (int a2 = 0; a2 < td.n; ++a2)
          for (int a3 = 0; a3 < tr.n; ++a3) {
            // coefficient product
            double cr = tu.cr[a0], ci = tu.ci[a0], xr, xi;
            xr = cr * tl.cr[a1] - ci * tl.ci[a1]; xi = cr * tl.ci[a1] + ci * tl.cr[a1]; cr = xr; ci = xi;
            xr = cr * td.cr[a2] - ci * td.ci[a2]; xi = cr * td.ci[a2] + ci * td.cr[a2]; cr = xr; ci = xi;
            xr = cr * tr.cr[a3] - ci * tr.ci[a3]; xi = cr * tr.ci[a3] + ci * tr.cr[a3]; cr = xr; ci = xi;
            const int64_t oa = tu.k[a0] * sU + tl.k[a1] * sL + td.k[a2] * sDn + tr.k[a3] * sR;
            const int64_t ob = tu.b[a0] * sU + tl.b[a1] * sL + td.b[a2] * sDn + tr.b[a3] * sR;
            // v = sum over physical pairs of A_s[oa] conj(A_s'[ob])
            double vr = 0.0, vi = 0.0;
            const int np = sigma >= 0 ? ph.n : d;
            for (int j = 0; j < np; ++j) {
              const int s1 = sigma >= 0 ? ph.k[j] : j, s2 = sigma >= 0 ? ph.b[j] : j;
              const double pr = A_cr(Ac, s1 * sS + oa), pi = A_ci(Ac, s1 * sS + oa);
              const double qr = A_cr(Ac, s2 * sS + ob), qi = -A_ci(Ac, s2 * sS + ob);
              double tr_ = pr * qr - pi * qi, ti_ = pr * qi + pi * qr;
              if (sigma >= 0) {
                const double wr = ph.cr[j], wi = ph.ci[j];
                const double yr = wr * tr_ - wi * ti_, yi = wr * ti_ + wi * tr_;
                tr_ = yr; ti_ = yi;
              }
              vr += tr_; vi += ti_;
            }
            ar += cr * vr - ci * vi;
            ai += cr * vi + ci * vr;
          }
    (void)ai;
    out[e] = ar;
  }
}

hipError_t double_layer_cplx(hipStream_t s, const double* Ac, int d, int D, int sigma, double* out_rot[4]) {
  const int64_t n = (int64_t)D * D * D * D * D * D * D * D;
  const size_t t5 = (size_t)d * D * D * D * D * 16;
  if (sigma >= d * d) return hipErrorInvalidValue;
  if (!span_ok(Ac, t5, "complex double layer A")) return hipErrorInvalidValue;
  for (int r = 0; r < 4; ++r)
    if (!span_ok(out_rot[r], n * 8, "complex double layer out")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(double_layer_cplx_kernel, dim3((unsigned)blocks, 4), dim3(256), 0, s, Ac, d, D, sigma,
                     out_rot[0], out_rot[1], out_rot[2], out_rot[3]);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void sumsq_partial(const double* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) acc += x[e] * x[e];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sum_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

static const int kPartials = 256;

hipError_t sumsq(hipStream_t s, const double* x, int64_t n, double* partial, double* out) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > kPartials) blocks = kPartials;
  if (blocks < 1) blocks = 1;
  if (!span_ok(x, n * 8, "sumsq x") || !span_ok(partial, blocks * 8, "sumsq partial") || !span_ok(out, 8, "sumsq out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(sumsq_partial, dim3((unsigned)blocks), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, s, partial, (int)blocks, out);
  return hipGetLastError();
}

__global__ void scale_rsqrt_kernel(double* __restrict__ x, int64_t n, const double* __restrict__ nrm2) {
  double v = *nrm2;
  if (!(v > 0.0)) return;
  double f = 1.0 / sqrt(v);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) x[e] *= f;
}

hipError_t scale_by_rsqrt(hipStream_t s, double* x, int64_t n, const double* nrm2) {
  if (!span_ok(x, n * 8, "scale x") || !span_ok(nrm2, 8, "scale nrm2")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scale_rsqrt_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, nrm2);
  return hipGetLastError();
}

__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) bad |= !isfinite(x[e]);
  if (bad) *flag = 1;  // benign race: every writer stores the same value
}

hipError_t nonfinite(hipStream_t s, const double* x, int64_t n, int* flag) {
  if (!span_ok(x, n * 8, "nonfinite x") || !span_ok(flag, 4, "nonfinite flag")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// counter-based normals: u = splitmix64(seed + 2i), splitmix64(seed + 2i + 1)
// mapped to (0,1], Box-Muller.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void randn_kernel(double* __restrict__ out, int64_t n, uint64_t seed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t a = splitmix64(seed + 2ull * (uint64_t)e);
    uint64_t b = splitmix64(seed + 2ull * (uint64_t)e + 1ull);
    double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    out[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

hipError_t randn(hipStream_t s, double* out, int64_t n, uint64_t seed) {
  if (!span_ok(out, n * 8, "randn out")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(randn_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, n, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grouped copy / conversion and grouped Frobenius normalisation
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void convert_group_kernel(XferSet x) {
  const int j = blockIdx.y;
  const TI* __restrict__ in = (const TI*)x.src[j];
  TO* __restrict__ out = (TO*)x.dst[j];
  const int64_t n = x.n[j];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = from_double<TO>(to_double<TI>(in[e]));
}

template <typename TI>
static hipError_t conv_to(hipStream_t s, int tout, dim3 grid, const XferSet& x) {
  if (tout == F64) hipLaunchKernelGGL((convert_group_kernel<TI, double>), grid, dim3(256), 0, s, x);
  else if (tout == F32) hipLaunchKernelGGL((convert_group_kernel<TI, float>), grid, dim3(256), 0, s, x);
  else if (tout == BF16) hipLaunchKernelGGL((convert_group_kernel<TI, __bf16>), grid, dim3(256), 0, s, x);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t convert_group(hipStream_t s, int tin, int tout, const XferSet& x, int njobs) {
  if (njobs <= 0) return hipSuccess;
  if (njobs > MAXJ) return hipErrorInvalidValue;
  int64_t nmax = 0;
  for (int j = 0; j < njobs; ++j) {
    if (x.n[j] < 0) return hipErrorInvalidValue;
    if (!span_ok(x.src[j], x.n[j] * dtype_size(tin), "convert_group src") ||
        !span_ok(x.dst[j], x.n[j] * dtype_size(tout), "convert_group dst"))
      return hipErrorInvalidValue;
    nmax = std::max(nmax, x.n[j]);
  }
  if (dry_run() || nmax == 0) return hipSuccess;
  int64_t blocks = std::min<int64_t>(2048, std::max<int64_t>(1, (nmax + 255) / 256));
  dim3 grid((unsigned)blocks, (unsigned)njobs);
  if (tin == F64) return conv_to<double>(s, tout, grid, x);
  if (tin == F32) return conv_to<float>(s, tout, grid, x);
  if (tin == BF16) return conv_to<__bf16>(s, tout, grid, x);
  return hipErrorInvalidValue;
}

constexpr int kNormParts = 64;

__global__ void norm_partial_kernel(NormSet x, double* __restrict__ part) {
  __shared__ double red[4];
  const int j = blockIdx.y;
  const double* __restrict__ p = x.p[j];
  const int64_t n = x.n[j];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) acc += p[e] * p[e];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[j * kNormParts + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void norm_scale_kernel(NormSet x, const double* __restrict__ part) {
  __shared__ double f;
  const int j = blockIdx.y;
  if (threadIdx.x < 64) {
    double v = part[j * kNormParts + threadIdx.x];  // kNormParts == one wave
    v = wave_sum(v);
    if (threadIdx.x == 0) f = v > 0.0 ? 1.0 / sqrt(v) : 1.0;
  }
  __syncthreads();
  double* __restrict__ p = x.p[j];
  const int64_t n = x.n[j];
  const double g = f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) p[e] *= g;
}

hipError_t normalize_group(hipStream_t s, const NormSet& x, int njobs, double* partial) {
  if (njobs <= 0) return hipSuccess;
  if (njobs > MAXJ) return hipErrorInvalidValue;
  int64_t nmax = 0;
  for (int j = 0; j < njobs; ++j) {
    if (x.n[j] < 0 || !span_ok(x.p[j], x.n[j] * 8, "normalize_group")) return hipErrorInvalidValue;
    nmax = std::max(nmax, x.n[j]);
  }
  if (!span_ok(partial, (size_t)njobs * kNormParts * 8, "normalize_group partial")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  // every one of the kNormParts partial slots is written (zero for idle blocks)
  hipLaunchKernelGGL(norm_partial_kernel, dim3(kNormParts, njobs), dim3(256), 0, s, x, partial);
  int64_t blocks = std::min<int64_t>(2048, std::max<int64_t>(1, (nmax + 255) / 256));
  hipLaunchKernelGGL(norm_scale_kernel, dim3((unsigned)blocks, njobs), dim3(256), 0, s, x, partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// three-term bf16 split (see kernels.h)
// ---------------------------------------------------------------------------
// one element: o[0], o[K], o[2K] of its output row
__device__ __forceinline__ void split3_store(double x, int a_side, __bf16* o, int64_t K) {
  const __bf16 hi = (__bf16)(float)x;
  const __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
  o[0] = hi;
  o[K] = a_side ? hi : lo;
  o[2 * K] = a_side ? lo : hi;
}

template <typename TI>
__global__ void split3_kernel(const TI* __restrict__ in, DevView v, int64_t rows, int64_t K, int a_side,
                              __bf16* __restrict__ out) {
  const int64_t n = rows * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / K, k = e - r * K;
    split3_store((double)in[row_off(v, (int32_t)r) + col_off(v, (int32_t)k)], a_side, out + r * 3 * K + k, K);
  }
}

// several float64 splits of one shape, job = blockIdx.y
constexpr int MAXJ3 = 8;
struct Split3Set {
  const double* in[MAXJ3];
  __bf16* out[MAXJ3];
  DevView v[MAXJ3];
  int a_side[MAXJ3];
};

__global__ void split3_group_kernel(Split3Set j, int64_t rows, int64_t K) {
  const int q = blockIdx.y;
  const double* __restrict__ in = j.in[q];
  __bf16* __restrict__ out = j.out[q];
  const DevView v = j.v[q];
  const int a_side = j.a_side[q];
  const int64_t n = rows * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / K, k = e - r * K;
    split3_store(in[row_off(v, (int32_t)r) + col_off(v, (int32_t)k)], a_side, out + r * 3 * K + k, K);
  }
}

hipError_t split3_bf16_group(hipStream_t s, const Split3Job* jobs, int njobs, int64_t rows, int64_t K) {
  if (njobs < 0 || rows <= 0 || K <= 0 || rows > INT32_MAX || K > INT32_MAX) return hipErrorInvalidValue;
  for (int i = 0; i < njobs; ++i)
    if (!span_ok(jobs[i].in, (size_t)(view_max(jobs[i].view, rows, K) + 1) * 8, "split3 in") ||
        !span_ok(jobs[i].out, (size_t)rows * 3 * K * 2, "split3 out"))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(8192, (rows * K + 255) / 256);
  for (int j0 = 0; j0 < njobs; j0 += MAXJ3) {
    const int cnt = std::min(MAXJ3, njobs - j0);
    Split3Set set{};
    for (int i = 0; i < cnt; ++i) {
      const Split3Job& jb = jobs[j0 + i];
      set.in[i] = (const double*)jb.in;
      set.out[i] = (__bf16*)jb.out;
      set.v[i] = dev_view(jb.view, rows, K);
      set.a_side[i] = jb.a_side ? 1 : 0;
    }
    hipLaunchKernelGGL(split3_group_kernel, dim3((unsigned)blocks, (unsigned)cnt), dim3(256), 0, s, set, rows, K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t split3_bf16(hipStream_t s, int tin, const void* in, const View& vin, int64_t rows, int64_t K, bool a_side,
                       void* out) {
  if (rows <= 0 || K <= 0 || rows > INT32_MAX || K > INT32_MAX || (tin != F32 && tin != F64))
    return hipErrorInvalidValue;
  if (!span_ok(in, (size_t)(view_max(vin, rows, K) + 1) * dtype_size(tin), "split3 in") ||
      !span_ok(out, (size_t)rows * 3 * K * 2, "split3 out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const DevView dv = dev_view(vin, rows, K);
  const int64_t blocks = std::min<int64_t>(8192, (rows * K + 255) / 256);
  if (tin == F32)
    hipLaunchKernelGGL((split3_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s, (const float*)in, dv, rows, K,
                       a_side ? 1 : 0, (__bf16*)out);
  else
    hipLaunchKernelGGL((split3_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, s, (const double*)in, dv, rows,
                       K, a_side ? 1 : 0, (__bf16*)out);
  return hipGetLastError();
}

// 32 x 32 tiles through LDS: coalesced reads along c, coalesced writes along r
__global__ void split3_transpose_kernel(const float* __restrict__ in, int64_t R, int64_t C, int a_side,
                                        __bf16* __restrict__ out) {
  __shared__ float t[32][33];
  const int64_t b = blockIdx.z;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows of 32
  const float* src = in + b * R * C;
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    t[i][tx] = (r < R && c < C) ? src[r * C + c] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < C && r < R) {
      const float x = t[tx][i];
      const __bf16 hi = (__bf16)x;
      const __bf16 lo = (__bf16)(x - (float)hi);
      __bf16* o = out + (b * C + c) * 3 * R + r;
      o[0] = hi;
      o[R] = a_side ? hi : lo;
      o[2 * R] = a_side ? lo : hi;
    }
  }
}

hipError_t split3_transpose_bf16(hipStream_t s, const float* in, int64_t nb, int64_t R, int64_t C, bool a_side,
                                 void* out) {
  if (nb <= 0 || R <= 0 || C <= 0 || nb > 65535) return hipErrorInvalidValue;
  if (!span_ok(in, (size_t)nb * R * C * 4, "split3t in") || !span_ok(out, (size_t)nb * C * 3 * R * 2, "split3t out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32), (unsigned)nb);
  hipLaunchKernelGGL(split3_transpose_kernel, grid, dim3(256), 0, s, in, R, C, a_side ? 1 : 0, (__bf16*)out);
  return hipGetLastError();
}

// batched transpose out[b][c][r] = in[b][r][c] (float), 32 x 32 LDS tiles
__global__ void transpose_batched_kernel(const float* __restrict__ in, int64_t R, int64_t C, float* __restrict__ out) {
  __shared__ float t[32][33];
  const int64_t b = blockIdx.z;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const float* src = in + b * R * C;
  float* dst = out + b * R * C;
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < R && c < C) t[i][tx] = src[r * C + c];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < C && r < R) dst[c * R + r] = t[tx][i];
  }
}

hipError_t transpose_batched(hipStream_t s, const float* in, int64_t nb, int64_t R, int64_t C, float* out) {
  if (nb <= 0 || R <= 0 || C <= 0 || nb > 65535) return hipErrorInvalidValue;
  if (!span_ok(in, (size_t)nb * R * C * 4, "transpose in") || !span_ok(out, (size_t)nb * R * C * 4, "transpose out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32), (unsigned)nb);
  hipLaunchKernelGGL(transpose_batched_kernel, grid, dim3(256), 0, s, in, R, C, out);
  return hipGetLastError();
}

}  // namespace ctmk
