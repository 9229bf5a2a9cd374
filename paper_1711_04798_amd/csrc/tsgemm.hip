// Tall-skinny GEMM split over K, for products C (M x N) = op(A) (M x K) B (K x N)
// with few columns (N <= 192) and a long contraction: the half-system
// applications of the projector solver (n x n enlarged corner times an
// n x k block) and the n-long contractions of the absorption.  The plain
// tiled kernel gives these shapes too few work-groups and re-reads the block
// B per row tile; here each work-group takes 64 rows of A and one K chunk,
// holds all N columns, and writes a partial product; a second kernel sums the
// K chunks in a fixed order (deterministic) into C.
//   f32: v_mfma_f32_16x16x4f32, f64: v_mfma_f64_16x16x4f64; lane l feeds
//   A[l%16][k0 + l/16] and B[k0 + l/16][l%16].
#include "kernels.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace ctmk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct TsCfg;
template <> struct TsCfg<float> { static constexpr int BK = 32; typedef v4f V; };
template <> struct TsCfg<double> { static constexpr int BK = 16; typedef v4d V; };

constexpr int BM = 64;        // rows per work-group (16 per wave)
constexpr int NMAX = 192;     // columns held by one work-group

template <typename T>
__device__ __forceinline__ typename TsCfg<T>::V mfma(T a, T b, typename TsCfg<T>::V c);
template <>
__device__ __forceinline__ v4f mfma<float>(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4d mfma<double>(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A element (m, k) at m * lda + k (A_KFAST) or k * lda + m; B (k, n) at k * ldb + n.
// part[(gi * nsplit + s)][m][n], row-major M x N.
// VEC (float only): A is read in 16-byte chunks along its contiguous index
// (needs lda, K and M multiples of 4 and a 16-byte aligned base)
template <typename T, bool A_KFAST, int NT, bool VEC>
__global__ void __launch_bounds__(256, 2)
ts_partial_kernel(int32_t M, int32_t N, int32_t K, int64_t lda, int64_t ldb, int32_t kchunk, int32_t nsplit,
                  int32_t mtiles, GemmGroup g, T* __restrict__ part) {
  constexpr int BK = TsCfg<T>::BK, LDK = BK + 1, NP = NT * 16;
  __shared__ T As[2][BM * LDK];
  __shared__ T Bs[2][NP * LDK];
  // launch order: row tile fastest, then K chunk, then problem
  const int bid = blockIdx.x;
  const int mt = bid % mtiles;
  const int sk = (bid / mtiles) % nsplit;
  const int gi = bid / (mtiles * nsplit);
  const T* __restrict__ A = (const T*)g.A[gi];
  const T* __restrict__ B = (const T*)g.B[gi];
  const int m0 = mt * BM;
  const int kbeg = sk * kchunk, kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  constexpr int AE = BM * BK / 256;                 // A elements per thread
  constexpr int BE = (NP * BK + 255) / 256;         // B elements per thread
  T ra[AE], rb[BE];
  // vector form: chunk e of 4 consecutive elements along the contiguous index
  //   k-fast: row e / (BK / 4), k 4 (e % (BK / 4)); m-fast: k e / (BM / 4), m 4 (e % (BM / 4))
  auto chunk_rk = [&](int e, int& r, int& kk) {
    if (A_KFAST) { r = e / (BK / 4); kk = (e % (BK / 4)) * 4; }
    else { kk = e / (BM / 4); r = (e % (BM / 4)) * 4; }
  };
  auto gload = [&](int k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < AE / 4; ++j) {
        int r, kk;
        chunk_rk(tid + 256 * j, r, kk);
        const int m = m0 + r, k = k0 + kk;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (A_KFAST ? (m < M && k < kend) : (m < M && k < kend))
          v = *reinterpret_cast<const float4*>(A_KFAST ? A + (int64_t)m * lda + k : A + (int64_t)k * lda + m);
        ra[4 * j] = v.x; ra[4 * j + 1] = v.y; ra[4 * j + 2] = v.z; ra[4 * j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < AE; ++j) {
        const int e = tid + 256 * j;
        const int r = A_KFAST ? e / BK : e % BM, kk = A_KFAST ? e % BK : e / BM;
        const int m = m0 + r, k = k0 + kk;
        ra[j] = (m < M && k < kend) ? A[A_KFAST ? (int64_t)m * lda + k : (int64_t)k * lda + m] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < BE; ++j) {
      const int e = tid + 256 * j;
      const int n = e % NP, kk = e / NP;
      const int k = k0 + kk;
      rb[j] = (kk < BK && n < N && k < kend) ? B[(int64_t)k * ldb + n] : T(0);
    }
  };
  auto lstore = [&](int buf) {
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < AE / 4; ++j) {
        int r, kk;
        chunk_rk(tid + 256 * j, r, kk);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (A_KFAST) As[buf][r * LDK + kk + i] = ra[4 * j + i];
          else As[buf][(r + i) * LDK + kk] = ra[4 * j + i];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < AE; ++j) {
        const int e = tid + 256 * j;
        const int r = A_KFAST ? e / BK : e % BM, kk = A_KFAST ? e % BK : e / BM;
        As[buf][r * LDK + kk] = ra[j];
      }
    }
#pragma unroll
    for (int j = 0; j < BE; ++j) {
      const int e = tid + 256 * j;
      const int n = e % NP, kk = e / NP;
      if (kk < BK) Bs[buf][n * LDK + kk] = rb[j];
    }
  };

  typedef typename TsCfg<T>::V V;
  V acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[j][q] = 0;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    lstore(0);
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const T av = As[cur][(wave * 16 + lr) * LDK + ks + lk];
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = mfma<T>(av, Bs[cur][(j * 16 + lr) * LDK + ks + lk], acc[j]);
    }
    if (kt + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }

  // partial product rows: f32 4 (l/16) + q, f64 (l/16) + 4 q; column l % 16
  T* __restrict__ P = part + ((int64_t)gi * nsplit + sk) * M * N;
  constexpr bool F64 = sizeof(T) == 8;
  const int rb0 = F64 ? lk : lk * 4, rst = F64 ? 4 : 1;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int n = j * 16 + lr;
    if (n >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + wave * 16 + rb0 + rst * q;
      if (m < M) P[(int64_t)m * N + n] = acc[j][q];
    }
  }
}

// ---------------------------------------------------------------------------
// Register-streaming form for float32 with N <= 64: one wave computes 64
// rows x NT*16 columns over a K chunk with no LDS and no barrier, three
// 16-wide K blocks in flight in registers; B (small, L2-resident) is read
// element by element.  MFMA step i of a 16-wide K block contracts
// k + 4 g + i over the lane groups g = l / 16, and B is read in that order:
// B[k + 4 g + i][16 cb + r], r = l % 16.  k-fast A (A[m][k]): lane l reads the
// 16-byte piece A[m0 + 16 rb + r][k + 4 g .. + 3], value i feeding step i of
// row block rb (rows m0 + 16 rb + 0..15).  m-fast A (A[k][m]): lane l reads
// A[k + 4 g + i][m0 + 4 r .. + 3] for step i, value q feeding row block q,
// which then holds the rows m0 + 4 r' + q, r' = 0..15 (16 lanes read 256
// contiguous bytes of a row of A either way).
// ---------------------------------------------------------------------------
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float comp(const float4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// R row blocks of 16 per wave (R = 2: twice the waves for the same K
// chunks).  m-fast A: lane l reads R consecutive rows per K step (16 or 8
// bytes), value q feeding row block q, which holds rows m0 + R r' + q.
template <int NT, bool AK, int R = 4>
__global__ void __launch_bounds__(256, 2)
ts_stream_kernel(int32_t M, int32_t N, int32_t K, int64_t lda, int64_t ldb, int32_t kchunk, int32_t nsplit,
                 int32_t mtiles, int32_t ntasks, GemmGroup g, float* __restrict__ part) {
  static_assert(R == 4 || R == 2, "row blocks per wave");
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= ntasks) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int mt = task % mtiles;
  const int sk = (task / mtiles) % nsplit;
  const int gi = task / (mtiles * nsplit);
  const float* __restrict__ A = (const float*)g.A[gi];
  const float* __restrict__ B = (const float*)g.B[gi];
  const int m0 = mt * 16 * R;
  const int kbeg = sk * kchunk, kend = min(K, kbeg + kchunk);
  const float* arow[R];
#pragma unroll
  for (int rb = 0; rb < R; ++rb)
    arow[rb] = AK ? A + (int64_t)min(m0 + rb * 16 + lr, M - 1) * lda : A + min(m0 + R * lr, M - R);
  int ncol[NT];
#pragma unroll
  for (int cb = 0; cb < NT; ++cb) ncol[cb] = min(cb * 16 + lr, N - 1);
  v4f acc[R][NT];
#pragma unroll
  for (int rb = 0; rb < R; ++rb)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int NA = AK ? R : 4;  // A loads per K block
  float4 a[3][NA];
  float b[3][NT][4];
  // K block t of the chunk into ring slot st.  Addresses are clamped to the
  // chunk's last four columns, so the loads carry no condition and no select
  // (either would make the wave wait for the ring right after issuing it);
  // whole blocks are always in range, and a block past the chunk is loaded
  // but never used.
  auto load = [&](int st, int t) {
    const int kc = min(kbeg + t * 16 + 4 * lg, kend - 4);  // kend - kbeg >= 4, multiples of 4
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      if constexpr (AK || R == 4) {
        a[st][j] = *reinterpret_cast<const float4*>(AK ? arow[j] + kc : arow[0] + (int64_t)(kc + j) * lda);
      } else {
        const float2 v = *reinterpret_cast<const float2*>(arow[0] + (int64_t)(kc + j) * lda);
        a[st][j] = make_float4(v.x, v.y, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NT; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) b[st][cb][i] = B[(int64_t)(kc + i) * ldb + ncol[cb]];
  };
  // ragged last block: lane groups past the chunk end contribute zeros
  auto mask = [&](int st, bool kin) {
#pragma unroll
    for (int j = 0; j < NA; ++j)
      if (!kin) a[st][j] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int cb = 0; cb < NT; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) b[st][cb][i] = kin ? b[st][cb][i] : 0.f;
  };
  auto compute = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int rb = 0; rb < R; ++rb) {
        const float av = AK ? comp(a[st][rb], i) : comp(a[st][i], rb);
#pragma unroll
        for (int cb = 0; cb < NT; ++cb) acc[rb][cb] = mfma4(av, b[st][cb][i], acc[rb][cb]);
      }
  };
  // A region loads the next block into the slot just freed and computes the
  // following block, the loads spread evenly among its MFMAs: issued in a
  // burst between MFMA blocks, the same loads leave the matrix cores idle
  // about half the time
  constexpr int NL = NA + 4 * NT;                 // loads per block
  constexpr int NM = 4 * R * NT;                  // MFMAs per block
  auto region = [&](int ls, int lt, int cs) {
    load(ls, lt);
    compute(cs);
    if constexpr (NM >= NL) {
      constexpr int per = NM / NL;
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one VMEM read
        __builtin_amdgcn_sched_group_barrier(0x008, per, 0);  // then MFMAs
      }
      if constexpr (NM > per * NL) __builtin_amdgcn_sched_group_barrier(0x008, NM - per * NL, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  const int span = kend - kbeg;
  const int nfull = span / 16;
  __builtin_amdgcn_sched_barrier(0);
  load(0, 0);
  load(1, 1);
  load(2, 2);
  __builtin_amdgcn_sched_barrier(0);
  // block bb lives in slot bb % 3; blocks past nfull are loaded and dropped
  int bb = 0;
  if (nfull > 0) {
    compute(0);
    bb = 1;
  }
  __builtin_amdgcn_sched_barrier(0);
  for (; bb + 3 <= nfull; bb += 3) {
    region(0, bb + 2, 1);
    region(1, bb + 3, 2);
    region(2, bb + 4, 0);
  }
  if (bb < nfull) compute(1);
  if (bb + 1 < nfull) compute(2);
  // ragged last block (every slot is free by now): lane groups past the chunk
  // end contribute zeros
  if (nfull * 16 < span) {
    load(0, nfull);
    mask(0, kbeg + nfull * 16 + 4 * lg < kend);
    compute(0);
  }
  float* __restrict__ P = part + ((int64_t)gi * nsplit + sk) * M * N;
#pragma unroll
  for (int rb = 0; rb < R; ++rb)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      const int n = cb * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = AK ? m0 + rb * 16 + 4 * lg + q : m0 + R * (4 * lg + q) + rb;
        if (m < M && n < N) P[(int64_t)m * N + n] = acc[rb][cb][q];
      }
    }
}

template <typename T, typename TO>
__global__ void ts_reduce_kernel(const T* __restrict__ part, int32_t M, int32_t N, int32_t nsplit, int64_t ldc,
                                 GemmGroup g) {
  const int gi = blockIdx.y;
  const T* __restrict__ p = part + (int64_t)gi * nsplit * M * N;
  TO* __restrict__ C = (TO*)g.C[gi];
  const int64_t MN = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MN; e += (int64_t)gridDim.x * blockDim.x) {
    const T acc = ordered_sum(p + e, nsplit, MN);
    const int64_t m = e / N, n = e - m * N;
    C[m * ldc + n] = (TO)acc;
  }
}

// the same, float32 partials into a float32 output and a float64 copy
__global__ void ts_reduce2_kernel(const float* __restrict__ part, int32_t M, int32_t N, int32_t nsplit, int64_t ldc,
                                  GemmGroup g, GemmGroup g2) {
  const int gi = blockIdx.y;
  const float* __restrict__ p = part + (int64_t)gi * nsplit * M * N;
  float* __restrict__ C = (float*)g.C[gi];
  double* __restrict__ C2 = (double*)g2.C[gi];
  const int64_t MN = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MN; e += (int64_t)gridDim.x * blockDim.x) {
    const float acc = ordered_sum(p + e, nsplit, MN);
    const int64_t m = e / N, n = e - m * N;
    C[m * ldc + n] = acc;
    C2[m * ldc + n] = (double)acc;
  }
}

template <typename T, bool AK, bool VEC>
hipError_t launch_partial(hipStream_t s, int nt, dim3 grid, int32_t M, int32_t N, int32_t K, int64_t lda,
                          int64_t ldb, int32_t kchunk, int32_t nsplit, int32_t mtiles, const GemmGroup& g,
                          T* part) {
#define TS_CASE(NTV)                                                                                  \
  case NTV:                                                                                           \
    hipLaunchKernelGGL((ts_partial_kernel<T, AK, NTV, VEC>), grid, dim3(256), 0, s, M, N, K, lda, ldb, \
                       kchunk, nsplit, mtiles, g, part);                                              \
    break;
  switch (nt) {
    TS_CASE(1) TS_CASE(2) TS_CASE(3) TS_CASE(4) TS_CASE(5) TS_CASE(6)
    TS_CASE(7) TS_CASE(8) TS_CASE(9) TS_CASE(10) TS_CASE(11) TS_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef TS_CASE
  return hipGetLastError();
}

}  // namespace

// the register-streaming form is the default; CTM_TS_FORM=lds selects the
// LDS-tiled form for every shape (both compute the same sums in other orders)
static bool stream_form() {
  static const bool v = [] {
    const char* e = std::getenv("CTM_TS_FORM");
    return !(e && std::strcmp(e, "lds") == 0);
  }();
  return v;
}

// rows per wave of the register-streaming form for k-fast and m-fast A:
// 32 (CTM_TS_ROWS=64, CTM_TS_ROWS_M=64 select 64).  With about one wave per
// SIMD at the split counts the tuner picks, a 64-row wave spent half its
// time waiting for its loads; 32-row waves double the waves per SIMD for the
// same K chunks and partials
static int ts_rows_ak() {
  static const int v = [] {
    const char* e = std::getenv("CTM_TS_ROWS");
    return e && std::atoi(e) == 64 ? 64 : 32;
  }();
  return v;
}
static int ts_rows_mk() {
  static const int v = [] {
    const char* e = std::getenv("CTM_TS_ROWS_M");
    return e && std::atoi(e) == 64 ? 64 : 32;
  }();
  return v;
}

bool ts_gemm_supported(int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va, const View& vb,
                       const View& vc) {
  if (!((ta == F32 && (tc == F32 || tc == F64)) || (ta == F64 && tc == F64))) return false;
  if (N < 1 || N > NMAX || M < 1 || K < 1 || M > INT32_MAX || K > INT32_MAX) return false;
  // plain strided operands only
  const bool a_plain = (va.r_hs == 0 && va.c_hs == 0) && (va.c_ls == 1 || va.r_ls == 1);
  const bool b_plain = vb.r_hs == 0 && vb.c_hs == 0 && vb.c_ls == 1;
  const bool c_plain = vc.r_hs == 0 && vc.c_hs == 0 && vc.c_ls == 1;
  return a_plain && b_plain && c_plain;
}

int64_t ts_gemm_scratch_elems(int64_t M, int64_t N, int groups, int nsplit) {
  return (int64_t)nsplit * M * N * groups;
}

static hipError_t ts_gemm_v(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va,
                            const View& vb, const View& vc, const GemmGroup& g, int groups, void* scratch,
                            int64_t scratch_bytes, int64_t target, const GemmGroup* c2);

hipError_t ts_gemm(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va, const View& vb,
                   const View& vc, const GemmGroup& g, int groups, void* scratch, int64_t scratch_bytes,
                   const GemmGroup* c2) {
  if (groups < 1 || groups > MAXG || !ts_gemm_supported(ta, tc, M, N, K, va, vb, vc)) return hipErrorInvalidValue;
  if (c2 && (ta != F32 || tc != F32)) return hipErrorInvalidValue;
  // split count target from the tile table (about 2048 wave tasks by default)
  const TileKey key{TK_TS, ta, tc, va.c_ls == 1, 1, groups, M, N, K};
  int v = tile_lookup(key, -1);
  if (v < 0 && tile_tuning_on() && !dry_run()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      // every variant writes C from A and B only, so the trials are harmless
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        float best_ms = 1e30f;
        int best = 3;
        for (int t = 0; t < TILE_VARIANTS[TK_TS]; ++t) {
          float ms_min = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess ||
                ts_gemm_v(s, ta, tc, M, N, K, va, vb, vc, g, groups, scratch, scratch_bytes, (int64_t)256 << t,
                          c2) != hipSuccess ||
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
  if (v < 0 || v >= TILE_VARIANTS[TK_TS]) v = 3;
  return ts_gemm_v(s, ta, tc, M, N, K, va, vb, vc, g, groups, scratch, scratch_bytes, (int64_t)256 << v, c2);
}

static hipError_t ts_gemm_v(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va,
                            const View& vb, const View& vc, const GemmGroup& g, int groups, void* scratch,
                            int64_t scratch_bytes, int64_t target, const GemmGroup* c2) {
  const bool ak = va.c_ls == 1;
  const int64_t lda = ak ? va.r_ls : va.c_ls, ldb = vb.r_ls, ldc = vc.r_ls;
  const size_t ea = dtype_size(ta), ec = dtype_size(tc);
  const size_t sa = (size_t)(view_max(va, M, K) + 1) * ea, sb = (size_t)(view_max(vb, K, N) + 1) * ea,
               sc = (size_t)(view_max(vc, M, N) + 1) * ec;
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], sa, "ts A") || !span_ok(g.B[i], sb, "ts B") || !span_ok(g.C[i], sc, "ts C") ||
        (c2 && !span_ok(c2->C[i], (size_t)(view_max(vc, M, N) + 1) * 8, "ts C2")))
      return hipErrorInvalidValue;
  // enough work-groups to fill the chip several times over, K chunks of at
  // least 8 steps, and partials that fit the scratch
  const int BK = ta == F32 ? 32 : 16;
  const int64_t mtiles = (M + BM - 1) / BM;
  int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>((target + mtiles * groups - 1) / (mtiles * groups),
                                                          K / (8 * BK)));
  while (nsplit > 1 && ts_gemm_scratch_elems(M, N, groups, (int)nsplit) * (int64_t)ea > scratch_bytes) nsplit /= 2;
  if (ts_gemm_scratch_elems(M, N, groups, (int)nsplit) * (int64_t)ea > scratch_bytes) return hipErrorInvalidValue;
  const int64_t kchunk = ((K + nsplit - 1) / nsplit + BK - 1) / BK * BK;
  nsplit = (K + kchunk - 1) / kchunk;
  if (!span_ok(scratch, (size_t)ts_gemm_scratch_elems(M, N, groups, (int)nsplit) * ea, "ts scratch"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const int nt = (int)((N + 15) / 16);
  dim3 grid((unsigned)(mtiles * nsplit * groups));
  hipError_t e;
  // 16-byte A loads when every chunk start is 16-byte aligned and chunks never
  // straddle the M or K edge
  bool vec = ta == F32 && lda % 4 == 0 && K % 4 == 0 && M % 4 == 0;
  for (int i = 0; i < groups && vec; ++i) vec = ((uintptr_t)g.A[i] & 15) == 0;
  const int32_t M32 = (int32_t)M, N32 = (int32_t)N, K32 = (int32_t)K, kc32 = (int32_t)kchunk,
                ns32 = (int32_t)nsplit, mt32 = (int32_t)mtiles;
  if (ta == F32 && vec && N <= 64 && stream_form()) {
    // register-streaming form: 32 or 64 rows per wave, K chunks of whole
    // three-block groups, about target waves
    const int rows = ak ? ts_rows_ak() : ts_rows_mk();
    const int64_t mt64 = (M + rows - 1) / rows;
    int64_t ns2 = std::max<int64_t>(1, std::min<int64_t>((target + mt64 * groups - 1) / (mt64 * groups), K / 48));
    while (ns2 > 1 && ts_gemm_scratch_elems(M, N, groups, (int)ns2) * 4 > scratch_bytes) ns2 /= 2;
    int64_t kc2 = ((K + ns2 - 1) / ns2 + 47) / 48 * 48;
    ns2 = (K + kc2 - 1) / kc2;
    if (ts_gemm_scratch_elems(M, N, groups, (int)ns2) * 4 <= scratch_bytes &&
        span_ok(scratch, (size_t)ts_gemm_scratch_elems(M, N, groups, (int)ns2) * 4, "ts scratch")) {
      const int64_t ntasks = mt64 * ns2 * groups;
      dim3 g2((unsigned)((ntasks + 3) / 4));
      const int nt2 = (int)((N + 15) / 16);
#define TS2_LAUNCH(NTV, AKV, RV)                                                                           \
  hipLaunchKernelGGL((ts_stream_kernel<NTV, AKV, RV>), g2, dim3(256), 0, s, M32, N32, K32, lda, ldb,         \
                     (int32_t)kc2, (int32_t)ns2, (int32_t)mt64, (int32_t)ntasks, g, (float*)scratch)
#define TS2_CASE(NTV)                                                                                        \
  case NTV:                                                                                                  \
    if (ak && rows == 32) TS2_LAUNCH(NTV, true, 2);                                                          \
    else if (ak) TS2_LAUNCH(NTV, true, 4);                                                                   \
    else if (rows == 32) TS2_LAUNCH(NTV, false, 2);                                                          \
    else TS2_LAUNCH(NTV, false, 4);                                                                          \
    break;
      switch (nt2) {
        TS2_CASE(1) TS2_CASE(2) TS2_CASE(3) TS2_CASE(4)
        default: return hipErrorInvalidValue;
      }
#undef TS2_CASE
#undef TS2_LAUNCH
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      nsplit = ns2;
      goto reduce;
    }
  }
  if (ta == F32) {
    float* ps = (float*)scratch;
    if (vec)
      e = ak ? launch_partial<float, true, true>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps)
             : launch_partial<float, false, true>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps);
    else
      e = ak ? launch_partial<float, true, false>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps)
             : launch_partial<float, false, false>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps);
  } else {
    double* ps = (double*)scratch;
    e = ak ? launch_partial<double, true, false>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps)
           : launch_partial<double, false, false>(s, nt, grid, M32, N32, K32, lda, ldb, kc32, ns32, mt32, g, ps);
  }
  if (e != hipSuccess) return e;
reduce:
  const int64_t blocks = std::min<int64_t>(1024, std::max<int64_t>(1, (M * N + 255) / 256));
  dim3 rg((unsigned)blocks, (unsigned)groups);
  if (c2)
    hipLaunchKernelGGL(ts_reduce2_kernel, rg, dim3(256), 0, s, (const float*)scratch, (int32_t)M, (int32_t)N,
                       (int32_t)nsplit, ldc, g, *c2);
  else if (ta == F32 && tc == F32)
    hipLaunchKernelGGL((ts_reduce_kernel<float, float>), rg, dim3(256), 0, s, (const float*)scratch, (int32_t)M,
                       (int32_t)N, (int32_t)nsplit, ldc, g);
  else if (ta == F32)
    hipLaunchKernelGGL((ts_reduce_kernel<float, double>), rg, dim3(256), 0, s, (const float*)scratch, (int32_t)M,
                       (int32_t)N, (int32_t)nsplit, ldc, g);
  else
    hipLaunchKernelGGL((ts_reduce_kernel<double, double>), rg, dim3(256), 0, s, (const double*)scratch, (int32_t)M,
                       (int32_t)N, (int32_t)nsplit, ldc, g);
  return hipGetLastError();
}

}  // namespace ctmk
