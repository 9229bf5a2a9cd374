// Enlarged-corner double-layer contraction in bf16 on gfx950 MFMA.
//
//   Q[(g,dn),(b,r)] = sum_{(l,u)} Y[(g,b),(l,u)] * b[(l,u),(dn,r)]
//
// with Y (bf16, row-major M x K, M = chi^2, K = D^4) and the double layer
// stored transposed, bT = b^T (bf16, row-major N x K, N = D^4).  Both operands
// are K-contiguous, so 16-byte global loads land in LDS tiles [row][k] that
// feed v_mfma_f32_16x16x32_bf16 directly (lane l reads row l%16, k 8(l/16) ..
// +7).  Workgroup tile 256 x 144, four waves of 64 x 144 (4 x 9 MFMA tiles),
// K step 32, register-staged double buffering.  The f32 result is written
// through the two-level output view of the enlarged-corner matrix.
#include "kernels.h"

#include <hip/hip_bf16.h>

namespace ctmk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 144, BK = 32, LDK = BK + 8;  // LDS row: 40 bf16 = 80 B
constexpr int TM = 4, TN = 9;                              // 16x16 tiles per wave
constexpr int A_CHUNKS = BM * BK / 8 / 256;                // 16-byte chunks per thread: 4
constexpr int B_CHUNKS = (BN * BK / 8 + 255) / 256;        // 3 (576 chunks)

struct OutView {
  int32_t r_ext, c_ext;
  int64_t r_ls, r_hs, c_ls, c_hs;
};

__device__ __forceinline__ u32x4 load16(const __bf16* p, bool ok) {
  if (ok) return *reinterpret_cast<const u32x4*>(p);
  u32x4 z = {0u, 0u, 0u, 0u};
  return z;
}

__global__ void __launch_bounds__(256, 2)
corner_bf16_kernel(int32_t M, int32_t N, int32_t K, OutView vc, GemmGroup g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * LDK];
  const int gi = blockIdx.z;
  const __bf16* __restrict__ A = (const __bf16*)g.A[gi];
  const __bf16* __restrict__ Bt = (const __bf16*)g.B[gi];
  float* __restrict__ C = (float*)g.C[gi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  // load slots: chunk e covers row e / 4, k 8 (e % 4) .. +7 of the tile
  u32x4 ra[A_CHUNKS], rb[B_CHUNKS];
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < A_CHUNKS; ++j) {
      const int e = tid + 256 * j, row = e >> 2, kc = (e & 3) * 8;
      const int m = m0 + row, k = k0 + kc;
      ra[j] = load16(A + (int64_t)m * K + k, m < M && k < K);
    }
#pragma unroll
    for (int j = 0; j < B_CHUNKS; ++j) {
      const int e = tid + 256 * j, row = e >> 2, kc = (e & 3) * 8;
      const int n = n0 + row, k = k0 + kc;
      rb[j] = load16(Bt + (int64_t)n * K + k, e < BN * 4 && n < N && k < K);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < A_CHUNKS; ++j) {
      const int e = tid + 256 * j, row = e >> 2, kc = (e & 3) * 8;
      *reinterpret_cast<u32x4*>(&As[buf][row * LDK + kc]) = ra[j];
    }
#pragma unroll
    for (int j = 0; j < B_CHUNKS; ++j) {
      const int e = tid + 256 * j, row = e >> 2, kc = (e & 3) * 8;
      if (e < BN * 4) *reinterpret_cast<u32x4*>(&Bs[buf][row * LDK + kc]) = rb[j];
    }
  };

  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + BK - 1) / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    v8bf av[TM], bv[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      av[i] = *reinterpret_cast<const v8bf*>(&As[cur][(wave * 64 + i * 16 + lr) * LDK + lk]);
#pragma unroll
    for (int j = 0; j < TN; ++j)
      bv[j] = *reinterpret_cast<const v8bf*>(&Bs[cur][(j * 16 + lr) * LDK + lk]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }

  // epilogue: acc[i][j][q] = C[4 (lane/16) + q][lane % 16] of tile (i, j)
  const int lc = lane & 15, lr4 = (lane >> 4) * 4;
  int64_t coff[TN];
  bool cok[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + j * 16 + lc;
    cok[j] = n < N;
    const int h = n / vc.c_ext, l = n - h * vc.c_ext;
    coff[j] = (int64_t)h * vc.c_hs + (int64_t)l * vc.c_ls;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + wave * 64 + i * 16 + lr4 + q;
      if (m >= M) continue;
      const int h = m / vc.r_ext, l = m - h * vc.r_ext;
      const int64_t roff = (int64_t)h * vc.r_hs + (int64_t)l * vc.r_ls;
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (cok[j]) C[roff + coff[j]] = acc[i][j][q];
    }
}

}  // namespace

bool corner_bf16_supported(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && (K % 8) == 0 && M <= INT32_MAX && N <= INT32_MAX;
}

hipError_t corner_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const View& vc, const GemmGroup& g,
                       int groups) {
  if (!corner_bf16_supported(M, N, K) || groups < 1 || groups > MAXG) return hipErrorInvalidValue;
  const size_t sc = (size_t)(view_max(vc, M, N) + 1) * 4;
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], (size_t)M * K * 2, "corner A") || !span_ok(g.B[i], (size_t)N * K * 2, "corner Bt") ||
        !span_ok(g.C[i], sc, "corner C") || ((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  OutView ov;
  ov.r_ext = (int32_t)(vc.r_ext > M ? M : vc.r_ext);
  ov.c_ext = (int32_t)(vc.c_ext > N ? N : vc.c_ext);
  ov.r_ls = vc.r_ls; ov.r_hs = vc.r_hs; ov.c_ls = vc.c_ls; ov.c_hs = vc.c_hs;
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)groups);
  hipLaunchKernelGGL(corner_bf16_kernel, grid, dim3(256), 0, s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g);
  return hipGetLastError();
}

}  // namespace ctmk
