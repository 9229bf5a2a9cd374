// Enlarged-corner double-layer contraction in bf16 on gfx950 MFMA.
//
//   Q[(g,dn),(b,r)] = sum_{(l,u)} Y[(g,b),(l,u)] * b[(l,u),(dn,r)]
//
// with Y (bf16, row-major M x K, M = chi^2, K = D^4) and the double layer
// stored transposed, bT = b^T (bf16, row-major N x K, N = D^4).  Both operands
// are K-contiguous, so 16-byte global loads land in LDS tiles [row][k]
// (chunk-swizzled, see lds_off) that feed v_mfma_f32_16x16x32_bf16 directly
// (lane l reads row l%16, k 8(l/16) .. +7).  Workgroup tile 256 x 144, four waves of 64 x 144 (4 x 9 MFMA tiles),
// K step 32, register-staged double buffering.  The f32 result is written
// through the two-level output view of the enlarged-corner matrix.
#include "kernels.h"

#include <hip/hip_bf16.h>

#include <cstdlib>
#include <cstring>

namespace ctmk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 144, BK = 32, LDK = BK;      // LDS row: 32 bf16 = 64 B, no padding
constexpr int TM = 4, TN = 9;                              // 16x16 tiles per wave
constexpr int A_CHUNKS = BM * BK / 8 / 256;                // 16-byte chunks per thread: 4
constexpr int B_CHUNKS = (BN * BK / 8 + 255) / 256;        // 3 (576 chunks)

struct OutView {
  int32_t r_ext, c_ext;
  int64_t r_ls, r_hs, c_ls, c_hs;
};

// LDS rows hold four 16-byte chunks (8 bf16 of k each); chunk c of row r is
// stored in slot c ^ swz(r).  A fragment read takes 16 consecutive rows at one
// chunk and a tile store takes 4 consecutive rows at all chunks; with the
// swizzle both touch distinct banks in every group of 8 (32 banks) or 16
// (64 banks) lanes.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }
__device__ __forceinline__ int lds_off(int r, int chunk) { return r * LDK + ((chunk ^ swz(r)) << 3); }

__device__ __forceinline__ u32x4 load16(const __bf16* p, bool ok) {
  if (ok) return *reinterpret_cast<const u32x4*>(p);
  u32x4 z = {0u, 0u, 0u, 0u};
  return z;
}

// Work-groups are dealt to the 8 XCDs round-robin in launch order, and each
// XCD has its own L2.  Launch index L runs on XCD L % 8; it takes tile
// t = (L % 8) * per_xcd + L / 8 of the (problem, M tile, N tile) sequence
// with N fastest, so each XCD works through a contiguous run of tiles: the
// N tiles that share an A row block run side by side on one XCD (A is read
// from HBM once), and the few B tiles of a problem stay in that XCD's L2.
__global__ void __launch_bounds__(256, 2)
corner_bf16_kernel(int32_t M, int32_t N, int32_t K, OutView vc, GemmGroup g, int32_t mt, int32_t nt,
                   int32_t tiles, int32_t per_xcd) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * LDK];
  const int L = blockIdx.x;
  const int t = (L & 7) * per_xcd + (L >> 3);
  if (t >= tiles) return;  // padding of the last XCD's run (whole work-group)
  const int gi = t / (mt * nt);
  const int rem = t - gi * (mt * nt);
  const int m0 = (rem / nt) * BM, n0 = (rem % nt) * BN;
  const __bf16* __restrict__ A = (const __bf16*)g.A[gi];
  const __bf16* __restrict__ Bt = (const __bf16*)g.B[gi];
  float* __restrict__ C = (float*)g.C[gi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

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
      const int e = tid + 256 * j, row = e >> 2;
      *reinterpret_cast<u32x4*>(&As[buf][lds_off(row, e & 3)]) = ra[j];
    }
#pragma unroll
    for (int j = 0; j < B_CHUNKS; ++j) {
      const int e = tid + 256 * j, row = e >> 2;
      if (e < BN * 4) *reinterpret_cast<u32x4*>(&Bs[buf][lds_off(row, e & 3)]) = rb[j];
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
  const int lr = lane & 15, lc = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    v8bf av[TM], bv[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      av[i] = *reinterpret_cast<const v8bf*>(&As[cur][lds_off(wave * 64 + i * 16 + lr, lc)]);
#pragma unroll
    for (int j = 0; j < TN; ++j)
      bv[j] = *reinterpret_cast<const v8bf*>(&Bs[cur][lds_off(j * 16 + lr, lc)]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }

  // epilogue: acc[i][j][q] = C[4 (lane/16) + q][lane % 16] of tile (i, j)
  const int lcol = lane & 15, lr4 = (lane >> 4) * 4;
  int64_t coff[TN];
  bool cok[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + j * 16 + lcol;
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


// Second form of the same contraction: the tiles go from HBM to LDS by 16-byte
// direct-to-LDS loads (lane t of a wave fills bytes 16 t .. 16 t + 15 after the
// wave-uniform base) into three LDS stages, issued two K steps ahead (after
// the current step's MFMAs, so that they do not compete with its fragment
// reads; the stage they fill was released by the step's barrier), with no
// register staging.  The chunk a lane loads is chosen so that its LDS slot
// follows the lds_off swizzle.  Rows past the matrix edge load a clamped
// (valid) row whose results are never stored; in a partial last K step the
// chunks past K load a clamped chunk and the B side of those chunks is zeroed
// in LDS before use.
constexpr int STAGES = 3;
constexpr int STAGE_ELEMS = (BM + BN) * BK;

__device__ __forceinline__ void wait_vm(int n) {
  // s_waitcnt vmcnt(n), other counters unconstrained (gfx9 encoding)
  if (n >= 7) __builtin_amdgcn_s_waitcnt(0xF77);
  else if (n == 6) __builtin_amdgcn_s_waitcnt(0xF76);
  else __builtin_amdgcn_s_waitcnt(0xF70);
}
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }  // lgkmcnt(0)

// Output modes.  OUT_V4 (float output whose rows are contiguous in groups of
// 4: vc.r_ls = 1, r_ext, r_hs, c_ls, c_hs and M multiples of 4, 16-byte
// aligned C): a lane's four accumulator rows go out as one 16-byte store, so a
// transposed output is written as densely as a row-major one.  OUT_SPLIT
// (bf16 output): each result x is stored as the A-side three-term split hi,
// hi, lo (hi = bf16(x), lo = bf16(x - hi)) at offsets 0, sstride, 2 sstride
// from its place in the view.
// OUT_V4 with bf16 output (the same conditions, 8-byte aligned C): the four
// rows go out as one 8-byte store.
constexpr int OUT_PLAIN = 0, OUT_V4 = 1, OUT_SPLIT = 2;

template <typename TO, int MODE>
__global__ void __launch_bounds__(256, 2)
corner_bf16_dma_kernel(int32_t M, int32_t N, int32_t K, OutView vc, GemmGroup g, int32_t mt, int32_t nt,
                       int32_t tiles, int32_t per_xcd, int64_t sstride) {
  __shared__ __attribute__((aligned(16))) __bf16 smem[STAGES * STAGE_ELEMS];
  const int L = blockIdx.x;
  const int t = (L & 7) * per_xcd + (L >> 3);
  if (t >= tiles) return;
  const int gi = t / (mt * nt);
  const int rem = t - gi * (mt * nt);
  const int m0 = (rem / nt) * BM, n0 = (rem % nt) * BN;
  const __bf16* __restrict__ A = (const __bf16*)g.A[gi];
  const __bf16* __restrict__ Bt = (const __bf16*)g.B[gi];
  TO* __restrict__ C = (TO*)g.C[gi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nk = (K + BK - 1) / BK;
  const bool partial = (K % BK) != 0;
  const int n_issue = wave == 0 ? 7 : 6;  // loads per wave per K step

  // loads of K step kt into stage kt % 3.  A: 16 blocks of 64 chunks (4 per
  // wave); B: 9 blocks (waves take blocks w, w + 4, w + 8 < 9)
  auto issue = [&](int kt) {
    __bf16* As = smem + (kt % STAGES) * STAGE_ELEMS;
    __bf16* Bs = As + BM * BK;
    const int k0 = kt * BK;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int blk = j * 4 + wave, e = blk * 64 + lane, row = e >> 2;
      const int chunk = (e & 3) ^ swz(row);
      const int m = min(m0 + row, M - 1), k = min(k0 + chunk * 8, K - 8);
      __builtin_amdgcn_global_load_lds(A + (int64_t)m * K + k, As + blk * 512, 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int blk = j * 4 + wave;
      if (blk < 9) {
        const int e = blk * 64 + lane, row = e >> 2;
        const int chunk = (e & 3) ^ swz(row);
        const int n = min(n0 + row, N - 1), k = min(k0 + chunk * 8, K - 8);
        __builtin_amdgcn_global_load_lds(Bt + (int64_t)n * K + k, Bs + blk * 512, 16, 0, 0);
      }
    }
  };

  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int lr = lane & 15, lc = lane >> 4;
  issue(0);
  if (nk > 1) issue(1);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's loads of step kt are done once at most those of step kt + 1
    // are outstanding; the barrier then covers every wave's loads, and every
    // wave's reads of the stage that step kt + 2 refills
    wait_vm(kt + 1 < nk ? n_issue : 0);
    __bf16* As = smem + (kt % STAGES) * STAGE_ELEMS;
    __bf16* Bs = As + BM * BK;
    if (partial && kt == nk - 1) {
      const int k0 = kt * BK;
      for (int e = tid; e < BN * 4; e += 256) {
        const int row = e >> 2, c = e & 3;
        if (k0 + c * 8 >= K) *reinterpret_cast<u32x4*>(&Bs[lds_off(row, c)]) = u32x4{0u, 0u, 0u, 0u};
      }
      wait_lgkm0();
    }
    // a bare barrier: __syncthreads() would also wait for the loads of the
    // next step (its fence drains every outstanding memory operation)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    v8bf av[TM], bv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) bv[j] = *reinterpret_cast<const v8bf*>(&Bs[lds_off(j * 16 + lr, lc)]);
#pragma unroll
    for (int i = 0; i < TM; ++i) av[i] = *reinterpret_cast<const v8bf*>(&As[lds_off(wave * 64 + i * 16 + lr, lc)]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (kt + 2 < nk) issue(kt + 2);
  }

  const int lcol = lane & 15, lr4 = (lane >> 4) * 4;
  int64_t coff[TN];
  bool cok[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + j * 16 + lcol;
    cok[j] = n < N;
    const int h = n / vc.c_ext, l = n - h * vc.c_ext;
    coff[j] = (int64_t)h * vc.c_hs + (int64_t)l * vc.c_ls;
  }
  if constexpr (MODE == OUT_V4) {
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int m = m0 + wave * 64 + i * 16 + lr4;
      if (m >= M) continue;
      const int h = m / vc.r_ext, l = m - h * vc.r_ext;
      const int64_t roff = (int64_t)h * vc.r_hs + l;
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (cok[j]) {
          if constexpr (sizeof(TO) == 4) {
            *reinterpret_cast<float4*>(C + roff + coff[j]) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
          } else {
            union { __bf16 h[4]; uint2 u; } pk;
#pragma unroll
            for (int q = 0; q < 4; ++q) pk.h[q] = (__bf16)acc[i][j][q];
            *reinterpret_cast<uint2*>(C + roff + coff[j]) = pk.u;
          }
        }
    }
    return;
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
        if (cok[j]) {
          if constexpr (MODE == OUT_SPLIT) {
            const float x = acc[i][j][q];
            const __bf16 hi = (__bf16)x;
            TO* o = C + roff + coff[j];
            o[0] = hi;
            o[sstride] = hi;
            o[2 * sstride] = (__bf16)(x - (float)hi);
          } else {
            C[roff + coff[j]] = (TO)acc[i][j][q];
          }
        }
    }
}

}  // namespace

bool corner_bf16_supported(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && (K % 8) == 0 && M <= INT32_MAX && N <= INT32_MAX;
}

hipError_t corner_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const View& vc, const GemmGroup& g,
                       int groups, int tout, int64_t split_stride) {
  if (!corner_bf16_supported(M, N, K) || groups < 1 || groups > MAXG || (tout != F32 && tout != BF16) ||
      split_stride < 0 || (split_stride > 0 && tout != BF16))
    return hipErrorInvalidValue;
  const size_t sc = (size_t)(view_max(vc, M, N) + 1 + 2 * split_stride) * dtype_size(tout);
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], (size_t)M * K * 2, "corner A") || !span_ok(g.B[i], (size_t)N * K * 2, "corner Bt") ||
        !span_ok(g.C[i], sc, "corner C") || ((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  OutView ov;
  ov.r_ext = (int32_t)(vc.r_ext > M ? M : vc.r_ext);
  ov.c_ext = (int32_t)(vc.c_ext > N ? N : vc.c_ext);
  ov.r_ls = vc.r_ls; ov.r_hs = vc.r_hs; ov.c_ls = vc.c_ls; ov.c_hs = vc.c_hs;
  const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN, tiles = mt * nt * groups;
  if (tiles > INT32_MAX / 2) return hipErrorInvalidValue;
  const int64_t per_xcd = (tiles + 7) / 8;
  static const bool use_dma = [] {
    const char* e = std::getenv("CTM_CORNER_STAGING");  // "registers" selects the first form (fp32 output)
    return !(e && std::strcmp(e, "registers") == 0);
  }();
  const dim3 grid((unsigned)(8 * per_xcd));
  bool v4 = use_dma && split_stride == 0 && vc.r_ls == 1 && ov.r_ext % 4 == 0 && vc.r_hs % 4 == 0 &&
            vc.c_ls % 4 == 0 && vc.c_hs % 4 == 0 && M % 4 == 0;
  for (int i = 0; i < groups && v4; ++i) v4 = ((uintptr_t)g.C[i] & (tout == F32 ? 15 : 7)) == 0;
  const int64_t z = 0;
  if (tout == BF16 && split_stride > 0)
    hipLaunchKernelGGL((corner_bf16_dma_kernel<__bf16, OUT_SPLIT>), grid, dim3(256), 0, s, (int32_t)M, (int32_t)N,
                       (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, split_stride);
  else if (tout == BF16 && v4)
    hipLaunchKernelGGL((corner_bf16_dma_kernel<__bf16, OUT_V4>), grid, dim3(256), 0, s, (int32_t)M, (int32_t)N,
                       (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, z);
  else if (tout == BF16)
    hipLaunchKernelGGL((corner_bf16_dma_kernel<__bf16, OUT_PLAIN>), grid, dim3(256), 0, s, (int32_t)M, (int32_t)N,
                       (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, z);
  else if (v4)
    hipLaunchKernelGGL((corner_bf16_dma_kernel<float, OUT_V4>), grid, dim3(256), 0, s, (int32_t)M, (int32_t)N,
                       (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, z);
  else if (use_dma)
    hipLaunchKernelGGL((corner_bf16_dma_kernel<float, OUT_PLAIN>), grid, dim3(256), 0, s, (int32_t)M, (int32_t)N,
                       (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, z);
  else
    hipLaunchKernelGGL(corner_bf16_kernel, grid, dim3(256), 0, s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g,
                       (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd);
  return hipGetLastError();
}

}  // namespace ctmk
