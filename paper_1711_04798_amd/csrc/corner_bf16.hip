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

#include <algorithm>
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
  // s_waitcnt vmcnt(n) for n <= 7 (larger n wait for 7), other counters
  // unconstrained (gfx9 encoding)
  switch (n) {
    case 0: __builtin_amdgcn_s_waitcnt(0xF70); break;
    case 1: __builtin_amdgcn_s_waitcnt(0xF71); break;
    case 2: __builtin_amdgcn_s_waitcnt(0xF72); break;
    case 3: __builtin_amdgcn_s_waitcnt(0xF73); break;
    case 4: __builtin_amdgcn_s_waitcnt(0xF74); break;
    case 5: __builtin_amdgcn_s_waitcnt(0xF75); break;
    case 6: __builtin_amdgcn_s_waitcnt(0xF76); break;
    default: __builtin_amdgcn_s_waitcnt(0xF77); break;
  }
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
// OUT_PACKA (bf16 output): the product is the enlarged corner's intermediate
// Y of the next product, element (m, n) = ((b, u), (g, l)) with m = b D2 + u
// and n = g D2 + l going to row R = g chi + b, column k = l D2 + u of Y, and Y
// is stored in the packed fragment layout that the next product reads as its
// A operand (see corner_bf16_packed_a_elems).  A lane's four accumulator rows
// are four consecutive u (D2 % 4 == 0), i.e. four consecutive k of one packed
// lane slot: one 8-byte store.
constexpr int OUT_PLAIN = 0, OUT_V4 = 1, OUT_SPLIT = 2, OUT_PACKA = 3;

struct Aux {
  int64_t sstride;   // OUT_SPLIT: offset of the second and third terms
  int32_t chi, d2;   // OUT_PACKA: R = g chi + b, k = l d2 + u
  int32_t kb;        // OUT_PACKA: k blocks of 32 per 16-row block of Y
};

// BF: B is held in the packed fragment layout of corner_bf16_pack_b (1 KiB
// blocks of 16 rows x 32 k in MFMA operand order, k blocks outermost): each
// B block of a K step is one contiguous 1 KiB direct-to-LDS load, and the
// fragment read of an LDS block is lane l at byte 16 l (no bank conflicts;
// the row-major form reads 16 rows at one 16-byte column, which the LDS
// serves at half rate).  Rows past N and k past K are zeros in the packed
// layout, so no clamping or zeroing is needed on the B side.
// AF: A is held in the packed layout of OUT_PACKA ([M / 16][K / 32] blocks
// of 1 KiB in MFMA operand order, rows padded to whole 256-row tiles): the
// same contiguous loads and linear fragment reads as BF; the k past K of a
// partial last step are zeroed in LDS (the padding is never written).
template <typename TO, int MODE, bool BF, bool AF, int RT = 4>
__global__ void __launch_bounds__(256, 2)
corner_bf16_dma_kernel(int32_t M, int32_t N, int32_t K, OutView vc, GemmGroup g, int32_t mt, int32_t nt,
                       int32_t tiles, int32_t per_xcd, Aux aux) {
  // RT row tiles of 16 per wave: BM = 64 RT rows per work-group
  constexpr int BMR = 64 * RT, SE = (BMR + BN) * BK;
  __shared__ __attribute__((aligned(16))) __bf16 smem[STAGES * SE];
  const int L = blockIdx.x;
  const int t = (L & 7) * per_xcd + (L >> 3);
  if (t >= tiles) return;
  const int gi = t / (mt * nt);
  const int rem = t - gi * (mt * nt);
  const int m0 = (rem / nt) * BMR, n0 = (rem % nt) * BN;
  const __bf16* __restrict__ A = (const __bf16*)g.A[gi];
  const __bf16* __restrict__ Bt = (const __bf16*)g.B[gi];
  TO* __restrict__ C = (TO*)g.C[gi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nk = (K + BK - 1) / BK;
  const bool partial = (K % BK) != 0;
  const int n_issue = wave == 0 ? RT + 3 : RT + 2;  // loads per wave per K step

  // loads of K step kt into stage kt % 3.  A: 4 RT blocks of 64 chunks (RT
  // per wave); B: 9 blocks (waves take blocks w, w + 4, w + 8 < 9)
  auto issue = [&](int kt) {
    __bf16* As = smem + (kt % STAGES) * SE;
    __bf16* Bs = As + BMR * BK;
    const int k0 = kt * BK;
#pragma unroll
    for (int j = 0; j < RT; ++j) {
      const int blk = j * 4 + wave;
      if constexpr (AF) {
        const int64_t pb = (int64_t)(m0 / 16 + blk) * nk + kt;
        __builtin_amdgcn_global_load_lds(A + pb * 512 + lane * 8, As + blk * 512, 16, 0, 0);
      } else {
        const int e = blk * 64 + lane, row = e >> 2;
        const int chunk = (e & 3) ^ swz(row);
        const int m = min(m0 + row, M - 1), k = min(k0 + chunk * 8, K - 8);
        __builtin_amdgcn_global_load_lds(A + (int64_t)m * K + k, As + blk * 512, 16, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int blk = j * 4 + wave;
      if (blk < 9) {
        if constexpr (BF) {
          // packed block (kt, n0 / 16 + blk) of nt * 9 row blocks per k block
          const int64_t pb = (int64_t)kt * (nt * 9) + n0 / 16 + blk;
          __builtin_amdgcn_global_load_lds(Bt + pb * 512 + lane * 8, Bs + blk * 512, 16, 0, 0);
        } else {
          const int e = blk * 64 + lane, row = e >> 2;
          const int chunk = (e & 3) ^ swz(row);
          const int n = min(n0 + row, N - 1), k = min(k0 + chunk * 8, K - 8);
          __builtin_amdgcn_global_load_lds(Bt + (int64_t)n * K + k, Bs + blk * 512, 16, 0, 0);
        }
      }
    }
  };

  v4f acc[RT][TN];
#pragma unroll
  for (int i = 0; i < RT; ++i)
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
    __bf16* As = smem + (kt % STAGES) * SE;
    __bf16* Bs = As + BMR * BK;
    if (!BF && partial && kt == nk - 1) {
      const int k0 = kt * BK;
      for (int e = tid; e < BN * 4; e += 256) {
        const int row = e >> 2, c = e & 3;
        if (k0 + c * 8 >= K) *reinterpret_cast<u32x4*>(&Bs[lds_off(row, c)]) = u32x4{0u, 0u, 0u, 0u};
      }
      wait_lgkm0();
    }
    if (AF && partial && kt == nk - 1) {
      // lane slot t of each block holds k = 8 (t / 16) .. + 7 of the step
      const int k0 = kt * BK;
      for (int e = tid; e < BMR * 4; e += 256) {
        const int blk = e >> 6, t = e & 63;
        if (k0 + (t >> 4) * 8 >= K) *reinterpret_cast<u32x4*>(&As[blk * 512 + t * 8]) = u32x4{0u, 0u, 0u, 0u};
      }
      wait_lgkm0();
    }
    // a bare barrier: __syncthreads() would also wait for the loads of the
    // next step (its fence drains every outstanding memory operation)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    v8bf av[RT], bv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j)
      bv[j] = BF ? *reinterpret_cast<const v8bf*>(&Bs[j * 512 + lane * 8])
                 : *reinterpret_cast<const v8bf*>(&Bs[lds_off(j * 16 + lr, lc)]);
#pragma unroll
    for (int i = 0; i < RT; ++i)
      av[i] = AF ? *reinterpret_cast<const v8bf*>(&As[(wave * RT + i) * 512 + lane * 8])
                 : *reinterpret_cast<const v8bf*>(&As[lds_off(wave * RT * 16 + i * 16 + lr, lc)]);
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (kt + 2 < nk) issue(kt + 2);
  }

  const int lcol = lane & 15, lr4 = (lane >> 4) * 4;
  if constexpr (MODE == OUT_PACKA) {
    // column n = (g, l): row R = g chi + b, column k = l D2 + u
    int gj[TN], lj[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + j * 16 + lcol;
      gj[j] = n < N ? n / aux.d2 : -1;
      lj[j] = n - gj[j] * aux.d2;
    }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int m = m0 + wave * RT * 16 + i * 16 + lr4;  // rows m .. m + 3: u .. u + 3 of one b
      if (m >= M) continue;
      const int b = m / aux.d2, u = m - b * aux.d2;
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (gj[j] >= 0) {
          const int R = gj[j] * aux.chi + b, k = lj[j] * aux.d2 + u;
          const int64_t off =
              ((int64_t)(R >> 4) * aux.kb + (k >> 5)) * 512 + ((R & 15) + 16 * ((k >> 3) & 3)) * 8 + (k & 7);
          union { __bf16 h[4]; uint2 u2; } pk;
#pragma unroll
          for (int q = 0; q < 4; ++q) pk.h[q] = (__bf16)acc[i][j][q];
          *reinterpret_cast<uint2*>(C + off) = pk.u2;
        }
    }
    return;
  }
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
    for (int i = 0; i < RT; ++i) {
      const int m = m0 + wave * RT * 16 + i * 16 + lr4;
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
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + wave * RT * 16 + i * 16 + lr4 + q;
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
            o[aux.sstride] = hi;
            o[2 * aux.sstride] = (__bf16)(x - (float)hi);
          } else {
            C[roff + coff[j]] = (TO)acc[i][j][q];
          }
        }
    }
}

// out[kb][rb][l][j] = bT[16 rb + l % 16][32 kb + 8 (l / 16) + j], zero past
// N rows or K columns; rb < rbp (N padded to whole 144-row tiles).
__global__ void pack_b_kernel(const __bf16* __restrict__ bT, int64_t N, int64_t K, int64_t rbp, int64_t total,
                              __bf16* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e & 7), l = (int)((e >> 3) & 63);
    const int64_t blk = e >> 9, rb = blk % rbp, kb = blk / rbp;
    const int64_t row = rb * 16 + (l & 15), k = kb * 32 + (l >> 4) * 8 + j;
    out[e] = (row < N && k < K) ? bT[row * K + k] : (__bf16)0.0f;
  }
}

struct Launch {
  dim3 grid;
  hipStream_t s;
  int32_t M, N, K;
  OutView ov;
  GemmGroup g;
  int32_t mt, nt, tiles, per_xcd;
  Aux aux;
};

template <typename TO, int MODE, bool BF, bool AF, int RT = 4>
void launch(const Launch& l) {
  hipLaunchKernelGGL((corner_bf16_dma_kernel<TO, MODE, BF, AF, RT>), l.grid, dim3(256), 0, l.s, l.M, l.N, l.K, l.ov,
                     l.g, l.mt, l.nt, l.tiles, l.per_xcd, l.aux);
}

// the float32-output product with 64 RT rows per work-group, operands
// packed (BF, AF) or row-major
template <bool BF, bool AF, int RT>
void launch_f32(const Launch& l, bool v4) {
  if (v4) launch<float, OUT_V4, BF, AF, RT>(l);
  else launch<float, OUT_PLAIN, BF, AF, RT>(l);
}
template <int RT>
void launch_f32_rt(const Launch& l, bool v4, bool b_packed, bool a_packed) {
  if (b_packed && a_packed) launch_f32<true, true, RT>(l, v4);
  else if (b_packed) launch_f32<true, false, RT>(l, v4);
  else launch_f32<false, false, RT>(l, v4);
}

}  // namespace

static bool corner_use_dma() {
  static const bool v = [] {
    const char* e = std::getenv("CTM_CORNER_STAGING");  // "registers" selects the first form (fp32 output)
    return !(e && std::strcmp(e, "registers") == 0);
  }();
  return v;
}

bool corner_packed_b() {
  static const bool v = [] {
    const char* e = std::getenv("CTM_CORNER_B");  // "rowmajor" keeps the double layer row-major
    return corner_use_dma() && !(e && std::strcmp(e, "rowmajor") == 0);
  }();
  return v;
}

bool corner_packed_a() {
  static const bool v = [] {
    const char* e = std::getenv("CTM_CORNER_A");  // "rowmajor" keeps the intermediate Y row-major
    return corner_packed_b() && !(e && std::strcmp(e, "rowmajor") == 0);
  }();
  return v;
}

int64_t corner_bf16_packed_b_elems(int64_t N, int64_t K) {
  if (N <= 0 || K <= 0) return 0;
  return ((K + BK - 1) / BK) * ((N + BN - 1) / BN * (BN / 16)) * 512;
}

hipError_t corner_bf16_pack_b(hipStream_t s, const void* bT, int64_t N, int64_t K, void* out) {
  const int64_t total = corner_bf16_packed_b_elems(N, K);
  if (total <= 0 || (K % 8) != 0) return hipErrorInvalidValue;
  if (!span_ok(bT, (size_t)N * K * 2, "pack_b in") || !span_ok(out, (size_t)total * 2, "pack_b out"))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const int64_t rbp = (N + BN - 1) / BN * (BN / 16);
  const int blocks = (int)std::min<int64_t>(8192, (total + 255) / 256);
  hipLaunchKernelGGL(pack_b_kernel, dim3(blocks), dim3(256), 0, s, (const __bf16*)bT, N, K, rbp, total,
                     (__bf16*)out);
  return hipGetLastError();
}

int64_t corner_bf16_packed_a_elems(int64_t M, int64_t K) {
  if (M <= 0 || K <= 0) return 0;
  // whole 256-row tiles and one more: the row tiles of every variant (64,
  // 128, 192 or 256 rows per work-group) stay inside
  return ((M + BM - 1) / BM + 1) * (BM / 16) * ((K + BK - 1) / BK) * 512;
}

hipError_t corner_bf16_to_packed_a(hipStream_t s, int64_t M, int64_t N, int64_t K, int64_t chi, int64_t d2,
                                   const GemmGroup& g, int groups) {
  // the output is Y (chi^2 x d2^2) of the next product: M = N = chi d2, rows
  // (b, u) with d2 % 4 == 0 so that a lane's four rows stay in one b
  if (!corner_bf16_supported(M, N, K) || groups < 1 || groups > MAXG || M != chi * d2 || N != chi * d2 ||
      d2 % 4 != 0 || chi * chi > INT32_MAX || d2 * d2 > INT32_MAX)
    return hipErrorInvalidValue;
  for (int i = 0; i < groups; ++i)
    if ((uintptr_t)g.C[i] & 7) return hipErrorInvalidValue;
  const int64_t ym = chi * chi, yk = d2 * d2;
  const size_t sc = (size_t)corner_bf16_packed_a_elems(ym, yk) * 2;
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], (size_t)M * K * 2, "corner A") || !span_ok(g.B[i], (size_t)N * K * 2, "corner Bt") ||
        !span_ok(g.C[i], sc, "corner packed Y") || ((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (!corner_use_dma()) return hipErrorInvalidValue;
  OutView ov{};
  ov.r_ext = (int32_t)std::min<int64_t>(M, INT32_MAX);
  ov.c_ext = (int32_t)std::min<int64_t>(N, INT32_MAX);
  const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN, tiles = mt * nt * groups;
  if (tiles > INT32_MAX / 2) return hipErrorInvalidValue;
  const int64_t per_xcd = (tiles + 7) / 8;
  Aux aux{0, (int32_t)chi, (int32_t)d2, (int32_t)((yk + BK - 1) / BK)};
  const Launch L{dim3((unsigned)(8 * per_xcd)), s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g, (int32_t)mt,
                 (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, aux};
  launch<__bf16, OUT_PACKA, false, false>(L);
  return hipGetLastError();
}

bool corner_bf16_supported(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && (K % 8) == 0 && M <= INT32_MAX && N <= INT32_MAX;
}

// The float32-output product with 64 rt rows per work-group (the variants
// compute every element with the same K order: bitwise equal).
static hipError_t launch_rt(hipStream_t s, int64_t M, int64_t N, int64_t K, const OutView& ov, bool v4,
                            const GemmGroup& g, int groups, int rt, bool b_packed, bool a_packed) {
  const int64_t bm = 64 * rt;
  const int64_t mt = (M + bm - 1) / bm, nt = (N + BN - 1) / BN, tiles = mt * nt * groups;
  if (tiles > INT32_MAX / 2) return hipErrorInvalidValue;
  const int64_t per_xcd = (tiles + 7) / 8;
  const Launch L{dim3((unsigned)(8 * per_xcd)), s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g, (int32_t)mt,
                 (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd, Aux{0, 0, 0, 0}};
  if (rt == 2) launch_f32_rt<2>(L, v4, b_packed, a_packed);
  else if (rt == 3) launch_f32_rt<3>(L, v4, b_packed, a_packed);
  else launch_f32_rt<4>(L, v4, b_packed, a_packed);
  return hipGetLastError();
}

// TK_CORNER variant v -> rows per work-group 64 rt: v = 0, 1, 2 -> rt = 4, 3, 2
static int rt_of(int v) { return v == 2 ? 2 : v == 1 ? 3 : 4; }

// Rows per work-group of a float32-output product: the tile table's entry; else,
// while table tuning is on (outside capture), the fastest variant timed on
// the call's own operands (each overwrites C); else 256 rows, or 128 when
// 256-row tiles would not fill two rounds of two work-groups per CU (the
// tail round of a small live extent).
static int corner_rows(hipStream_t s, int64_t M, int64_t N, int64_t K, const OutView& ov, bool v4,
                       const GemmGroup& g, int groups, bool b_packed, bool a_packed) {
  static const int forced = [] {  // CTM_CORNER_ROWS=256|192|128 overrides the choice
    const char* e = std::getenv("CTM_CORNER_ROWS");
    const int r = e ? std::atoi(e) : 0;
    return r == 256 ? 4 : r == 192 ? 3 : r == 128 ? 2 : 0;
  }();
  if (forced) return forced;
  const TileKey key{TK_CORNER, BF16, F32, a_packed ? 1 : 0, b_packed ? 1 : 0, groups, M, N, K};
  int v = tile_lookup(key, -1);
  if (v >= 0 && v < TILE_VARIANTS[TK_CORNER]) return rt_of(v);
  if (tile_tuning_on() && !dry_run()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
        hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      float best_ms = 1e30f;
      int best = 0;
      for (int t = 0; t < TILE_VARIANTS[TK_CORNER]; ++t) {
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          if (hipEventRecord(e0, s) != hipSuccess ||
              launch_rt(s, M, N, K, ov, v4, g, groups, rt_of(t), b_packed, a_packed) != hipSuccess ||
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
    if (v >= 0) return rt_of(v);
  }
  const int64_t tiles256 = (M + 255) / 256 * ((N + BN - 1) / BN) * groups;
  return tiles256 < 4 * 256 ? 2 : 4;
}

hipError_t corner_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const View& vc, const GemmGroup& g,
                       int groups, int tout, int64_t split_stride, bool b_packed, bool a_packed) {
  if (!corner_bf16_supported(M, N, K) || groups < 1 || groups > MAXG || (tout != F32 && tout != BF16) ||
      split_stride < 0 || (split_stride > 0 && tout != BF16) || (b_packed && (tout != F32 || split_stride)) ||
      (a_packed && !b_packed))
    return hipErrorInvalidValue;
  const size_t sc = (size_t)(view_max(vc, M, N) + 1 + 2 * split_stride) * dtype_size(tout);
  const size_t sb = b_packed ? (size_t)corner_bf16_packed_b_elems(N, K) * 2 : (size_t)N * K * 2;
  const size_t sa = a_packed ? (size_t)corner_bf16_packed_a_elems(M, K) * 2 : (size_t)M * K * 2;
  for (int i = 0; i < groups; ++i)
    if (!span_ok(g.A[i], sa, "corner A") || !span_ok(g.B[i], sb, "corner Bt") ||
        !span_ok(g.C[i], sc, "corner C") || ((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15))
      return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  OutView ov;
  ov.r_ext = (int32_t)(vc.r_ext > M ? M : vc.r_ext);
  ov.c_ext = (int32_t)(vc.c_ext > N ? N : vc.c_ext);
  ov.r_ls = vc.r_ls; ov.r_hs = vc.r_hs; ov.c_ls = vc.c_ls; ov.c_hs = vc.c_hs;
  const bool use_dma = corner_use_dma();
  const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN, tiles = mt * nt * groups;
  if (tiles > INT32_MAX / 2) return hipErrorInvalidValue;
  const int64_t per_xcd = (tiles + 7) / 8;
  if (b_packed && !use_dma) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(8 * per_xcd));
  bool v4 = use_dma && split_stride == 0 && vc.r_ls == 1 && ov.r_ext % 4 == 0 && vc.r_hs % 4 == 0 &&
            vc.c_ls % 4 == 0 && vc.c_hs % 4 == 0 && M % 4 == 0;
  for (int i = 0; i < groups && v4; ++i) v4 = ((uintptr_t)g.C[i] & (tout == F32 ? 15 : 7)) == 0;
  Aux aux{split_stride, 0, 0, 0};
  const Launch L{grid, s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g, (int32_t)mt, (int32_t)nt, (int32_t)tiles,
                 (int32_t)per_xcd, aux};
  if (tout == BF16 && use_dma && tiles < 256) {
    // fewer 256-row tiles than CUs: 128 rows per work-group (the same K
    // order per element, bitwise equal)
    const int64_t mt2 = (M + 127) / 128, tiles2 = mt2 * nt * groups, px2 = (tiles2 + 7) / 8;
    const Launch L2{dim3((unsigned)(8 * px2)), s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g, (int32_t)mt2,
                    (int32_t)nt, (int32_t)tiles2, (int32_t)px2, aux};
    if (split_stride > 0) launch<__bf16, OUT_SPLIT, false, false, 2>(L2);
    else if (v4) launch<__bf16, OUT_V4, false, false, 2>(L2);
    else launch<__bf16, OUT_PLAIN, false, false, 2>(L2);
  } else if (tout == BF16 && split_stride > 0) launch<__bf16, OUT_SPLIT, false, false>(L);
  else if (tout == BF16 && v4) launch<__bf16, OUT_V4, false, false>(L);
  else if (tout == BF16) launch<__bf16, OUT_PLAIN, false, false>(L);
  else if (use_dma)
    return launch_rt(s, M, N, K, ov, v4, g, groups, corner_rows(s, M, N, K, ov, v4, g, groups, b_packed, a_packed),
                     b_packed, a_packed);
  else
    hipLaunchKernelGGL(corner_bf16_kernel, grid, dim3(256), 0, s, (int32_t)M, (int32_t)N, (int32_t)K, ov, g,
                       (int32_t)mt, (int32_t)nt, (int32_t)tiles, (int32_t)per_xcd);
  return hipGetLastError();
}

}  // namespace ctmk
