// Internal launch interface of the gfx950 kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <utility>
#include <vector>

namespace ctmk {

// ---------------------------------------------------------------------------
// Host-side bounds registry.  Every launcher checks that each buffer span it
// is about to touch lies inside a single workspace allocation and refuses the
// launch otherwise (hipErrorInvalidValue), so an indexing mistake in the host
// orchestration becomes an error instead of a device fault.  In dry-run mode
// the launchers only check and never touch the device; this lets the whole
// orchestration run on a machine without a GPU.
// ---------------------------------------------------------------------------
struct Registry {
  uintptr_t lo = 0, hi = 0;                          // workspace range
  std::vector<std::pair<uintptr_t, size_t>> allocs;  // sorted by start
  bool dry = false;
  int violations = 0;
  const char* last = nullptr;
};
extern thread_local Registry* g_reg;
// true if [p, p + bytes) lies inside one registered allocation, or entirely
// outside the workspace (caller-owned buffers)
bool span_ok(const void* p, size_t bytes, const char* what);
inline bool dry_run() { return g_reg && g_reg->dry; }

enum DType : int { F64 = 0, F32 = 1, BF16 = 2 };

inline size_t dtype_size(int t) { return t == F64 ? 8 : (t == F32 ? 4 : 2); }

// A matrix view with two-level row and column indices:
// element (r, c) lives at  base + (r / r_ext) * r_hs + (r % r_ext) * r_ls
//                               + (c / c_ext) * c_hs + (c % c_ext) * c_ls
// (in elements).  A plain row-major matrix has r_ext = c_ext = huge,
// r_ls = ld, c_ls = 1.
struct View {
  int64_t r_ext, r_ls, r_hs;
  int64_t c_ext, c_ls, c_hs;
};

inline View rowmajor(int64_t ld) { return View{INT64_MAX / 4, ld, 0, INT64_MAX / 4, 1, 0}; }
inline View colmajor(int64_t ld) { return View{INT64_MAX / 4, 1, 0, INT64_MAX / 4, ld, 0}; }
inline View transposed(const View& v) {
  return View{v.c_ext, v.c_ls, v.c_hs, v.r_ext, v.r_ls, v.r_hs};
}
// largest element offset a view reaches over rows [0, R) and columns [0, C)
int64_t view_max(const View& v, int64_t R, int64_t C);

constexpr int MAXG = 32;  // problems per grouped launch

struct GemmGroup {
  const void* A[MAXG];
  const void* B[MAXG];
  void* C[MAXG];
};

// C = alpha * A(MxK) B(KxN) + beta * C for `groups` problems of identical
// shape and views, with element types ta (= tb) and tc.  Inputs F64 or F32
// run on the matching MFMA; BF16 inputs run on the bf16 MFMA with f32
// accumulation.  beta != 0 reads C.
hipError_t gemm(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K,
                double alpha, const View& va, const View& vb, double beta,
                const View& vc, const GemmGroup& g, int groups);

// float64 C = alpha A B + beta C with K split over slices that write partial
// products to `scratch` (needs slices * M * N * groups doubles; the slice
// count is chosen to fill the GPU and shrunk to fit the scratch), summed in
// a fixed order.  Falls back to gemm() when one slice suffices.
hipError_t gemm_splitk(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const View& va,
                       const View& vb, double beta, const View& vc, const GemmGroup& g, int groups,
                       double* scratch, int64_t scratch_elems);

// bf16 enlarged-corner contraction C(view) = A B with A = Y row-major M x K
// and B given transposed (Bt row-major N x K), f32 output through a two-level
// view; needs K % 8 == 0 and 16-byte aligned operands.
// Split-K GEMM for few columns (N <= 192) and plain strided operands:
// f32 -> f32/f64 and f64 -> f64.  `scratch` holds the K-chunk partials.
bool ts_gemm_supported(int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va, const View& vb,
                       const View& vc);
// c2, when given (ta = tc = F32 only): a second output, float64 through the
// same view, written by the same reduction as C
hipError_t ts_gemm(hipStream_t s, int ta, int tc, int64_t M, int64_t N, int64_t K, const View& va, const View& vb,
                   const View& vc, const GemmGroup& g, int groups, void* scratch, int64_t scratch_bytes,
                   const GemmGroup* c2 = nullptr);

// out[b][c][r] = in[b][r][c], float32, nb matrices R x C.
hipError_t transpose_batched(hipStream_t s, const float* in, int64_t nb, int64_t R, int64_t C, float* out);

bool corner_bf16_supported(int64_t M, int64_t N, int64_t K);

// Three-term bf16 split of float data for products with fp32-like accuracy:
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)); A-side rows [hi | hi | lo],
// B-side rows [hi | lo | hi], so that one bf16 product over 3K gives
// hi.hi + hi.lo + lo.hi.  `in` is read through the view (rows x K), out is
// row-major rows x 3K.  tin = F32 or F64.
hipError_t split3_bf16(hipStream_t s, int tin, const void* in, const View& vin, int64_t rows, int64_t K, bool a_side,
                       void* out);
// Several float64 splits of one shape (rows x K) in grouped launches.
struct Split3Job {
  const void* in;
  View view;
  bool a_side;
  void* out;
};
hipError_t split3_bf16_group(hipStream_t s, const Split3Job* jobs, int njobs, int64_t rows, int64_t K);
// The same for float32 `in` = nb matrices [R][C] (row-major, batch-major),
// transposed on the way: out row (b, c) = split of in[b][.][c], length 3R.
hipError_t split3_transpose_bf16(hipStream_t s, const float* in, int64_t nb, int64_t R, int64_t C, bool a_side,
                                 void* out);
// C (tout = F32 or BF16, through the view vc) = A Bt^T, A bf16 M x K and
// Bt bf16 N x K row-major (16-byte aligned, K % 8 == 0), fp32 accumulation.
// split_stride > 0 (tout = BF16): each result is stored as its A-side split
// hi, hi, lo at offsets 0, split_stride, 2 split_stride from its view place.
// b_packed (tout = F32, no split): Bt is in the packed fragment layout of
// corner_bf16_pack_b instead of row-major.
// a_packed (with b_packed): A is in the packed layout that
// corner_bf16_to_packed_a writes.
hipError_t corner_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const View& vc, const GemmGroup& g,
                       int groups, int tout = F32, int64_t split_stride = 0, bool b_packed = false,
                       bool a_packed = false);
// The enlarged corner's second product, taken transposed: the edge (A,
// rows (b, u)) times X (Bt, rows (g, l)), both bf16 row-major with K = chi,
// M = N = chi d2, d2 % 4 == 0, written as Y = [(g, b)][(l, u)] (chi^2 x d2^2,
// from element ((b, u), (g, l))) in bf16 in the packed A layout of the next
// product: [chi^2 / 16, padded to whole 256-row tiles][d2^2 / 32 rounded
// up][64 lanes][8], block (rb, kb) lane t holding Y[16 rb + t % 16][32 kb +
// 8 (t / 16) .. + 7]; the padding is not written.
int64_t corner_bf16_packed_a_elems(int64_t M, int64_t K);
hipError_t corner_bf16_to_packed_a(hipStream_t s, int64_t M, int64_t N, int64_t K, int64_t chi, int64_t d2,
                                   const GemmGroup& g, int groups);
// Packed fragment layout of a bf16 N x K row-major Bt for the corner kernel:
// [K / 32 (rounded up)][N / 16 (rounded up to whole 144-row tiles)][64 lanes][8],
// block (kb, rb) lane l holding Bt[16 rb + l % 16][32 kb + 8 (l / 16) .. + 7]
// (zeros past N and K).  Elements of the packed form, and the packing.
int64_t corner_bf16_packed_b_elems(int64_t N, int64_t K);
// Whether the moves use the packed form (default; environment variable
// CTM_CORNER_B=rowmajor, or CTM_CORNER_STAGING=registers, selects row-major).
bool corner_packed_b();
// The same for the intermediate Y (CTM_CORNER_A=rowmajor keeps it row-major).
bool corner_packed_a();
hipError_t corner_bf16_pack_b(hipStream_t s, const void* bT, int64_t N, int64_t K, void* out);

// out[perm-ordered] = in, generic permutation of an up-to-8-d row-major tensor
// with type conversion.  out dims are in_dims[perm[i]].
// Tile-shape autotuning of the generic GEMM.  While enabled on the calling
// thread, the first launch of each (types, M, N, K, operand order, groups)
// outside stream capture times every tile variant on the real operands
// (beta must be 0, so reruns are harmless; every variant sums K in the same
// order, so results are bitwise identical) and caches the fastest for the
// process.  Disabled, or while the stream is being captured, a cached choice
// or the 64 x 64 default is used.
void set_tuning(bool on);
int tuned_entries();

// ---------------------------------------------------------------------------
// Tile table: the launch variant of each kernel family per operand shape,
// written by the project's tuner and loaded from its file, or filled in
// process (the generic GEMM's tile timing above; the split counts of the
// tall-skinny and split-K products while table tuning is on).
//   TK_GEMM:   generic GEMM tile (0..3: 64x64, 32x32, 128x64, 128x128)
//   TK_TS:     tall-skinny split-K product, about 256 << v wave tasks
//              (v = 0..4, default 3)
//   TK_SPLITK: float64 split-K Gram products, about 128 << v work-groups
//              (v = 0..3, default 2)
// Variants of TK_TS / TK_SPLITK split K differently, so they change the
// summation order (results differ at the rounding level); a process that
// uses one table is deterministic.
// ---------------------------------------------------------------------------
//   TK_CORNER: the bf16 corner kernel with float32 output (ak, bk: operands
//              packed), rows per work-group (v = 0, 1, 2: 256, 192, 128;
//              bitwise-equal results)
enum TileKernel : int { TK_GEMM = 0, TK_TS = 1, TK_SPLITK = 2, TK_CORNER = 3 };
constexpr int TILE_KINDS = 4;
constexpr int TILE_VARIANTS[TILE_KINDS] = {4, 5, 4, 3};
struct TileKey {
  int kernel, ta, tc, ak, bk, groups;
  int64_t M, N, K;
  bool operator<(const TileKey& o) const;
};
// the stored variant of `k`, else dflt
int tile_lookup(const TileKey& k, int dflt);
void tile_set(const TileKey& k, int variant);
void tile_clear();
std::vector<std::pair<TileKey, int>> tile_entries();
// while on (process-wide), the first launch of each TK_TS / TK_SPLITK shape
// outside stream capture times every variant and stores the fastest
void tile_tuning(bool on);
bool tile_tuning_on();

// Grouped element copy / conversion: dst[j][i] = (tout) src[j][i], i < n[j].
constexpr int MAXJ = 32;
struct XferSet {
  const void* src[MAXJ];
  void* dst[MAXJ];
  int64_t n[MAXJ];
};
hipError_t convert_group(hipStream_t s, int tin, int tout, const XferSet& x, int njobs);

// Grouped Frobenius normalisation p[j] /= ||p[j]||, float64; `partial` holds
// MAXJ * 64 doubles of scratch.  Sums are taken in a fixed order.
struct NormSet {
  double* p[MAXJ];
  int64_t n[MAXJ];
};
hipError_t normalize_group(hipStream_t s, const NormSet& x, int njobs, double* partial);

hipError_t permute(hipStream_t s, int tin, const void* in, int tout, void* out,
                   int ndim, const int64_t* in_dims, const int* perm);

// Type conversion / copy of n elements.
hipError_t convert(hipStream_t s, int tin, const void* in, int tout, void* out, int64_t n);

// a[(u,u'),(l,l'),(d,d'),(r,r')] = sum_s A[s,u,l,d,r] * B[s,u',l',d',r'], written in
// four rotated layouts (see kernels.hip).
hipError_t double_layer(hipStream_t s, const double* A, const double* B, int d,
                        int D, double* out_rot[4], int64_t out_layout);

// Real form of the double layer of a complex ket Ac ([d][D^4] complex,
// interleaved; the bra is its conjugate) in the basis V-bar (up, left), V
// (down, right) of the doubled legs (see kernels.hip); sigma >= 0 gives the
// open double layer of physical slot sigma (physical pair in basis V).
hipError_t double_layer_cplx(hipStream_t s, const double* Ac, int d, int D, int sigma, double* out_rot[4]);

// Sum of squares of n float64 into *out (deterministic two-pass).
hipError_t sumsq(hipStream_t s, const double* x, int64_t n, double* partial, double* out);
// x *= 1/sqrt(*nrm2) (if > 0) for n float64.
hipError_t scale_by_rsqrt(hipStream_t s, double* x, int64_t n, const double* nrm2);
// Sets *flag = 1 if any of n float64 is not finite (flag must be zeroed first).
hipError_t nonfinite(hipStream_t s, const double* x, int64_t n, int* flag);

// Fill out with n standard normals from the counter-based generator
// (splitmix64 of seed + index, Box-Muller).
hipError_t randn(hipStream_t s, double* out, int64_t n, uint64_t seed);

// sum_{i < count} p[i * stride], added in order i = 0, 1, ... from zero, with
// eight loads in flight (a loop of dependent load-add steps would wait for
// memory once per term)
template <typename T>
__device__ __forceinline__ T ordered_sum(const T* __restrict__ p, int count, int64_t stride) {
  T acc = 0;
  for (int i0 = 0; i0 < count; i0 += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i0 + u < count ? p[(int64_t)(i0 + u) * stride] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < count) acc += v[u];
  }
  return acc;
}

}  // namespace ctmk
