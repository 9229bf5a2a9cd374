// Warm-start network of the CTM library: forward pass, loss and gradient,
// Adam, on gfx950 in float64.  The products of each pass run on the library's
// MFMA GEMM; bias, activation, loss, column sums and the optimiser are the
// elementwise kernels below.  Every reduction sums in a fixed order, so
// results are deterministic.
#include "ctm_mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.h"

ctm_status ctm_internal_fail(ctm_status s, const char* msg);

using namespace ctmk;

namespace {

#define MLP_HIP(x)                                                   \
  do {                                                               \
    hipError_t e_ = (x);                                             \
    if (e_ != hipSuccess) return ctm_internal_fail(CTM_E_HIP, #x);   \
  } while (0)

constexpr int kParts = 256;

struct Layout {
  int64_t W1, b1, W2, b2, W3, b3, total;
};

Layout layout(const ctm_mlp_shape& s) {
  Layout L;
  const int64_t i = s.n_in, h = s.n_hidden, o = s.n_out;
  L.W1 = 0;
  L.b1 = L.W1 + i * h;
  L.W2 = L.b1 + h;
  L.b2 = L.W2 + h * h;
  L.W3 = L.b2 + h;
  L.b3 = L.W3 + h * o;
  L.total = L.b3 + o;
  return L;
}

bool shape_ok(const ctm_mlp_shape* s) {
  return s && s->n_in >= 1 && s->n_in <= 64 && s->n_hidden >= 1 && s->n_hidden <= 1024 && s->n_out >= 1 &&
         s->n_out <= 4096;
}

struct Work {
  double *h1, *h2, *y, *dy, *d1, *d2, *part, *loss;
};

Work carve(const ctm_mlp_shape& s, int64_t B, void* ws, size_t* need) {
  Work w{};
  size_t off = 0;
  char* base = (char*)ws;
  auto take = [&](int64_t n) {
    off = (off + 255) & ~size_t(255);
    double* p = base ? (double*)(base + off) : nullptr;
    off += (size_t)n * 8;
    return p;
  };
  const int64_t h = s.n_hidden, o = s.n_out;
  w.h1 = take(B * h);
  w.h2 = take(B * h);
  w.y = take(B * o);
  w.dy = take(B * o);
  w.d1 = take(B * h);
  w.d2 = take(B * h);
  w.part = take(kParts);
  w.loss = take(1);
  if (need) *need = off + 256;
  return w;
}

hipError_t mm(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A, const View& va,
              const double* B, const View& vb, double* C) {
  GemmGroup g{};
  g.A[0] = A;
  g.B[0] = B;
  g.C[0] = C;
  return gemm(st, F64, F64, M, N, K, 1.0, va, vb, 0.0, rowmajor(N), g, 1);
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

// z[r][c] = act(z[r][c] + b[c]) with act = tanh (act != 0) or the identity,
// then 10^z if exp10 != 0
__global__ void bias_act_kernel(double* __restrict__ z, const double* __restrict__ b, int64_t rows, int cols,
                                int act, int to_exp10) {
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double v = z[e] + b[e % cols];
    if (act) v = tanh(v);
    if (to_exp10) v = exp10(v);
    z[e] = v;
  }
}

// r = y - t; dy = 2 r / (rows cols); part[block] = sum r^2 over the block's elements
__global__ void loss_kernel(const double* __restrict__ y, const double* __restrict__ t, int64_t n, double scale,
                            double* __restrict__ dy, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double r = y[e] - t[e];
    acc += r * r;
    dy[e] = 2.0 * r * scale;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const double* __restrict__ part, int np, double scale, double* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

// out[c] = sum_r a[r][c], rows in order
__global__ void colsum_kernel(const double* __restrict__ a, int64_t rows, int cols, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int64_t r = 0; r < rows; ++r) acc += a[r * cols + c];
  out[c] = acc;
}

// d[e] *= 1 - h[e]^2 (derivative of tanh through its output)
__global__ void dtanh_kernel(double* __restrict__ d, const double* __restrict__ h, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    d[e] *= 1.0 - h[e] * h[e];
}

__global__ void adam_kernel(int64_t n, double* __restrict__ p, const double* __restrict__ g, double* __restrict__ m,
                            double* __restrict__ v, double lr, double b1, double b2, double eps, double c1,
                            double c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double ge = g[e];
    double me = b1 * m[e] + (1.0 - b1) * ge;
    double ve = b2 * v[e] + (1.0 - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrt(ve / c2) + eps);
  }
}

__global__ void features_kernel(const double* __restrict__ theta, int64_t B, double* __restrict__ x) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < B; r += (int64_t)gridDim.x * blockDim.x) {
    double t1 = theta[2 * r], t2 = theta[2 * r + 1];
    x[3 * r] = cos(t1);
    x[3 * r + 1] = sin(t1);
    x[3 * r + 2] = t2;
  }
}

__global__ void targets_kernel(const double* __restrict__ s, int64_t n, double floor, double* __restrict__ t) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    t[e] = log10(fmax(s[e], floor));
}

// forward into w.h1, w.h2 and y
ctm_status forward_impl(const ctm_mlp_shape& s, const double* p, const double* x, int64_t B, double* y,
                        int exp10, const Work& w, hipStream_t st) {
  const Layout L = layout(s);
  const int64_t i = s.n_in, h = s.n_hidden, o = s.n_out;
  MLP_HIP(mm(st, B, h, i, x, rowmajor(i), p + L.W1, rowmajor(h), w.h1));
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(B * h)), dim3(256), 0, st, w.h1, p + L.b1, B, (int)h, 1, 0);
  MLP_HIP(mm(st, B, h, h, w.h1, rowmajor(h), p + L.W2, rowmajor(h), w.h2));
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(B * h)), dim3(256), 0, st, w.h2, p + L.b2, B, (int)h, 1, 0);
  MLP_HIP(mm(st, B, o, h, w.h2, rowmajor(h), p + L.W3, rowmajor(o), y));
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(B * o)), dim3(256), 0, st, y, p + L.b3, B, (int)o, 0, exp10);
  MLP_HIP(hipGetLastError());
  return CTM_OK;
}

ctm_status loss_grad_impl(const ctm_mlp_shape& s, const double* p, const double* x, const double* t, int64_t B,
                          double* loss, double* g, const Work& w, hipStream_t st) {
  const Layout L = layout(s);
  const int64_t i = s.n_in, h = s.n_hidden, o = s.n_out;
  ctm_status r = forward_impl(s, p, x, B, w.y, 0, w, st);
  if (r != CTM_OK) return r;
  const double scale = 1.0 / ((double)B * (double)o);
  hipLaunchKernelGGL(loss_kernel, dim3(kParts), dim3(256), 0, st, w.y, t, B * o, scale, w.dy, w.part);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, w.part, kParts, scale, loss);
  // output layer
  MLP_HIP(mm(st, h, o, B, w.h2, transposed(rowmajor(h)), w.dy, rowmajor(o), g + L.W3));
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((o + 255) / 256)), dim3(256), 0, st, w.dy, B, (int)o, g + L.b3);
  MLP_HIP(mm(st, B, h, o, w.dy, rowmajor(o), p + L.W3, transposed(rowmajor(o)), w.d2));
  hipLaunchKernelGGL(dtanh_kernel, dim3(blocks_for(B * h)), dim3(256), 0, st, w.d2, w.h2, B * h);
  // second layer
  MLP_HIP(mm(st, h, h, B, w.h1, transposed(rowmajor(h)), w.d2, rowmajor(h), g + L.W2));
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((h + 255) / 256)), dim3(256), 0, st, w.d2, B, (int)h, g + L.b2);
  MLP_HIP(mm(st, B, h, h, w.d2, rowmajor(h), p + L.W2, transposed(rowmajor(h)), w.d1));
  hipLaunchKernelGGL(dtanh_kernel, dim3(blocks_for(B * h)), dim3(256), 0, st, w.d1, w.h1, B * h);
  // first layer
  MLP_HIP(mm(st, i, h, B, x, transposed(rowmajor(i)), w.d1, rowmajor(h), g + L.W1));
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((h + 255) / 256)), dim3(256), 0, st, w.d1, B, (int)h, g + L.b1);
  MLP_HIP(hipGetLastError());
  return CTM_OK;
}

ctm_status adam_impl(int64_t n, double* p, const double* g, double* m, double* v, int step, double lr, double b1,
                     double b2, double eps, hipStream_t st) {
  const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  MLP_HIP(hipGetLastError());
  return CTM_OK;
}

ctm_status check_ws(const ctm_mlp_shape* s, int32_t B, void* ws, size_t bytes) {
  if (!shape_ok(s)) return ctm_internal_fail(CTM_E_INVALID, "mlp shape");
  if (B < 1) return ctm_internal_fail(CTM_E_INVALID, "batch must be >= 1");
  size_t need = 0;
  carve(*s, B, nullptr, &need);
  if (!ws || bytes < need) return ctm_internal_fail(CTM_E_NOMEM, "mlp workspace too small");
  if (((uintptr_t)ws) & 255) return ctm_internal_fail(CTM_E_INVALID, "workspace must be 256-byte aligned");
  return CTM_OK;
}

}  // namespace

extern "C" {

int64_t ctm_mlp_param_count(const ctm_mlp_shape* s) { return shape_ok(s) ? layout(*s).total : -1; }

ctm_status ctm_mlp_workspace_size(const ctm_mlp_shape* s, int32_t batch, size_t* bytes) {
  if (!shape_ok(s) || batch < 1 || !bytes) return ctm_internal_fail(CTM_E_INVALID, "mlp shape / batch");
  carve(*s, batch, nullptr, bytes);
  return CTM_OK;
}

ctm_status ctm_mlp_features(const double* theta, int32_t batch, double* x, void* stream) {
  if (!theta || !x || batch < 1) return ctm_internal_fail(CTM_E_INVALID, "features args");
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for(batch)), dim3(256), 0, (hipStream_t)stream, theta,
                     (int64_t)batch, x);
  MLP_HIP(hipGetLastError());
  return CTM_OK;
}

ctm_status ctm_mlp_targets(const double* spectra, int64_t count, double floor, double* t, void* stream) {
  if (!spectra || !t || count < 1 || !(floor > 0)) return ctm_internal_fail(CTM_E_INVALID, "targets args");
  hipLaunchKernelGGL(targets_kernel, dim3(blocks_for(count)), dim3(256), 0, (hipStream_t)stream, spectra, count,
                     floor, t);
  MLP_HIP(hipGetLastError());
  return CTM_OK;
}

ctm_status ctm_mlp_forward(const ctm_mlp_shape* s, const double* params, const double* x, int32_t batch, double* y,
                           int32_t exp10, void* ws, size_t ws_bytes, void* stream) {
  ctm_status r = check_ws(s, batch, ws, ws_bytes);
  if (r != CTM_OK) return r;
  if (!params || !x || !y) return ctm_internal_fail(CTM_E_INVALID, "null pointer");
  Work w = carve(*s, batch, ws, nullptr);
  return forward_impl(*s, params, x, batch, y, exp10 ? 1 : 0, w, (hipStream_t)stream);
}

ctm_status ctm_mlp_loss_grad(const ctm_mlp_shape* s, const double* params, const double* x, const double* t,
                             int32_t batch, double* loss, double* grad, void* ws, size_t ws_bytes, void* stream) {
  ctm_status r = check_ws(s, batch, ws, ws_bytes);
  if (r != CTM_OK) return r;
  if (!params || !x || !t || !loss || !grad) return ctm_internal_fail(CTM_E_INVALID, "null pointer");
  Work w = carve(*s, batch, ws, nullptr);
  return loss_grad_impl(*s, params, x, t, batch, loss, grad, w, (hipStream_t)stream);
}

ctm_status ctm_mlp_adam(int64_t n, double* params, const double* grad, double* m, double* v, int32_t step,
                        double lr, double beta1, double beta2, double eps, void* stream) {
  if (n < 1 || !params || !grad || !m || !v || step < 1) return ctm_internal_fail(CTM_E_INVALID, "adam args");
  return adam_impl(n, params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

ctm_status ctm_mlp_train(const ctm_mlp_shape* s, double* params, double* m, double* v, double* grad, int32_t step0,
                         const double* x, const double* t, int32_t batch, int32_t steps, double lr,
                         double* loss_hist, void* ws, size_t ws_bytes, void* stream) {
  ctm_status r = check_ws(s, batch, ws, ws_bytes);
  if (r != CTM_OK) return r;
  if (!params || !m || !v || !grad || !x || !t || steps < 0 || step0 < 0)
    return ctm_internal_fail(CTM_E_INVALID, "train args");
  Work w = carve(*s, batch, ws, nullptr);
  const int64_t n = layout(*s).total;
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < steps; ++i) {
    double* lp = loss_hist ? loss_hist + i : w.loss;
    r = loss_grad_impl(*s, params, x, t, batch, lp, grad, w, st);
    if (r != CTM_OK) return r;
    r = adam_impl(n, params, grad, m, v, step0 + i + 1, lr, 0.9, 0.999, 1e-8, st);
    if (r != CTM_OK) return r;
  }
  return CTM_OK;
}

}  // extern "C"
