/*
 * ctm_mlp.h -- learned warm start of the CTM environment (gfx950).
 *
 * Not part of the paper's method: a form beyond it.  A three-layer perceptron
 * maps the parameters theta = (t1, t2) of a family of PEPS tensors to the
 * log10 of the normalised singular values of the four corners of the
 * converged environment; the predicted spectra initialise diagonal corners
 * (ctm_init with CTM_INIT_DIAG).  Plain CTM from the trivial start generates
 * the training targets and remains the fallback.
 *
 * Definitions (all float64, row-major):
 *   features   x = (cos t1, sin t1, t2)                       [B][3]
 *   layers     h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3
 *   parameters one flat vector W1[n_in][n_hidden], b1[n_hidden],
 *              W2[n_hidden][n_hidden], b2, W3[n_hidden][n_out], b3[n_out]
 *   targets    t = log10(max(s, floor)) of each normalised corner spectrum s
 *   loss       mean over batch and outputs of (y - t)^2
 *   optimiser  Adam (Kingma & Ba 2015) with bias correction, full batch
 *
 * Every pointer argument except *_host is device memory owned by the caller;
 * the workspace must hold ctm_mlp_workspace_size() bytes and be 256-byte
 * aligned.  Work is enqueued on `stream` (hipStream_t, NULL = default) and is
 * asynchronous unless stated.  Statuses and ctm_last_error() as in ctm.h.
 */
#ifndef CTM_MLP_H
#define CTM_MLP_H

#include "ctm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_in;      /* 3 for the (cos t1, sin t1, t2) features            */
  int32_t n_hidden;  /* width of both hidden layers (1..1024)              */
  int32_t n_out;     /* 4 * chi                                            */
} ctm_mlp_shape;

/* Number of parameters (length of the flat parameter vector). */
int64_t ctm_mlp_param_count(const ctm_mlp_shape* shape);

/* Workspace bytes for batches of up to `batch` rows. */
ctm_status ctm_mlp_workspace_size(const ctm_mlp_shape* shape, int32_t batch, size_t* bytes);

/* theta [batch][2] -> x [batch][3] = (cos t1, sin t1, t2). */
ctm_status ctm_mlp_features(const double* theta, int32_t batch, double* x, void* stream);

/* spectra [count] -> targets [count], t = log10(max(s, floor)), floor > 0. */
ctm_status ctm_mlp_targets(const double* spectra, int64_t count, double floor, double* t, void* stream);

/* y [batch][n_out] = network(x); with exp10 != 0 the outputs are 10^y, the
 * predicted spectra in the layout of ctm_init's spectrum_host. */
ctm_status ctm_mlp_forward(const ctm_mlp_shape* shape, const double* params, const double* x,
                           int32_t batch, double* y, int32_t exp10, void* ws, size_t ws_bytes,
                           void* stream);

/* loss (device scalar) and its gradient grad [param_count] at params. */
ctm_status ctm_mlp_loss_grad(const ctm_mlp_shape* shape, const double* params, const double* x,
                             const double* t, int32_t batch, double* loss, double* grad, void* ws,
                             size_t ws_bytes, void* stream);

/* One Adam step (step counts from 1) on n parameters with moments m, v. */
ctm_status ctm_mlp_adam(int64_t n, double* params, const double* grad, double* m, double* v,
                        int32_t step, double lr, double beta1, double beta2, double eps, void* stream);

/* `steps` full-batch Adam steps numbered step0 + 1 .. step0 + steps (beta1 =
 * 0.9, beta2 = 0.999, eps = 1e-8); loss_hist [steps] (device, may be NULL)
 * receives the loss before each step.  grad: device scratch [param_count]. */
ctm_status ctm_mlp_train(const ctm_mlp_shape* shape, double* params, double* m, double* v,
                         double* grad, int32_t step0, const double* x, const double* t,
                         int32_t batch, int32_t steps, double lr, double* loss_hist, void* ws,
                         size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CTM_MLP_H */
