/*
 * Simple update of the 2x2 checkerboard iPEPS (tensors A at x + y even, B at
 * x + y odd): imaginary-time evolution by first-order Suzuki-Trotter steps
 * e^{-dtau H_r} e^{-dtau H_l} e^{-dtau H_u} e^{-dtau H_d}, each factor a
 * product of two-body gates g = e^{-dtau h} on one type of link (Sec. II B),
 * applied with bond weights and truncated to the bond dimension D by an SVD
 * (the simple update that Sec. II D uses to start the ground-state search).
 *
 * Many instances of equal (d, D), each with its own bond Hamiltonians (a
 * scan over couplings), are updated in lock-step on one GPU.  Bond types and
 * their order in every buffer: 0 = h0 = A.r - B.l (H_r), 1 = h1 = B.r - A.l
 * (H_l), 2 = v0 = A.d - B.u (H_u), 3 = v1 = B.d - A.u (H_d); the first site
 * of a bond is the left (upper) one.  One Trotter step updates the bonds in
 * that order.  All arithmetic is float64 on the device.
 *
 * Tensors Gamma[s][u][l][d][r] (legs as in ctm.h) carry no weights; the
 * iPEPS of the state puts sqrt(lambda) of every bond on both of its legs
 * (ctm_su_peps).  A bond update multiplies the weights of the two tensors'
 * other legs in, factors each tensor as Q R, applies the gate to
 * R_X lambda R_Y, keeps the D largest singular values above 1e-12 times the
 * largest (normalised to unit Euclidean norm: the new weights), rebuilds both
 * tensors, divides the other legs' weights out (weights below 1e-12 times the
 * largest of their bond count as zero) and divides each tensor by its
 * Frobenius norm.  Limits: d^2 D <= 192, d^2 <= 192.
 */
#ifndef CTM_SU_H
#define CTM_SU_H

#include <stddef.h>
#include <stdint.h>

#include "ctm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_su_s* ctm_su;

/* Device workspace bytes for n_inst instances of physical dimension d and
 * bond dimension D. */
ctm_status ctm_su_workspace_size(int32_t n_inst, int32_t d, int32_t D, size_t* bytes);

/*
 * Creates the state.  T_dev: device float64 [n_inst][2][d][D][D][D][D]
 * (Gamma of A, then of B); lam_dev: device float64 [n_inst][4][D] (bond
 * weights in the bond order above); both are copied.  ws: device buffer of
 * at least ctm_su_workspace_size bytes, 256-byte aligned, owned by the
 * caller and used until ctm_su_destroy.  stream: HIP stream (NULL: default).
 */
ctm_status ctm_su_init(int32_t n_inst, int32_t d, int32_t D, const double* T_dev, const double* lam_dev,
                       void* ws, size_t ws_bytes, void* stream, ctm_su* out);

/*
 * Gates g = exp(-dtau h) of every bond of every instance from the bond
 * Hamiltonians h_dev: device float64 [n_inst][4][d^2][d^2], row-major on
 * (s_first, s_second) x (s_first', s_second') (h is symmetrised).  Computed
 * on the device from the eigendecomposition of h.  Syncs.
 */
ctm_status ctm_su_set_gates(ctm_su su, const double* h_dev, double dtau);

/*
 * Trotter steps until every instance's weights change by less than tol over
 * one step (read back every check_every steps) or max_steps.  steps_out
 * (may be NULL): steps done; change_out (host [n_inst], may be NULL): the
 * largest weight change over the last step of each instance.
 */
ctm_status ctm_su_evolve(ctm_su su, int32_t max_steps, double tol, int32_t check_every, int32_t* steps_out,
                         double* change_out);

/* Copies the tensors Gamma (device [n_inst][2][d D^4], may be NULL) and the
 * weights (device [n_inst][4][D], may be NULL) out.  Syncs. */
ctm_status ctm_su_state(ctm_su su, double* T_out_dev, double* lam_out_dev);

/* The iPEPS tensors of the state, Gamma times sqrt(lambda) on all four legs,
 * device [n_inst][2][d D^4] (A, then B), ready for ctm_init.  Syncs. */
ctm_status ctm_su_peps(ctm_su su, double* A_out_dev);

void ctm_su_destroy(ctm_su su);

#ifdef __cplusplus
}
#endif

#endif
