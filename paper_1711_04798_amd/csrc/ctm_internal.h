// Internal hooks between the library's translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "ctm.h"

// The edges that bound a cut between columns `column - 1` and `column` of a
// context's environment, rows 0 .. Ly-1: the left edges T4 of column
// `column` and the right edges T2 of column `column - 1`, float64 at the live
// extent chi (legs [prev][(ket, bra)][next], clockwise around the site).
struct CtmEdgeRing {
  hipStream_t stream;
  int chi, D, Ly;
  bool dry;
  const double* T4[4];
  const double* T2[4];
};

ctm_status ctm_internal_edge_ring(ctm_ctx x, int inst, int column, CtmEdgeRing* out);

// Records `msg` as the thread's last error message and returns `s`.
ctm_status ctm_internal_fail(ctm_status s, const char* msg);
