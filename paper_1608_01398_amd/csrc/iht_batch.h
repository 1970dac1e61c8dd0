// iht_batch.h -- batched gradient pass (many solves sharing one packed genotype matrix).
#pragma once
#include "iht_internal.h"

namespace iht {

// Per-solve view of its subject set: u, v [p] and mask [n_pad] of the stats handle, and |T|.
struct BatchSolve {
  const double* u;
  const double* v;
  const double* mask;
  int64_t nT;
};

int32_t batch_t_pad(int32_t T);
size_t batch_r8_bytes(const Layout& L, int32_t T);

// G[t * ldg + j] = (X_st^T R_t)_j for t < T, using R [T][n] (entries outside each solve's subject
// set ignored). Work areas: R8 (batch_r8_bytes), scale and rsum (T_pad doubles each); sv is a
// device array of T BatchSolve entries.
hipError_t launch_gradient_batch(const uint8_t* tiled, const Layout& L, const double* R, int32_t T, const BatchSolve* sv,
                                 int8_t* R8, double* scale, double* rsum, double* G, int64_t ldg, hipStream_t st);

}  // namespace iht
