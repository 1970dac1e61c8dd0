// iht_batch.h -- batched gradient pass (many solves sharing one packed genotype matrix).
#pragma once
#include "iht_internal.h"

namespace iht {

// Most subjects the matrix-core pass takes: its int32 sums (dosage <= 2 times a digit of
// magnitude <= 127, per subject) stay exact while 254 n <= 2^31 - 1.
constexpr int64_t kBatchMaxSubjects = 2147483647LL / 254;

int32_t batch_t_pad(int32_t T);
size_t batch_r8_bytes(const Layout& L, int32_t T);
// SNPs per block of the matrix-core pass the autotuner chose for this matrix and T (0: not tuned yet).
int32_t batch_tuned_snps(const Layout& L, int32_t T);

// G[t * ldg + j] = (X_st^T R_t)_j, with R_t = R + t * ldr (entries outside the solve's subject set
// ignored). Slot s < *count computes solve t = slots[s]; with slots == NULL and count == NULL the
// slots are the solves 0..T-1. Work areas: R8 (batch_r8_bytes), scale and rsum (T_pad doubles
// each); sv is a device array of T BatchSolve entries. A solve's result does not depend on which
// slot it occupies or on the other solves of the launch. With fs (device [T]), fs[t].gerr receives
// a bound on |G_tj - (X_st^T R_t)_j| valid for every SNP j (the quantisation error of the residual,
// summed against a standardised column: |T_t| s_t / 254^2, twice the rounding bound); with rq
// (device, row t at rq + t * ldr, n_pad entries), the centred residual the digits were taken from.
// With gmax (device, row t at gmax + t * batch_gmax_ld(L)), entry c of solve t's row receives the
// largest |G_tj| over the SNPs j in [128 c, 128 c + 128) (as the integer key of the FP64 bits).
hipError_t launch_gradient_batch(const uint8_t* tiled, const Layout& L, const double* R, int64_t ldr, int32_t T,
                                 const BatchSolve* sv, const int32_t* slots, const int32_t* count, int8_t* R8, double* scale,
                                 double* rsum, double* G, int64_t ldg, hipStream_t st, FitState* fs = nullptr,
                                 double* rq = nullptr, uint64_t* gmax = nullptr);
// Row length of the per-128-SNP maxima of launch_gradient_batch.
inline int64_t batch_gmax_ld(const Layout& L) { return (L.p_pad + kGmaxSnps - 1) / kGmaxSnps; }

}  // namespace iht
