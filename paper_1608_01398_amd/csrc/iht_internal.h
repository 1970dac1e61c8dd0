// iht_internal.h -- device layout, work buffers and launchers shared by the library's two sources.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace iht {

// Re-tiled genotype layout in HBM: subject tiles of 32 (8 packed bytes per SNP per tile), stored
// [tile][p_pad][8 B]. Inside the 8-byte segment of SNP j, byte b holds the original PLINK byte of
// 4-subject group (b + j) mod 8 of that tile, so that at every lookup step the lanes served
// together by the LDS read different groups of the table (conflict-free banks).
constexpr int kTileSubjects = 32;
constexpr int kSegBytes = 8;
constexpr int64_t kSnpAlign = 8192;  // p is padded to this (covers 1024 lanes x 8 SNPs per lane)
#ifndef IHT_PASS_THREADS
#define IHT_PASS_THREADS 512
#endif
#ifndef IHT_PASS_SNP_BARRIER
#define IHT_PASS_SNP_BARRIER 1
#endif
constexpr int kPassThreads = IHT_PASS_THREADS;  // one pass workgroup per CU (64 KB table + residual in LDS)
constexpr int kSmallThreads = 1024;
constexpr int kMaxUnpenalized = 64;  // dense covariates + intercept
constexpr int kTopkBins0 = 8192;     // first-level histogram: key bits 62..50
constexpr int kTopkMaxK = 4096;

struct Layout {
  int64_t n, p;
  int64_t ntiles;  // ceil(n / 32)
  int64_t n_pad;   // ntiles * 32
  int64_t p_pad;   // p rounded up to kSnpAlign
};

// Scalars of one solve, resident on the device; the host reads the flags once per decision.
struct FitState {
  double mu, omega, num, den;
  double loss, mean, Rsum;
  double dmax, bmax;
  int32_t same, accept, den_zero, conv;
  int32_t nonfinite, topk_error;
  int32_t go;  // proposal accepted (or support unchanged) and mu defined: the gated kernels run
  int32_t pad1;
};

// Top-k work area (counters are self-resetting: the last block of each kernel clears them).
struct TopkWork {
  uint32_t* hist;      // [kTopkBins0]
  uint32_t* counters;  // [8]: 0 hist ticket, 1 collect ticket, 2 n_sel, 3 n_cand
  uint32_t* state;     // [4]: bucket, n_above, n_eq, error
  int32_t* sel;        // [kTopkMaxK]
  uint64_t* cand_key;  // [p]
  int32_t* cand_idx;   // [p]
};

// ---- launchers (all asynchronous on `st`; return hipSuccess or the launch error) ----

hipError_t launch_retile(const uint8_t* raw, int64_t row_bytes, const Layout& L, uint8_t* tiled, hipStream_t st);

hipError_t launch_stats(const uint8_t* tiled, const Layout& L, const uint32_t* mask_bits, int64_t nT, double* u, double* v,
                        hipStream_t st);

// g = X_st^T r over the subject set (mask, nT): one pass kernel (plus a finalize kernel when the
// subjects are split over workgroups; `partial` then holds split * p_pad (D, M) pairs). The pass
// writes the subject-set mean of r and R = sum of the centred residual to fs.
hipError_t launch_gradient(const uint8_t* tiled, const Layout& L, const double* r, const double* mask, int64_t nT,
                           const double* u, const double* v, FitState* fs, int precision, double* g, double* partial,
                           const int32_t* gate, hipStream_t st);
size_t gradient_partial_bytes(const Layout& L);

hipError_t launch_decode_cols(const uint8_t* tiled, const Layout& L, const int64_t* cols, int32_t kc, const double* u,
                              const double* v, const double* mask, double* out, hipStream_t st);

// Top-k of |w_j| (w given) or of |beta_j + mu g_j|; writes support (ascending) and the w values there.
hipError_t launch_topk_w(const double* w, int64_t p, int32_t k, const TopkWork& tw, int64_t* support, double* vals,
                         hipStream_t st);
hipError_t launch_topk_step(const double* beta, const double* g, const double* mu, int64_t p, int32_t k, const TopkWork& tw,
                            int64_t* support, double* vals, hipStream_t st);
size_t topk_cand_capacity_bytes(int64_t p);

// ---- single-workgroup solve steps ----
struct Unpen {
  const float* Z;  // [cz][n] column-major covariates
  int32_t cz;
  int32_t icpt;
};

hipError_t launch_check_finite(const double* y, const float* Z, int64_t n, int32_t cz, const double* mask, FitState* fs,
                               hipStream_t st);
// r = mask*(y - X_cols b - Z bc), loss and covariate gradient gc; trace[idx] = loss.
// Gated launches (residual, gradient, commit) do nothing when *gate == 0; gate may be NULL.
hipError_t launch_residual(const double* y, const double* X, const double* bvals, int32_t kc, Unpen U, const double* bc,
                           const double* mask, const Layout& L, double* r, double* gc, double* trace, int32_t trace_idx,
                           FitState* fs, const int32_t* gate, hipStream_t st);
hipError_t launch_mu(const double* Xs, const int64_t* S, int32_t k, const double* g, Unpen U, const double* gc,
                     const double* mask, const Layout& L, FitState* fs, hipStream_t st);
hipError_t launch_bt_check(const int64_t* S, const double* Xs, const int64_t* Sp, const double* Xp, const double* betap_vals,
                           int32_t k, const double* beta, Unpen U, const double* bc, const double* gc, double* bcp,
                           double c, const double* mask, const Layout& L, FitState* fs, double* work, hipStream_t st);
hipError_t launch_shrink(FitState* fs, double shrink, hipStream_t st);
hipError_t launch_commit(int64_t* S, const int64_t* Sp, const double* betap_vals, int32_t k, double* beta, double* bc,
                         const double* bcp, int32_t nc, double tol, FitState* fs, const int32_t* gate, hipStream_t st);
hipError_t launch_output(const int64_t* S, int32_t k, const double* beta, const double* bc, int32_t nc, int64_t* support,
                         double* beta_S, double* beta_cov, hipStream_t st);
hipError_t launch_fill(double* x, int64_t n, double val, hipStream_t st);
hipError_t launch_zero_u32(uint32_t* x, int32_t n, hipStream_t st);
hipError_t launch_scatter(const int64_t* idx, const double* vals, int32_t k, double* out, hipStream_t st);

}  // namespace iht
