// iht_internal.h -- device layout, work buffers and launchers shared by the library's sources.
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
#define IHT_PASS_THREADS 1024
#endif
#ifndef IHT_PASS_SNP_BARRIER
#define IHT_PASS_SNP_BARRIER 0
#endif
#ifndef IHT_PASS_MAX_NS
#define IHT_PASS_MAX_NS 4
#endif
constexpr int kPassThreads = IHT_PASS_THREADS;  // one pass workgroup per CU (128 KB of table in LDS)
constexpr int kPassMaxNS = IHT_PASS_MAX_NS;     // SNPs per lane, at most
#ifndef IHT_PASS_PIPE_DEPTH
#define IHT_PASS_PIPE_DEPTH 1
#endif
constexpr int kPassPipeDepth = IHT_PASS_PIPE_DEPTH;  // lookup units in flight ahead of the one summed
#ifndef IHT_PASS_UNIT
#define IHT_PASS_UNIT 4
#endif
constexpr int kSmallThreads = 1024;
constexpr int kMaxUnpenalized = 64;  // dense covariates + intercept
constexpr int kTopkBins0 = 8192;     // first-level histogram: key bits 62..50
constexpr int kTopkMaxK = 4096;
constexpr int kCertifyMaxK = 512;    // largest k of a certified (matrix-core) projection

struct Layout {
  int64_t n, p;
  int64_t ntiles;  // ceil(n / 32)
  int64_t n_pad;   // ntiles * 32
  int64_t p_pad;   // p rounded up to kSnpAlign
};

// Scalars and control state of one solve, resident on the device. Every per-solve kernel checks
// its phase against these flags, so a launch over many solves touches only the ones concerned.
struct FitState {
  double mu, omega, num, den;
  double loss, mean, Rsum;
  double dmax, bmax;
  double gerr;  // bound on |g~_j - g_j| of the last matrix-core gradient (0: exact gradient)
  int32_t same, accept, den_zero, conv;
  int32_t nonfinite, topk_error;
  int32_t go;       // proposal accepted (or support unchanged): residual, gradient and commit run
  int32_t active;   // still iterating
  int32_t need_bt;  // proposal rejected: halve mu and propose again
  int32_t nbt;      // halvings in this iteration
  int32_t iter;     // committed iterations
  int32_t status;   // IHT_OK / IHT_NOT_CONVERGED / IHT_STALLED / IHT_ENONFINITE
  int32_t xcur;     // which of the solve's two column caches holds the columns of S
  int32_t polish_steps;
  int32_t fresh;   // admitted, before its first proposal: the initial state is computed for it
  int32_t retire;  // finished and being written out (refinement and outputs run for it)
};

// Launch phases of the per-solve kernels: every solve; solves still iterating and not waiting for
// a halving (the next proposal: a solve whose proposal was rejected would only repeat it, since
// the step size changes only by a halving); those whose proposal needs a halving; those whose
// proposal was accepted; newly admitted solves with finite inputs (the initial residual, gradient
// and support); newly admitted solves still iterating (the first step size and proposal); solves
// being written out.
enum : int32_t {
  kPhaseAll = 0,
  kPhaseActive = 1,
  kPhaseBacktrack = 2,
  kPhaseGo = 3,
  kPhaseInit = 4,
  kPhaseFresh = 5,
  kPhaseRetire = 6
};

__device__ __forceinline__ bool fs_selected(const FitState* fs, int32_t phase) {
  if (phase == kPhaseAll) return true;
  if (phase == kPhaseInit) return fs->fresh != 0 && fs->nonfinite == 0;
  if (phase == kPhaseFresh) return fs->fresh != 0 && fs->active != 0;
  if (phase == kPhaseRetire) return fs->retire != 0;
  if (phase == kPhaseActive) return fs->active != 0 && fs->need_bt == 0;
  if (phase == kPhaseBacktrack) return fs->active != 0 && fs->need_bt != 0;
  return fs->active != 0 && fs->go != 0;
}

// Per-solve view of its subject set: u, v [p] and mask [n_pad] of the stats handle, and |T|.
struct BatchSolve {
  const double* u;
  const double* v;
  const double* mask;
  int64_t nT;
};

// Top-k work area of one row (counters are self-resetting: the last block of each kernel clears
// them). Rows are laid out kTopkRowWords apart in one small buffer; candidates `cap` apart.
struct TopkWork {
  uint32_t* hist;      // [kTopkBins0]
  uint32_t* counters;  // [8]: 0 hist ticket, 1 collect ticket, 2 n_sel, 3 n_cand, 4 filtered candidates,
                       // 5 saved list length, 6-7 approximate k-th key (certified selection)
  uint32_t* state;     // [8]: bucket, n_above, n_eq, error (bit 0 non-finite, bit 1 count mismatch)
  int32_t* sel;        // [kTopkMaxK]
  uint64_t* cand_key;  // [cap]
  int32_t* cand_idx;   // [cap]
};
constexpr int64_t kTopkRowWords = kTopkBins0 + 8 + 8 + kTopkMaxK;
constexpr int64_t kTopkErrorWord = kTopkBins0 + 8 + 3;  // state[3] of a row

// Many top-k problems in one launch (grid row t = problem t). Row t projects
//   w = g_t                     (beta == NULL), or
//   w = beta_t + mu_t g_t       (mu_t = fs[t].mu),
// keeping k_t = ks ? ks[t] : k0 entries; rows whose FitState is outside `phase` are skipped.
// With `prev` (k_t distinct indices per row, stride ldprev, e.g. the current support), the smallest
// |w| over them bounds the k_t-th largest from below, and one filtering pass keeps the entries at or
// above it as the candidates. With both beta and prev, prev must be the support of beta (beta zero
// elsewhere), ascending.
struct TopkJob {
  const double* beta;
  const double* g;
  int64_t ld;  // row stride of beta and g
  const FitState* fs;
  int32_t phase;
  int32_t k0;
  const int32_t* ks;
  int32_t kmax;  // >= every row's k
  int64_t* out;  // support rows (ascending), stride ldo
  int64_t ldo;
  double* vals;  // w at the support, stride ldo (may be NULL)
  uint32_t* small;  // row t at small + t * kTopkRowWords
  uint64_t* cand_key;
  int32_t* cand_idx;
  int64_t cap;  // candidate slots per row (>= p, >= 16384)
  const int64_t* prev;  // may be NULL
  int64_t ldprev;
  int32_t use_bound;  // set by launch_topk: the filter reads the bound k_topk_bound left in the row
  // Certified rows (certify != 0; needs fs, prev or a cold row, kmax <= 512): every g_j off the
  // exact support may be off by up to err = fs[t].gerr (times mu_t with beta), as after the
  // matrix-core pass. The filter keeps a margin of 2 err below its bound, and the entries of its list
  // within 2 err of the approximate k-th largest value get their exact FP64 gradient (the decoded
  // standardised column against rc) before the final selection, which is then the projection of
  // the exact w. Entries of g replaced that way hold the exact value afterwards.
  int32_t certify;
  int32_t prev_exact;    // set by launch_topk: the values at prev are exact (a warm row's support)
  const uint8_t* tiled;  // genotype layout [tile][p_pad][8 B]
  const BatchSolve* sv;  // [rows] subject set and standardisation of each row
  const double* rc;      // row t at rc + t * ldr: the centred residual the gradient was taken at
  int64_t ldr;
  int64_t n, p_pad, ntiles;
  // Optional (rows with beta): gmax + t * ldm holds the largest |g_j| of each 128 indices of row t as
  // the gradient pass left it (integer keys of the FP64 bits); the filter skips every 2048-entry
  // chunk whose largest |mu g| is below its threshold.
  const uint64_t* gmax;
  int64_t ldm;
};
constexpr int kGmaxSnps = 128;  // indices per entry of TopkJob::gmax

// ---- launchers (all asynchronous on `st`; return hipSuccess or the launch error) ----

hipError_t launch_retile(const uint8_t* raw, int64_t row_bytes, const Layout& L, uint8_t* tiled, hipStream_t st);

hipError_t launch_stats(const uint8_t* tiled, const Layout& L, const uint32_t* mask_bits, int64_t nT, double* u, double* v,
                        hipStream_t st);

// The subject set's FP64 mask [n_pad] from its bits [ntiles] (have_bits), or both for every subject.
hipError_t launch_subject_mask(const Layout& L, bool have_bits, uint32_t* bits, double* mask, hipStream_t st);

// g = X_st^T r over the subject set (mask, nT): a centring kernel (mean and R = sum of the centred
// residual into fs, centred residual into `work`), the pass kernel, and a finalize kernel when the
// subjects are split over workgroups. `work` holds gradient_work_bytes(L). With rc_ready the
// centred residual (and fs->Rsum) come from the caller and the centring kernel is skipped.
hipError_t launch_gradient(const uint8_t* tiled, const Layout& L, const double* r, const double* mask,
                           int64_t nT, const double* u, const double* v, FitState* fs, int precision, double* g,
                           double* work, const int32_t* gate, hipStream_t st, const double* rc_ready = nullptr);
size_t gradient_work_bytes(const Layout& L);

// Top-k of |w| (rows of TopkJob) over p entries for `rows` problems.
hipError_t launch_topk(const TopkJob& J, int64_t p, int32_t rows, hipStream_t st);
// Zero the error word and the filtered-candidate count of the rows of a top-k work area with
// flags[row] != 0 (rows 0 .. rows-1 if flags is NULL).
hipError_t launch_topk_clear_errors(uint32_t* small, int32_t rows, const int32_t* flags, hipStream_t st);

// Unpenalised columns: dense covariates and the intercept.
struct Unpen {
  const float* Z;  // [cz][n] column-major covariates
  int32_t cz;
  int32_t icpt;
};

hipError_t launch_fill(double* x, int64_t n, double val, hipStream_t st);
hipError_t launch_zero_u32(uint32_t* x, int64_t n, hipStream_t st);
hipError_t launch_scatter(const int64_t* idx, const double* vals, int32_t k, int64_t p, double* out, hipStream_t st);

}  // namespace iht
