// iht_solve.h -- device state of a set of IHT solves and the per-solve step launchers.
#pragma once
#include "iht_batch.h"
#include "iht_internal.h"

namespace iht {

// T solves sharing one genotype matrix; solve t works on its subject set sv[t], its trait
// Y + t * ldy and its model size ks[t] <= kmax. All arrays are device memory.
struct SolveSet {
  int32_t T, kmax;
  int64_t n, n_pad, p, p_pad;
  const BatchSolve* sv;  // [T]
  const int32_t* ks;     // [T]
  const double* Y;       // [T][ldy]
  int64_t ldy;
  Unpen U;
  double* beta;  // [T][p] dense coefficients (zero off the support)
  double* g;     // [T][p] gradient X_st^T r
  double* r;     // [T][n_pad] residual (zero outside the subject set)
  double* rc;    // [T][n_pad] residual centred over the subject set (gradient pass input)
  int64_t* S;    // [T][kmax] support, ascending
  int64_t* Sp;   // [T][kmax] proposed support
  double* betap;  // [T][kmax] proposal on Sp
  double* X;      // [T][2][kmax][n_pad] two caches of decoded support columns (FitState::xcur)
  double* bc;     // [T][kMaxUnpenalized] unpenalised coefficients
  double* bcp;    // [T][kMaxUnpenalized] their proposal
  double* gc;     // [T][kMaxUnpenalized] A_C^T r
  FitState* fs;   // [T]
  double* trace;  // [T][ldt] loss trace
  int64_t ldt;
  double* pw;     // [T][3][kmax + kMaxUnpenalized] polish vectors
  // subject-split steps: nb = solve_subject_blocks(n) workgroups per solve, each leaving its
  // partial sums in part (residual step) and pmu (step-size denominator)
  int32_t nb, pst;
  double* part;  // [T][nb][pst]
  double* pmu;   // [T][nb]
  double* ysum;  // [T][kYsumStride]: sum_T y, then sum_T A_c of the unpenalised columns
  int32_t family;  // IHT_GAUSSIAN or IHT_LOGISTIC (all solves of the set)
};

// Subjects per workgroup of the subject-split steps (one per lane).
constexpr int kSubjBlock = 64;
inline int32_t solve_subject_blocks(int64_t n) { return (int32_t)((n + kSubjBlock - 1) / kSubjBlock); }
// Partial sums per workgroup of the residual step: ||r||^2, sum rc, ||A Delta||^2, ||Delta||^2, the
// support-unchanged flag, then A_C^T r.
inline int32_t solve_partial_stride(int32_t nc) { return 5 + nc; }
constexpr int kYsumStride = 1 + kMaxUnpenalized;

// Where one solve's outputs go: support and beta_S [ld] (ld >= k), beta_cov [cz + intercept] or
// NULL, the loss trace [max_iter + 1] or NULL (kept in place).
struct OutRow {
  int64_t* support;
  double* beta_S;
  double* beta_cov;
  double* trace;
  int64_t ld;
};

// initial state of the admitted solves (admit[t] != 0, device [T]; every solve if NULL): beta = 0,
// control state, centring sums; marks them fresh
hipError_t solve_init(const SolveSet& Q, int32_t max_iter, const int32_t* admit, hipStream_t st);
// residual at beta = 0 (and its centred copy) of the solves with finite inputs
hipError_t solve_residual0(const SolveSet& Q, hipStream_t st);
// columns of S (which = 0, current cache) or S+ (which = 1, other cache) of the solves in `phase`
hipError_t solve_decode(const uint8_t* tiled, const SolveSet& Q, int32_t which, int32_t phase, hipStream_t st);
// backtracking test of the decoded proposal, and residual/loss/centred residual if it is taken
hipError_t solve_check_residual(const SolveSet& Q, int32_t phase, double c, int32_t max_backtrack, hipStream_t st);
// mode 1: commit accepted proposals, then the next step size of those still iterating;
// mode 0: first step size of the newly admitted solves
hipError_t solve_commit_mu(const SolveSet& Q, int32_t mode, double tol, int32_t max_iter, hipStream_t st);
hipError_t solve_shrink(const SolveSet& Q, double shrink, hipStream_t st);
// g on the accepted proposals' supports (phase go), exactly: each column of S+ (the proposal's cache)
// against the centred residual rq [T][n_pad] the gradient was taken at.
hipError_t solve_exact_support(const SolveSet& Q, const double* rq, hipStream_t st);
// FP64 refinement of the solves marked retire that converged
hipError_t solve_polish(const SolveSet& Q, double tol, int32_t max_steps, hipStream_t st);
// outputs of the solves marked retire into rows[t] (device [T])
hipError_t solve_output(const SolveSet& Q, const OutRow* rows, hipStream_t st);
// fresh (field 0) or retire (field 1) flag := value on the solves with flags[t] != 0 (all if NULL)
hipError_t solve_mark(const SolveSet& Q, const int32_t* flags, int32_t field, int32_t value, hipStream_t st);
// Held-out mean squared errors of q x r cross-validation solves (solve f * r + a: fold f held out,
// model size ks_path[a]; ks_solve[t] = its k), mse [r][q], and the k of least mean MSE. part holds
// ceil(n / 256) doubles per solve; fold_count [q] the size of each fold.
hipError_t cv_heldout_mse(const uint8_t* tiled, const Layout& L, const uint8_t* folds, int32_t q, int32_t r,
                          const BatchSolve* sv, const int32_t* ks_solve, const int32_t* ks_path, const int64_t* support,
                          const double* beta_S, int64_t ldk, const double* beta_cov, int64_t ldc, const Unpen& U,
                          const double* y, const int64_t* fold_count, double* part, double* mse, int32_t* k_best,
                          hipStream_t st);
// out [n] = X_st,S beta_S + A_C beta_cov for every subject, standardised with u, v; *err |= 1 if a
// support entry lies outside [0, p) (the entry is skipped). err must be cleared beforehand.
hipError_t launch_predict(const uint8_t* tiled, const Layout& L, const int64_t* support, const double* beta_S, int32_t k,
                          const double* u, const double* v, const Unpen& U, const double* beta_cov, double* out,
                          uint32_t* err, hipStream_t st);
// slots[0 .. *count) = the solves in `phase`, ascending.
hipError_t solve_slots(const FitState* fs, int32_t T, int32_t phase, int32_t* slots, int32_t* count, hipStream_t st);

}  // namespace iht
