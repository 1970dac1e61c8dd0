// iht_solve.hip -- per-solve step kernels of the IHT loop (one workgroup per solve).
//
// Every kernel here works on solve t = blockIdx.x (or blockIdx.z) of a SolveSet; a single fit is
// the case T = 1. The update is eq. (ihta) of Methods with the normalised step and the omega rule
// of "IHT step sizes"; the loss is eq. (leastsquaresloss). The per-solve control state (active,
// committed iterations, halvings, status) lives in FitState, so one launch serves solves that are
// at different points of their iteration.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "iht.h"
#include "iht_solve.h"

namespace iht {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kSubjUnroll = 4;  // subjects per thread in flight
constexpr int kColBatch = 4;    // support columns loaded together

__device__ double ssum(double x, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    sh[32] = t;
  }
  __syncthreads();
  return sh[32];
}

__device__ double smax(double x, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
    sh[32] = t;
  }
  __syncthreads();
  return sh[32];
}

// Solve t's slice of the set.
struct View {
  int t, k, nc;
  const double* mask;
  const double* y;
  double* beta;
  double* g;
  double* r;
  double* rc;  // centred residual (gradient pass input)
  int64_t* S;
  int64_t* Sp;
  double* betap;
  double* Xs;  // columns of S
  double* Xp;  // columns of S+
  double* bc;
  double* bcp;
  double* gc;
  FitState* fs;
  double* trace;
  int32_t* uidx;
  double* udel;
  double* pw;
};

__device__ __forceinline__ View view(const SolveSet& Q, int t) {
  View V;
  V.t = t;
  V.k = Q.ks[t];
  V.nc = Q.U.cz + Q.U.icpt;
  V.mask = Q.sv[t].mask;
  V.y = Q.Y + (int64_t)t * Q.ldy;
  V.beta = Q.beta + (int64_t)t * Q.p;
  V.g = Q.g + (int64_t)t * Q.p;
  V.r = Q.r + (int64_t)t * Q.n_pad;
  V.rc = Q.rc + (int64_t)t * Q.n_pad;
  V.S = Q.S + (int64_t)t * Q.kmax;
  V.Sp = Q.Sp + (int64_t)t * Q.kmax;
  V.betap = Q.betap + (int64_t)t * Q.kmax;
  V.fs = Q.fs + t;
  const int cur = V.fs->xcur;
  V.Xs = Q.X + ((int64_t)t * 2 + cur) * Q.kmax * Q.n_pad;
  V.Xp = Q.X + ((int64_t)t * 2 + (1 - cur)) * Q.kmax * Q.n_pad;
  V.bc = Q.bc + (int64_t)t * kMaxUnpenalized;
  V.bcp = Q.bcp + (int64_t)t * kMaxUnpenalized;
  V.gc = Q.gc + (int64_t)t * kMaxUnpenalized;
  V.trace = Q.trace + (int64_t)t * Q.ldt;
  V.uidx = Q.uidx + (int64_t)t * 2 * Q.kmax;
  V.udel = Q.udel + (int64_t)t * 2 * Q.kmax;
  V.pw = Q.pw + (int64_t)t * 3 * (Q.kmax + kMaxUnpenalized);
  return V;
}

// Unpenalised column c at subject i: covariate c, or the intercept's 1.
__device__ __forceinline__ double ucol(const Unpen& U, int64_t n, int c, int64_t i) {
  return c < U.cz ? (double)U.Z[(int64_t)c * n + i] : 1.0;
}

// Subjects i0 + w * kThreads (w < kSubjUnroll): clamped index and "inside the subject set".
__device__ __forceinline__ void subj_block(int64_t i0, int64_t n, const double* mask, int64_t (&ii)[kSubjUnroll],
                                           bool (&ok)[kSubjUnroll]) {
#pragma unroll
  for (int w = 0; w < kSubjUnroll; ++w) {
    const int64_t i = i0 + (int64_t)w * kThreads;
    ok[w] = i < n && mask[i < n ? i : 0] != 0.0;
    ii[w] = i < n ? i : 0;
  }
}

// sm[w] = sum_q X[q][ii[w]] b[q] + sum_c A_c(ii[w]) bcv[c]: SNP columns in support order, then the
// covariates, then the intercept.
__device__ __forceinline__ void apply_cols(const double* X, int64_t n_pad, const double* b, int kc, const Unpen& U,
                                           int64_t n, const double* bcv, const int64_t (&ii)[kSubjUnroll],
                                           double (&sm)[kSubjUnroll]) {
#pragma unroll
  for (int w = 0; w < kSubjUnroll; ++w) sm[w] = 0.0;
  // columns in groups of kColBatch: all their loads are issued before the (in-order) sums
  int q = 0;
  for (; q + kColBatch <= kc; q += kColBatch) {
    double xv[kColBatch][kSubjUnroll];
#pragma unroll
    for (int a = 0; a < kColBatch; ++a)
#pragma unroll
      for (int w = 0; w < kSubjUnroll; ++w) xv[a][w] = X[(int64_t)(q + a) * n_pad + ii[w]];
#pragma unroll
    for (int a = 0; a < kColBatch; ++a) {
      const double bq = b[q + a];
#pragma unroll
      for (int w = 0; w < kSubjUnroll; ++w) sm[w] += xv[a][w] * bq;
    }
  }
  for (; q < kc; ++q) {
    const double bq = b[q];
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w) sm[w] += X[(int64_t)q * n_pad + ii[w]] * bq;
  }
  for (int c = 0; c < U.cz; ++c) {
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w) sm[w] += (double)U.Z[(int64_t)c * n + ii[w]] * bcv[c];
  }
  if (U.icpt) {
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w) sm[w] += 1.0 * bcv[U.cz];
  }
}

// ---------------------------------------------------------------------------- initial state

// beta = 0 (eq. ihta starts from the zero vector), non-finite y or covariates inside the subject
// set flagged, mu = 1 so that the first projection of beta + mu g is the top-k of |g|.
__global__ __launch_bounds__(256) void k_zero_beta(SolveSet Q) {
  const int64_t total = (int64_t)Q.T * Q.p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) Q.beta[e] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_init(SolveSet Q, int32_t max_iter) {
  const int t = blockIdx.x;
  const double* mask = Q.sv[t].mask;
  const double* y = Q.Y + (int64_t)t * Q.ldy;
  for (int c = threadIdx.x; c < kMaxUnpenalized; c += kThreads) {
    Q.bc[(int64_t)t * kMaxUnpenalized + c] = 0.0;
    Q.bcp[(int64_t)t * kMaxUnpenalized + c] = 0.0;
    Q.gc[(int64_t)t * kMaxUnpenalized + c] = 0.0;
  }
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int b = 0;
  for (int64_t i = threadIdx.x; i < Q.n; i += kThreads) {
    if (mask[i] == 0.0) continue;
    if (!isfinite(y[i])) b = 1;
    for (int c = 0; c < Q.U.cz; ++c)
      if (!isfinite(Q.U.Z[(int64_t)c * Q.n + i])) b = 1;
  }
  if (b) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    FitState z{};
    z.mu = 1.0;
    z.nonfinite = bad;
    z.active = (bad || max_iter <= 0) ? 0 : 1;
    z.status = bad ? IHT_ENONFINITE : IHT_NOT_CONVERGED;
    Q.fs[t] = z;
  }
}

// ---------------------------------------------------------------------------- block-level steps
// Each step below is executed by the whole workgroup of one solve; `vec` is a block-shared vector of
// kTopkMaxK doubles, `sh` a small reduction scratch. Steps end with the block synchronised.

// Support columns of S (which = 0, into the current cache) or of S+ (which = 1, into the other
// cache): X[q][i] = v_j (x_ij - u_j) for j = that column, 0 for a missing entry and outside the
// subject set. Only the support's columns are ever decoded (Methods, "Bandwidth optimization of
// IHT").
__device__ __forceinline__ double decode_entry(const uint8_t* __restrict__ tiled, int64_t p_pad, int64_t j, int64_t i,
                                               const double* u, const double* v, const double* mask) {
  const int64_t tile = i / kTileSubjects;
  const int grp = (int)((i % kTileSubjects) >> 2);
  const int b = (grp - (int)(j & (kSegBytes - 1))) & (kSegBytes - 1);
  const uint8_t byte = tiled[(tile * p_pad + j) * kSegBytes + b];
  const int code = (byte >> (2 * (i & 3))) & 3;
  if (mask[i] == 0.0 || code == 1) return 0.0;
  const double d = (code == 0) ? 0.0 : (double)(code - 1);
  return v[j] * (d - u[j]);
}

// Wide decode (grid: subjects / 256 x kmax x T) of the columns of S (which = 0, into the current
// cache) or of S+ (which = 1, into the other cache) of the solves in `phase`.
__global__ __launch_bounds__(256) void k_decode(const uint8_t* __restrict__ tiled, SolveSet Q, int32_t which, int32_t phase) {
  const int t = blockIdx.z;
  const FitState* fs = Q.fs + t;
  if (!fs_selected(fs, phase)) return;
  const int q = blockIdx.y;
  if (q >= Q.ks[t]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q.n_pad) return;
  const int64_t* cols = (which ? Q.Sp : Q.S) + (int64_t)t * Q.kmax;
  const int cache = which ? 1 - fs->xcur : fs->xcur;
  double* out = Q.X + (((int64_t)t * 2 + cache) * Q.kmax + q) * Q.n_pad;
  out[i] = decode_entry(tiled, Q.p_pad, cols[q], i, Q.sv[t].u, Q.sv[t].v, Q.sv[t].mask);
}

// r = mask (y - A_{S+ u C} beta+) and loss = 1/2 ||r||^2 (eq. leastsquaresloss) into the trace
// (entry iter + 1), or at beta = 0 into entry 0 when `initial`; gc = A_C^T r. Then the residual
// centred over the subject set for the gradient pass: rc = r - mean on T, 0 elsewhere (up to
// n_pad), R = sum rc into fs (X_st^T 1_T = 0: centring leaves the gradient unchanged).
__device__ void blk_residual(const SolveSet& Q, const View& V, int initial, double* vec, double* sh) {
  __shared__ double bcl[kMaxUnpenalized];
  const int kc = initial ? 0 : V.k;
  for (int q = threadIdx.x; q < kc; q += kThreads) vec[q] = V.betap[q];
  for (int q = threadIdx.x; q < V.nc; q += kThreads) bcl[q] = initial ? 0.0 : V.bcp[q];
  __syncthreads();
  double rr = 0.0, rs = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < Q.n; i0 += (int64_t)kSubjUnroll * kThreads) {
    int64_t ii[kSubjUnroll];
    bool ok[kSubjUnroll];
    double sm[kSubjUnroll];
    subj_block(i0, Q.n, V.mask, ii, ok);
    apply_cols(V.Xp, Q.n_pad, vec, kc, Q.U, Q.n, bcl, ii, sm);
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w) {
      const int64_t i = i0 + (int64_t)w * kThreads;
      if (i < Q.n) {
        const double ri = ok[w] ? V.y[i] - sm[w] : 0.0;
        V.r[i] = ri;
        rr += ri * ri;
        rs += ri;  // zero outside the subject set
      }
    }
  }
  const double loss = 0.5 * ssum(rr, sh);
  const double mean = ssum(rs, sh) / (double)Q.sv[V.t].nT;
  for (int c = 0; c < V.nc; ++c) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < Q.n; i += kThreads) s += (V.mask[i] != 0.0) ? ucol(Q.U, Q.n, c, i) * V.r[i] : 0.0;
    s = ssum(s, sh);
    if (threadIdx.x == 0) V.gc[c] = s;
  }
  double R = 0.0;
  for (int64_t i = threadIdx.x; i < Q.n_pad; i += kThreads) {
    const double x = (i < Q.n && V.mask[i] != 0.0) ? V.r[i] - mean : 0.0;
    V.rc[i] = x;
    R += x;
  }
  R = ssum(R, sh);
  if (threadIdx.x == 0) {
    V.trace[initial ? 0 : V.fs->iter + 1] = loss;
    V.fs->loss = loss;
    V.fs->mean = mean;
    V.fs->Rsum = R;
  }
  __syncthreads();
}

// mu = ||g_{S u C}||^2 / ||A_{S u C} g_{S u C}||^2 ("IHT step sizes", normalised form). A zero
// denominator means the gradient vanishes on S u C: nothing can move, the solve ends there
// (converged).
__device__ void blk_mu(const SolveSet& Q, const View& V, double* vec, double* sh) {
  __shared__ double gcl[kMaxUnpenalized];
  for (int q = threadIdx.x; q < V.k; q += kThreads) vec[q] = V.g[V.S[q]];
  for (int q = threadIdx.x; q < V.nc; q += kThreads) gcl[q] = V.gc[q];
  __syncthreads();
  double num = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < V.k; ++q) num += vec[q] * vec[q];
    for (int q = 0; q < V.nc; ++q) num += gcl[q] * gcl[q];
  }
  double dd = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < Q.n; i0 += (int64_t)kSubjUnroll * kThreads) {
    int64_t ii[kSubjUnroll];
    bool ok[kSubjUnroll];
    double sm[kSubjUnroll];
    subj_block(i0, Q.n, V.mask, ii, ok);
    apply_cols(V.Xs, Q.n_pad, vec, V.k, Q.U, Q.n, gcl, ii, sm);
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w)
      if (ok[w]) dd += sm[w] * sm[w];
  }
  const double den = ssum(dd, sh);
  if (threadIdx.x == 0) {
    FitState* fs = V.fs;
    fs->num = num;
    fs->den = den;
    fs->nbt = 0;
    fs->go = 0;
    fs->need_bt = 0;
    if (den == 0.0) {
      fs->den_zero = 1;
      fs->mu = 0.0;
      fs->active = 0;
      fs->status = IHT_OK;
    } else {
      fs->den_zero = 0;
      fs->mu = num / den;
    }
  }
  __syncthreads();
}

// Support comparison, unpenalised proposal bcp = bc + mu gc and, when the support moved,
// omega = (1-c)||Delta||^2 / ||A Delta||^2 over S u S+ u C. The proposal is taken when the support is
// unchanged or mu < omega; otherwise the solve needs a halving, and with the budget spent it stops
// (stalled) keeping beta. Returns the accept flag (block-uniform).
__device__ int blk_bt_check(const SolveSet& Q, const View& V, double c, int32_t max_backtrack, double* sh) {
  __shared__ double dcl[kMaxUnpenalized];
  __shared__ int same_s, nu_s, acc_s;
  __shared__ double dd_s;
  const int k = V.k;
  const double mu = V.fs->mu;
  if (threadIdx.x == 0) {
    int same = 1;
    for (int q = 0; q < k; ++q)
      if (V.S[q] != V.Sp[q]) same = 0;
    same_s = same;
    double dd = 0.0;
    int nu = 0;
    if (!same) {
      // merge S and S+ ascending; uidx: q (column q of the S cache) or -(q+1) (column q of S+)
      int a = 0, b = 0;
      while (a < k || b < k) {
        if (b >= k || (a < k && V.S[a] < V.Sp[b])) {
          const double d = 0.0 - V.beta[V.S[a]];
          V.uidx[nu] = a;
          V.udel[nu++] = d;
          dd += d * d;
          ++a;
        } else if (a >= k || V.Sp[b] < V.S[a]) {
          const double d = V.betap[b] - 0.0;
          V.uidx[nu] = -(b + 1);
          V.udel[nu++] = d;
          dd += d * d;
          ++b;
        } else {
          const double d = V.betap[b] - V.beta[V.S[a]];
          V.uidx[nu] = -(b + 1);
          V.udel[nu++] = d;
          dd += d * d;
          ++a;
          ++b;
        }
      }
    }
    for (int q = 0; q < V.nc; ++q) {
      const double np = V.bc[q] + mu * V.gc[q];
      V.bcp[q] = np;
      const double d = np - V.bc[q];
      dcl[q] = d;
      dd += d * d;
    }
    nu_s = nu;
    dd_s = dd;
  }
  __syncthreads();
  double omega = 0.0;
  if (!same_s) {
    const int nu = nu_s;
    double sa = 0.0;
    for (int64_t i0 = threadIdx.x; i0 < Q.n; i0 += (int64_t)kSubjUnroll * kThreads) {
      int64_t ii[kSubjUnroll];
      bool ok[kSubjUnroll];
      double sm[kSubjUnroll];
      subj_block(i0, Q.n, V.mask, ii, ok);
#pragma unroll
      for (int w = 0; w < kSubjUnroll; ++w) sm[w] = 0.0;
      for (int q = 0; q < nu; ++q) {
        const int src = V.uidx[q];
        const double* col = (src >= 0) ? V.Xs + (int64_t)src * Q.n_pad : V.Xp + (int64_t)(-src - 1) * Q.n_pad;
        const double dq = V.udel[q];
#pragma unroll
        for (int w = 0; w < kSubjUnroll; ++w) sm[w] += col[ii[w]] * dq;
      }
      for (int cc = 0; cc < Q.U.cz; ++cc) {
#pragma unroll
        for (int w = 0; w < kSubjUnroll; ++w) sm[w] += (double)Q.U.Z[(int64_t)cc * Q.n + ii[w]] * dcl[cc];
      }
      if (Q.U.icpt) {
#pragma unroll
        for (int w = 0; w < kSubjUnroll; ++w) sm[w] += 1.0 * dcl[Q.U.cz];
      }
#pragma unroll
      for (int w = 0; w < kSubjUnroll; ++w)
        if (ok[w]) sa += sm[w] * sm[w];
    }
    const double dA = ssum(sa, sh);
    omega = (1.0 - c) * dd_s / dA;
  }
  if (threadIdx.x == 0) {
    FitState* fs = V.fs;
    const int accept = same_s ? 1 : (mu < omega ? 1 : 0);
    fs->same = same_s;
    fs->omega = omega;
    fs->accept = accept;
    fs->go = accept;
    fs->need_bt = accept ? 0 : 1;
    if (!accept && fs->nbt >= max_backtrack) {
      fs->need_bt = 0;
      fs->active = 0;
      fs->status = IHT_STALLED;
    }
    acc_s = accept;
  }
  __syncthreads();
  return acc_s;
}

// Convergence (S+ = S and ||beta+ - beta||_inf <= tol max(1, ||beta+||_inf); with S+ = S the union of
// the supports is S itself, so the norms run over S+ and C), then beta <- beta+, S <- S+, the column
// caches trade roles and one more iteration is counted. Returns 1 if the solve is still iterating.
__device__ int blk_commit(const SolveSet& Q, const View& V, double tol, int32_t max_iter, double* sh) {
  __shared__ int same_s, act_s;
  if (threadIdx.x == 0) same_s = 1;
  __syncthreads();
  double dmax = 0.0, bmax = 0.0;
  for (int q = threadIdx.x; q < V.k; q += kThreads) {
    if (V.S[q] != V.Sp[q]) atomicAnd(&same_s, 0);
    dmax = fmax(dmax, fabs(V.betap[q] - V.beta[V.Sp[q]]));
    bmax = fmax(bmax, fabs(V.betap[q]));
  }
  for (int q = threadIdx.x; q < V.nc; q += kThreads) {
    dmax = fmax(dmax, fabs(V.bcp[q] - V.bc[q]));
    bmax = fmax(bmax, fabs(V.bcp[q]));
  }
  dmax = smax(dmax, sh);
  bmax = smax(bmax, sh);
  const int same = same_s;
  const int conv = same && dmax <= tol * fmax(1.0, bmax);
  __syncthreads();
  for (int q = threadIdx.x; q < V.k; q += kThreads) V.beta[V.S[q]] = 0.0;
  __syncthreads();
  for (int q = threadIdx.x; q < V.k; q += kThreads) {
    V.beta[V.Sp[q]] = V.betap[q];
    V.S[q] = V.Sp[q];
  }
  for (int q = threadIdx.x; q < V.nc; q += kThreads) V.bc[q] = V.bcp[q];
  if (threadIdx.x == 0) {
    FitState* fs = V.fs;
    fs->conv = conv;
    fs->same = same;
    fs->dmax = dmax;
    fs->bmax = bmax;
    fs->iter += 1;
    fs->go = 0;
    fs->xcur ^= 1;  // the proposal's cache now holds the columns of S
    if (conv) {
      fs->active = 0;
      fs->status = IHT_OK;
    } else if (fs->iter >= max_iter) {
      fs->active = 0;
      fs->status = IHT_NOT_CONVERGED;
    }
    act_s = fs->active;
  }
  __syncthreads();
  return act_s;
}

// ---------------------------------------------------------------------------- step kernels

// Initial residual (at beta = 0) of the solves with finite inputs.
__global__ __launch_bounds__(kThreads) void k_residual0(SolveSet Q) {
  if (!fs_selected(Q.fs + blockIdx.x, kPhaseInit)) return;
  __shared__ double sh[40];
  __shared__ double vec[kTopkMaxK];
  const View V = view(Q, blockIdx.x);
  blk_residual(Q, V, 1, vec, sh);
}

// A proposal (S+, beta+ from the projection, its columns decoded) of the solves in `phase`: the
// backtracking test and, when the proposal is taken, its residual, loss and centred residual for
// the gradient pass.
__global__ __launch_bounds__(kThreads) void k_check_residual(SolveSet Q, int32_t phase, double c, int32_t max_backtrack) {
  if (!fs_selected(Q.fs + blockIdx.x, phase)) return;
  __shared__ double sh[40];
  __shared__ double vec[kTopkMaxK];
  const View V = view(Q, blockIdx.x);
  if (blk_bt_check(Q, V, c, max_backtrack, sh)) blk_residual(Q, V, 0, vec, sh);
}

// Commit of the accepted proposals (mode 1), then the step size of the next iteration for the
// solves that committed and still iterate; mode 0: step size of every active solve (first
// iteration).
__global__ __launch_bounds__(kThreads) void k_commit_mu(SolveSet Q, int32_t mode, double tol, int32_t max_iter) {
  __shared__ double sh[40];
  __shared__ double vec[kTopkMaxK];
  const FitState* fs = Q.fs + blockIdx.x;
  if (mode == 0) {
    if (!fs_selected(fs, kPhaseActive)) return;
    const View V = view(Q, blockIdx.x);
    blk_mu(Q, V, vec, sh);
    return;
  }
  if (!fs_selected(fs, kPhaseGo)) return;
  const View V = view(Q, blockIdx.x);
  if (blk_commit(Q, V, tol, max_iter, sh)) {
    const View V2 = view(Q, blockIdx.x);  // the column caches have traded roles
    blk_mu(Q, V2, vec, sh);
  }
}

__global__ void k_shrink(SolveSet Q, double shrink) {
  FitState* fs = Q.fs + blockIdx.x;
  if (threadIdx.x == 0 && fs_selected(fs, kPhaseBacktrack)) {
    fs->mu = fs->mu * shrink;
    fs->nbt += 1;
  }
}

// ---------------------------------------------------------------------------- FP64 polish

// r = mask (y - A_{S u C} x); returns ||r||^2.
__device__ double polish_resid(const SolveSet& Q, const View& V, const double* x, double* sh) {
  double rr = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < Q.n; i0 += (int64_t)kSubjUnroll * kThreads) {
    int64_t ii[kSubjUnroll];
    bool ok[kSubjUnroll];
    double sm[kSubjUnroll];
    subj_block(i0, Q.n, V.mask, ii, ok);
    apply_cols(V.Xs, Q.n_pad, x, V.k, Q.U, Q.n, x + V.k, ii, sm);
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w) {
      const int64_t i = i0 + (int64_t)w * kThreads;
      if (i < Q.n) {
        const double ri = ok[w] ? V.y[i] - sm[w] : 0.0;
        V.r[i] = ri;
        rr += ri * ri;
      }
    }
  }
  return ssum(rr, sh);  // its barriers also publish r to the whole block
}

// s = A_{S u C}^T r, one wave per column; returns ||s||^2.
__device__ double polish_grad(const SolveSet& Q, const View& V, double* s, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = V.k + V.nc;
  for (int q = w; q < m; q += kWaves) {
    double a = 0.0;
    if (q < V.k) {
      const double* col = V.Xs + (int64_t)q * Q.n_pad;
      for (int64_t i = lane; i < Q.n; i += 64) a += col[i] * V.r[i];
    } else {
      for (int64_t i = lane; i < Q.n; i += 64) a += ucol(Q.U, Q.n, q - V.k, i) * V.r[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) s[q] = a;
  }
  __syncthreads();
  double ss = 0.0;
  for (int q = threadIdx.x; q < m; q += kThreads) ss += s[q] * s[q];
  return ssum(ss, sh);
}

// ||A_{S u C} d||^2 over the subject set.
__device__ double polish_Anorm(const SolveSet& Q, const View& V, const double* d, double* sh) {
  double dd = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < Q.n; i0 += (int64_t)kSubjUnroll * kThreads) {
    int64_t ii[kSubjUnroll];
    bool ok[kSubjUnroll];
    double sm[kSubjUnroll];
    subj_block(i0, Q.n, V.mask, ii, ok);
    apply_cols(V.Xs, Q.n_pad, d, V.k, Q.U, Q.n, d + V.k, ii, sm);
#pragma unroll
    for (int w = 0; w < kSubjUnroll; ++w)
      if (ok[w]) dd += sm[w] * sm[w];
  }
  return ssum(dd, sh);
}

// With the support S fixed, the fixed point of the IHT map is the least-squares fit of y on S u C.
// A solve that converged with a reduced-precision gradient is refined to it in FP64 by conjugate
// gradients on the normal equations, over the exactly decoded columns of S, until the step is
// within tol max(1, ||x||_inf). The last loss-trace entry becomes the loss at the result.
__global__ __launch_bounds__(kThreads) void k_polish(SolveSet Q, double tol, int32_t max_steps) {
  if (Q.fs[blockIdx.x].status != IHT_OK) return;
  const View V = view(Q, blockIdx.x);
  __shared__ double sh[40];
  const int k = V.k, m = V.k + V.nc;
  const int64_t stride = Q.kmax + kMaxUnpenalized;
  double* x = V.pw;
  double* d = V.pw + stride;
  double* s = V.pw + 2 * stride;
  for (int q = threadIdx.x; q < k; q += kThreads) x[q] = V.beta[V.S[q]];
  for (int q = threadIdx.x; q < V.nc; q += kThreads) x[k + q] = V.bc[q];
  __syncthreads();
  double rr = polish_resid(Q, V, x, sh);
  double gamma = polish_grad(Q, V, s, sh);
  for (int q = threadIdx.x; q < m; q += kThreads) d[q] = s[q];
  __syncthreads();
  int steps = 0;
  while (steps < max_steps && gamma > 0.0) {
    const double delta = polish_Anorm(Q, V, d, sh);
    if (!(delta > 0.0)) break;
    const double alpha = gamma / delta;
    double dmax = 0.0, bmax = 0.0;
    for (int q = threadIdx.x; q < m; q += kThreads) {
      const double step = alpha * d[q];
      x[q] = x[q] + step;
      dmax = fmax(dmax, fabs(step));
      bmax = fmax(bmax, fabs(x[q]));
    }
    dmax = smax(dmax, sh);
    bmax = smax(bmax, sh);
    rr = polish_resid(Q, V, x, sh);
    const double gnew = polish_grad(Q, V, s, sh);
    const double ratio = gnew / gamma;
    for (int q = threadIdx.x; q < m; q += kThreads) d[q] = s[q] + ratio * d[q];
    __syncthreads();
    gamma = gnew;
    ++steps;
    if (dmax <= tol * fmax(1.0, bmax)) break;
  }
  for (int q = threadIdx.x; q < k; q += kThreads) V.beta[V.S[q]] = x[q];
  for (int q = threadIdx.x; q < V.nc; q += kThreads) V.bc[q] = x[k + q];
  if (threadIdx.x == 0) {
    V.fs->polish_steps = steps;
    V.fs->loss = 0.5 * rr;
    V.trace[V.fs->iter] = 0.5 * rr;
  }
}

// ---------------------------------------------------------------------------- outputs and slots

__global__ void k_output(SolveSet Q, int64_t* __restrict__ support, double* __restrict__ beta_S,
                         double* __restrict__ beta_cov, int64_t ldk, int64_t ldc) {
  const View V = view(Q, blockIdx.x);
  const bool valid = V.fs->nonfinite == 0;  // a solve rejected at the start never had a support
  for (int64_t q = threadIdx.x; q < ldk; q += blockDim.x) {
    const bool in = valid && q < V.k;
    support[(int64_t)V.t * ldk + q] = in ? V.S[q] : -1;
    beta_S[(int64_t)V.t * ldk + q] = in ? V.beta[V.S[q]] : 0.0;
  }
  if (beta_cov)
    for (int q = threadIdx.x; q < V.nc; q += blockDim.x) beta_cov[(int64_t)V.t * ldc + q] = valid ? V.bc[q] : 0.0;
}

// One wave: the solves in `phase`, ascending, packed into slots[0 .. *count).
__global__ __launch_bounds__(64) void k_slots(const FitState* __restrict__ fs, int32_t T, int32_t phase,
                                              int32_t* __restrict__ slots, int32_t* __restrict__ count) {
  const int lane = threadIdx.x;
  int base = 0;
  for (int t0 = 0; t0 < T; t0 += 64) {
    const int t = t0 + lane;
    const bool on = t < T && fs_selected(fs + t, phase);
    const uint64_t m = __ballot(on);
    if (on) slots[base + __popcll(m & ((1ull << lane) - 1ull))] = t;
    base += __popcll(m);
  }
  if (lane == 0) *count = base;
}

}  // namespace

// ---------------------------------------------------------------------------- launchers

hipError_t solve_init(const SolveSet& Q, int32_t max_iter, hipStream_t st) {
  const int64_t total = (int64_t)Q.T * Q.p;
  hipLaunchKernelGGL(k_zero_beta, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0, st, Q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_init, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, max_iter);
  return hipGetLastError();
}

hipError_t solve_residual0(const SolveSet& Q, hipStream_t st) {
  hipLaunchKernelGGL(k_residual0, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q);
  return hipGetLastError();
}

hipError_t solve_decode(const uint8_t* tiled, const SolveSet& Q, int32_t which, int32_t phase, hipStream_t st) {
  const dim3 grid((unsigned)((Q.n_pad + 255) / 256), (unsigned)Q.kmax, (unsigned)Q.T);
  hipLaunchKernelGGL(k_decode, grid, dim3(256), 0, st, tiled, Q, which, phase);
  return hipGetLastError();
}

hipError_t solve_check_residual(const SolveSet& Q, int32_t phase, double c, int32_t max_backtrack, hipStream_t st) {
  hipLaunchKernelGGL(k_check_residual, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, phase, c, max_backtrack);
  return hipGetLastError();
}

hipError_t solve_commit_mu(const SolveSet& Q, int32_t mode, double tol, int32_t max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_commit_mu, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, mode, tol, max_iter);
  return hipGetLastError();
}

hipError_t solve_shrink(const SolveSet& Q, double shrink, hipStream_t st) {
  hipLaunchKernelGGL(k_shrink, dim3((unsigned)Q.T), dim3(64), 0, st, Q, shrink);
  return hipGetLastError();
}

hipError_t solve_polish(const SolveSet& Q, double tol, int32_t max_steps, hipStream_t st) {
  hipLaunchKernelGGL(k_polish, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, tol, max_steps);
  return hipGetLastError();
}

hipError_t solve_output(const SolveSet& Q, int64_t* support, double* beta_S, double* beta_cov, int64_t ldk, int64_t ldc,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_output, dim3((unsigned)Q.T), dim3(256), 0, st, Q, support, beta_S, beta_cov, ldk, ldc);
  return hipGetLastError();
}

hipError_t solve_slots(const FitState* fs, int32_t T, int32_t phase, int32_t* slots, int32_t* count, hipStream_t st) {
  hipLaunchKernelGGL(k_slots, dim3(1), dim3(64), 0, st, fs, T, phase, slots, count);
  return hipGetLastError();
}

}  // namespace iht
