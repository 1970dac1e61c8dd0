// iht_solve.hip -- per-solve step kernels of the IHT loop.
//
// Every kernel here works on solve t = blockIdx.x (or blockIdx.y, blockIdx.z) of a SolveSet; a
// single fit is the case T = 1. The update is eq. (ihta) of Methods with the normalised step and the omega rule
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
// Only the admitted solves (admit[t] != 0; every solve if admit is NULL) are touched.
__global__ __launch_bounds__(256) void k_zero_beta(SolveSet Q, const int32_t* __restrict__ admit) {
  const int t = blockIdx.y;
  if (admit && !admit[t]) return;
  double* beta = Q.beta + (int64_t)t * Q.p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < Q.p; e += (int64_t)gridDim.x * 256) beta[e] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_init(SolveSet Q, int32_t max_iter, const int32_t* __restrict__ admit) {
  const int t = blockIdx.x;
  if (admit && !admit[t]) return;
  const double* mask = Q.sv[t].mask;
  const double* y = Q.Y + (int64_t)t * Q.ldy;
  for (int c = threadIdx.x; c < kMaxUnpenalized; c += kThreads) {
    Q.bc[(int64_t)t * kMaxUnpenalized + c] = 0.0;
    Q.bcp[(int64_t)t * kMaxUnpenalized + c] = 0.0;
    Q.gc[(int64_t)t * kMaxUnpenalized + c] = 0.0;
  }
  __shared__ int bad;
  __shared__ double sh[40];
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int b = 0;
  double sy = 0.0;
  for (int64_t i = threadIdx.x; i < Q.n; i += kThreads) {
    if (mask[i] == 0.0) continue;
    if (!isfinite(y[i]) || (Q.family == IHT_LOGISTIC && !(y[i] >= 0.0 && y[i] <= 1.0))) b = 1;
    sy += y[i];
    for (int c = 0; c < Q.U.cz; ++c)
      if (!isfinite(Q.U.Z[(int64_t)c * Q.n + i])) b = 1;
  }
  if (b) atomicOr(&bad, 1);
  // sums over the subject set of y and of the unpenalised columns (the centring constants)
  double* ys = Q.ysum + (int64_t)t * kYsumStride;
  sy = ssum(sy, sh);
  if (threadIdx.x == 0) ys[0] = sy;
  for (int c = 0; c < Q.U.cz + Q.U.icpt; ++c) {
    double sz = 0.0;
    for (int64_t i = threadIdx.x; i < Q.n; i += kThreads) sz += (mask[i] != 0.0) ? ucol(Q.U, Q.n, c, i) : 0.0;
    sz = ssum(sz, sh);
    if (threadIdx.x == 0) ys[1 + c] = sz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    FitState z{};
    z.mu = 1.0;
    z.nonfinite = bad;
    z.active = (bad || max_iter <= 0) ? 0 : 1;
    z.status = bad ? IHT_ENONFINITE : IHT_NOT_CONVERGED;
    z.fresh = 1;
    Q.fs[t] = z;
  }
}

// ---------------------------------------------------------------------------- support columns

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

// Wide decode (grid: subjects / 256 x kmax / kDecodeCols x T) of the columns of S (which = 0, into
// the current cache) or of S+ (which = 1, into the other cache) of the solves in `phase`: each
// thread takes one subject and up to kDecodeCols columns, their loads issued together. (One column
// per workgroup row made kmax x T rows of workgroups, most of them gated off in a server's launch,
// and their dispatch alone cost more than the decode.)
constexpr int kDecodeCols = 8;
__global__ __launch_bounds__(256) void k_decode(const uint8_t* __restrict__ tiled, SolveSet Q, int32_t which, int32_t phase) {
  const int t = blockIdx.z;
  const FitState* fs = Q.fs + t;
  if (!fs_selected(fs, phase)) return;
  const int q0 = blockIdx.y * kDecodeCols;
  const int k = Q.ks[t];
  if (q0 >= k) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q.n_pad) return;
  const int64_t* cols = (which ? Q.Sp : Q.S) + (int64_t)t * Q.kmax;
  const int cache = which ? 1 - fs->xcur : fs->xcur;
  double* out = Q.X + ((int64_t)t * 2 + cache) * Q.kmax * Q.n_pad;
  const BatchSolve& sv = Q.sv[t];
  // every load first (columns past k repeat the last one), then the arithmetic: no branch between
  // the loads, so all of them are in flight together
  const int64_t tile = i / kTileSubjects;
  const int grp = (int)((i % kTileSubjects) >> 2);
  const int sh = 2 * (int)(i & 3);
  const bool in = sv.mask[i] != 0.0;
  int64_t j[kDecodeCols];
  uint8_t byte[kDecodeCols];
  double uj[kDecodeCols], vj[kDecodeCols];
#pragma unroll
  for (int c = 0; c < kDecodeCols; ++c) j[c] = cols[min(q0 + c, k - 1)];
#pragma unroll
  for (int c = 0; c < kDecodeCols; ++c) {
    const int b = (grp - (int)(j[c] & (kSegBytes - 1))) & (kSegBytes - 1);
    byte[c] = tiled[(tile * Q.p_pad + j[c]) * kSegBytes + b];
    uj[c] = sv.u[j[c]];
    vj[c] = sv.v[j[c]];
  }
#pragma unroll
  for (int c = 0; c < kDecodeCols; ++c) {
    const int code = (byte[c] >> sh) & 3;
    const double d = (code == 0) ? 0.0 : (double)(code - 1);
    const double x = (!in || code == 1) ? 0.0 : vj[c] * (d - uj[c]);
    if (q0 + c < k) out[(int64_t)(q0 + c) * Q.n_pad + i] = x;
  }
}

// ---------------------------------------------------------------------------- subject-split steps
// The residual, backtracking and step-size steps split the subjects of each solve over nb =
// ceil(n / 64) workgroups (grid nb x T): lane l of workgroup b takes subject 64 b + l, and the four
// waves take every fourth support column, so that all column loads of a step are in flight at
// once. Every workgroup leaves its partial sums in Q.part (Q.pmu); a one-workgroup-per-solve kernel
// that follows adds them up in workgroup order, takes the solve's decisions and writes its state
// (the kernel boundary publishes the partials, no device-wide fence is needed). The summation
// order depends on n alone, never on the other solves of the launch.

constexpr int kMbThreads = 256;
constexpr int kMbWaves = kMbThreads / 64;
constexpr int kMbChunk = 512;  // support entries staged in LDS at a time
constexpr int kMbBatch = 8;    // column loads issued together by a lane

struct Stage {
  double coef[kMbChunk];
  int32_t col[kMbChunk];  // column (cache * kmax + q) of the solve's column caches, -1: entry skipped
  double ucoef[kMaxUnpenalized];
  double dcoef[kMaxUnpenalized];
  double red[kMbWaves][64];
  double sh[kMbWaves];
  int32_t flag;
};

__device__ __forceinline__ double wsum(double x) {  // wave sum, valid in lane 0
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

__device__ double bsum(double x, Stage& s) {  // workgroup sum, in every thread
  x = wsum(x);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s.sh[threadIdx.x >> 6] = x;
  __syncthreads();
  return (s.sh[0] + s.sh[1]) + (s.sh[2] + s.sh[3]);
}

__device__ double bmax(double x, Stage& s) {  // workgroup max, in every thread
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s.sh[threadIdx.x >> 6] = x;
  __syncthreads();
  return fmax(fmax(s.sh[0], s.sh[1]), fmax(s.sh[2], s.sh[3]));
}

// a + sum over the staged entries e = wave, wave + 4, ... of X[col_e][ii] coef_e.
__device__ __forceinline__ double acc_chunk(const double* __restrict__ Xt, int64_t n_pad, const Stage& s, int ne, int64_t ii,
                                            double a) {
  for (int e = threadIdx.x >> 6; e < ne; e += kMbBatch * kMbWaves) {
    double x[kMbBatch], cf[kMbBatch];
#pragma unroll
    for (int q = 0; q < kMbBatch; ++q) {
      const int idx = e + q * kMbWaves;
      const int c = idx < ne ? s.col[idx] : -1;
      x[q] = c >= 0 ? Xt[(int64_t)c * n_pad + ii] : 0.0;
      cf[q] = c >= 0 ? s.coef[idx] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kMbBatch; ++q) a += x[q] * cf[q];
  }
  return a;
}

// a + sum over the unpenalised columns c = wave, wave + 4, ... of A_c(ii) coef_c.
__device__ __forceinline__ double acc_unpen(const Unpen& U, int64_t n, const double* coef, int nc, int64_t ii, double a) {
  for (int c = threadIdx.x >> 6; c < nc; c += kMbWaves) a += ucol(U, n, c, ii) * coef[c];
  return a;
}

// Sum of the four wave partials of this lane's subject (in every wave).
__device__ __forceinline__ double combine_waves(double a, Stage& s) {
  __syncthreads();
  s.red[threadIdx.x >> 6][threadIdx.x & 63] = a;
  __syncthreads();
  const int l = threadIdx.x & 63;
  return (s.red[0][l] + s.red[1][l]) + (s.red[2][l] + s.red[3][l]);
}

__device__ __forceinline__ bool in_sorted(const int64_t* __restrict__ a, int k, int64_t x) {
  int lo = 0, hi = k;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < k && a[lo] == x;
}

// Sum over the solve's workgroups of partial field f of P0 (thread-strided, then the workgroup tree).
__device__ double sum_partials(const double* P0, int32_t nb, int32_t pst, int f, Stage& s) {
  double x = 0.0;
  for (int b = threadIdx.x; b < nb; b += kMbThreads) x += P0[(int64_t)b * pst + f];
  return bsum(x, s);
}

// Logistic family: sigma(x) = 1 / (1 + e^-x) without overflow, and the per-subject loss
// log(1 + e^x) - y x = max(x, 0) + log1p(e^-|x|) - y x.
__device__ __forceinline__ double sigmoid(double x) {
  if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
  const double e = exp(x);
  return e / (1.0 + e);
}
__device__ __forceinline__ double logistic_loss(double x, double y) {
  return ((x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)))) - y * x;
}

// Residual of the solves in `phase` at their proposal (kCheck), or at beta = 0 for every solve with
// finite inputs: r = mask (y - A_{S+ u C} beta+) and the residual centred over the subject set for
// the gradient pass, rc = r - m on T, 0 elsewhere (up to n_pad). The centring constant m is the
// mean of r over T in exact arithmetic: the decoded SNP columns sum to zero over T, so
// m = (sum_T y - sum_c bcp_c sum_T A_c) / |T|, known before r is. Any constant leaves the gradient
// unchanged (X_st^T 1_T = 0) as long as R = sum rc is the one used, and this one keeps rc small.
// Partial sums per workgroup: ||r||^2, R, ||A Delta||^2 and sum_T A_C r; the first workgroup adds
// ||Delta||^2 and the support-unchanged flag. k_decide turns them into the solve's state.
//
// With kCheck the proposal is under the backtracking test of "IHT step sizes": the unpenalised
// proposal is bcp = bc + mu gc and, when the support moved, omega = (1-c)||Delta||^2 / ||A Delta||^2
// over S u S+ u C, with Delta = beta+ - beta on S+, -beta on S \ S+, bcp - bc on C. r and rc are
// formed before the decision: until a proposal is taken nothing reads them.
//
// Logistic family: r = mask (y - sigma(eta)) with eta the fit above, rc = r (no centring constant is
// known in advance; any constant is exact), and the first partial is the loss sum_T [log(1 + e^eta)
// - y eta] instead of ||r||^2; the proposal is judged by that loss, so the omega sums are skipped.
template <bool kCheck>
__global__ __launch_bounds__(kMbThreads) void k_residual(SolveSet Q, int32_t phase) {
  const int t = blockIdx.y, b = blockIdx.x;
  if (!fs_selected(Q.fs + t, kCheck ? phase : kPhaseInit)) return;
  __shared__ Stage s;
  const View V = view(Q, t);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)b * kSubjBlock + lane;
  const bool in_n = i < Q.n;
  const int64_t ii = in_n ? i : 0;
  const bool ok = in_n && V.mask[ii] != 0.0;
  const int k = V.k, nc = V.nc;
  const double* Xt = Q.X + (int64_t)t * 2 * Q.kmax * Q.n_pad;
  const int cs = V.fs->xcur, cp = 1 - cs;
  const double mu = V.fs->mu;
  const double* ys = Q.ysum + (int64_t)t * kYsumStride;

  int same = 1;
  double fit = 0.0;
  if (kCheck) {
    int diff = 0;
    for (int q = threadIdx.x; q < k; q += kMbThreads) diff |= (V.S[q] != V.Sp[q]) ? 1 : 0;
    for (int q = threadIdx.x; q < nc; q += kMbThreads) s.ucoef[q] = V.bc[q] + mu * V.gc[q];
    same = __syncthreads_or(diff) ? 0 : 1;
    // fit at the proposal, A_{S+} beta+ + A_C bcp
    double a = 0.0;
    for (int e0 = 0; e0 < k; e0 += kMbChunk) {
      const int ne = min(kMbChunk, k - e0);
      __syncthreads();
      for (int e = threadIdx.x; e < ne; e += kMbThreads) {
        s.col[e] = cp * Q.kmax + e0 + e;
        s.coef[e] = V.betap[e0 + e];
      }
      __syncthreads();
      a = acc_chunk(Xt, Q.n_pad, s, ne, ii, a);
    }
    a = acc_unpen(Q.U, Q.n, s.ucoef, nc, ii, a);
    fit = combine_waves(a, s);
  }
  const bool logistic = Q.family == IHT_LOGISTIC;
  double msum = ys[0];
  if (kCheck)
    for (int q = 0; q < nc; ++q) msum -= s.ucoef[q] * ys[1 + q];
  const double m = logistic ? 0.0 : msum / (double)Q.sv[t].nT;
  const double ri = ok ? V.y[ii] - (logistic ? sigmoid(fit) : fit) : 0.0;
  const double rci = ok ? ri - m : 0.0;
  const double li = logistic ? (ok ? logistic_loss(fit, V.y[ii]) : 0.0) : ri * ri;
  if (w == 0 && i < Q.n_pad) {
    V.r[i] = ri;
    V.rc[i] = rci;
  }

  double ad2 = 0.0, dd = 0.0;
  if (kCheck && !same && !logistic) {
    double dd_t = 0.0, a = 0.0;
    for (int e0 = 0; e0 < 2 * k; e0 += kMbChunk) {
      const int ne = min(kMbChunk, 2 * k - e0);
      __syncthreads();
      for (int e = threadIdx.x; e < ne; e += kMbThreads) {
        const int q = e0 + e;
        int col;
        double d;
        if (q < k) {
          col = cp * Q.kmax + q;
          d = V.betap[q] - V.beta[V.Sp[q]];
        } else {
          const int64_t j = V.S[q - k];
          const bool kept = in_sorted(V.Sp, k, j);
          col = kept ? -1 : cs * Q.kmax + (q - k);
          d = kept ? 0.0 : 0.0 - V.beta[j];
        }
        s.col[e] = col;
        s.coef[e] = d;
        dd_t += d * d;
      }
      __syncthreads();
      a = acc_chunk(Xt, Q.n_pad, s, ne, ii, a);
    }
    for (int q = threadIdx.x; q < nc; q += kMbThreads) {
      const double d = s.ucoef[q] - V.bc[q];
      s.dcoef[q] = d;
      dd_t += d * d;
    }
    __syncthreads();
    a = acc_unpen(Q.U, Q.n, s.dcoef, nc, ii, a);
    const double x = combine_waves(a, s);
    ad2 = ok ? x * x : 0.0;
    if (b == 0) dd = bsum(dd_t, s);  // workgroup-uniform branch
  }

  if (w == 0) {
    double* P = Q.part + ((int64_t)t * Q.nb + b) * Q.pst;
    const double rr = wsum(li), R = wsum(rci), sa = wsum(ad2);
    if (lane == 0) {
      P[0] = rr;
      P[1] = R;
      P[2] = sa;
      P[3] = dd;
      P[4] = (double)same;
    }
    for (int q = 0; q < nc; ++q) {
      const double gq = wsum(ucol(Q.U, Q.n, q, ii) * ri);
      if (lane == 0) P[5 + q] = gq;
    }
  }
}

// The solve's state from the partial sums of k_residual (grid T). kCheck: the backtracking decision
// (taken when the support is unchanged or mu < omega; otherwise a halving is needed, and with the
// budget spent the solve stops, stalled, keeping beta) and bcp. For a taken proposal (and at the
// start): loss 1/2 ||r||^2 (eq. leastsquaresloss) into the trace (entry iter + 1, or 0), gc = A_C^T r
// and R for the gradient pass.
template <bool kCheck>
__global__ __launch_bounds__(kMbThreads) void k_decide(SolveSet Q, int32_t phase, double c, int32_t max_backtrack) {
  const int t = blockIdx.x;
  if (!fs_selected(Q.fs + t, kCheck ? phase : kPhaseInit)) return;
  __shared__ Stage s;
  const View V = view(Q, t);
  FitState* fs = V.fs;
  const double* P0 = Q.part + (int64_t)t * Q.nb * Q.pst;
  const int nc = V.nc;
  const bool logistic = Q.family == IHT_LOGISTIC;
  if (kCheck) {
    const double mu = fs->mu;
    const int same = P0[4] != 0.0 ? 1 : 0;
    double omega = 0.0;
    int accept = 1;
    if (logistic) {  // taken when the loss does not increase beyond the rounding of its sums
      accept = sum_partials(P0, Q.nb, Q.pst, 0, s) <= fs->loss + 1e-12 * fabs(fs->loss) ? 1 : 0;
    } else if (!same) {
      const double sa = sum_partials(P0, Q.nb, Q.pst, 2, s);
      omega = (1.0 - c) * P0[3] / sa;
      accept = mu < omega ? 1 : 0;
    }
    for (int q = threadIdx.x; q < nc; q += kMbThreads) V.bcp[q] = V.bc[q] + mu * V.gc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
      fs->same = same;
      fs->omega = omega;
      fs->accept = accept;
      fs->go = accept;
      fs->need_bt = accept ? 0 : 1;
      if (!accept && fs->nbt >= max_backtrack) {
        fs->need_bt = 0;
        fs->active = 0;
        fs->status = IHT_STALLED;
      }
    }
    if (!accept) return;
  }
  const double lsum = sum_partials(P0, Q.nb, Q.pst, 0, s);
  const double loss = logistic ? lsum : 0.5 * lsum;
  const double R = sum_partials(P0, Q.nb, Q.pst, 1, s);
  for (int q = 0; q < nc; ++q) {
    const double gq = sum_partials(P0, Q.nb, Q.pst, 5 + q, s);
    if (threadIdx.x == 0) V.gc[q] = gq;
  }
  if (threadIdx.x == 0) {
    V.trace[kCheck ? fs->iter + 1 : 0] = loss;
    fs->loss = loss;
    fs->Rsum = R;
  }
}

// Partial sums of the step-size denominator ||A_{S u C} g_{S u C}||^2 ("IHT step sizes", normalised
// form) over each workgroup's subjects, on S (mode 0, first iteration of the newly admitted solves) or on S+
// (mode 1, the solves whose proposal was taken). In mode 1 the first workgroup also commits the
// proposal: the convergence test (S+ = S and ||beta+ - beta||_inf <= tol max(1, ||beta+||_inf); with
// S+ = S the union of the supports is S itself, so the norms run over S+ and C), then beta <- beta+,
// S <- S+, bc <- bcp. The control state changes in k_mu.
__global__ __launch_bounds__(kMbThreads) void k_commit_den(SolveSet Q, int32_t mode, double tol) {
  const int t = blockIdx.y, b = blockIdx.x;
  if (!fs_selected(Q.fs + t, mode == 0 ? kPhaseFresh : kPhaseGo)) return;
  __shared__ Stage s;
  const View V = view(Q, t);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)b * kSubjBlock + lane;
  const bool in_n = i < Q.n;
  const int64_t ii = in_n ? i : 0;
  const bool ok = in_n && V.mask[ii] != 0.0;
  const int k = V.k, nc = V.nc;
  const double* Xt = Q.X + (int64_t)t * 2 * Q.kmax * Q.n_pad;
  const int64_t* Sn = mode ? V.Sp : V.S;
  const int cn = mode ? 1 - V.fs->xcur : V.fs->xcur;

  for (int q = threadIdx.x; q < nc; q += kMbThreads) s.ucoef[q] = V.gc[q];
  double a = 0.0;
  for (int e0 = 0; e0 < k; e0 += kMbChunk) {
    const int ne = min(kMbChunk, k - e0);
    __syncthreads();
    for (int e = threadIdx.x; e < ne; e += kMbThreads) {
      s.col[e] = cn * Q.kmax + e0 + e;
      s.coef[e] = V.g[Sn[e0 + e]];
    }
    __syncthreads();
    a = acc_chunk(Xt, Q.n_pad, s, ne, ii, a);
  }
  a = acc_unpen(Q.U, Q.n, s.ucoef, nc, ii, a);
  const double x = combine_waves(a, s);
  if (w == 0) {
    // logistic: curvature weight sigma (1 - sigma) at the current beta, sigma = y - r
    double wt = 1.0;
    if (Q.family == IHT_LOGISTIC && ok) {
      const double sg = V.y[ii] - V.r[ii];
      wt = sg * (1.0 - sg);
    }
    const double dd = wsum(ok ? wt * (x * x) : 0.0);
    if (lane == 0) Q.pmu[(int64_t)t * Q.nb + b] = dd;
  }
  if (mode == 0 || b != 0) return;

  // commit (first workgroup; the others read neither beta, S nor bc)
  FitState* fs = V.fs;
  int diff = 0;
  double dmax = 0.0, bmx = 0.0;
  for (int q = threadIdx.x; q < k; q += kMbThreads) {
    diff |= (V.S[q] != V.Sp[q]) ? 1 : 0;
    dmax = fmax(dmax, fabs(V.betap[q] - V.beta[V.Sp[q]]));
    bmx = fmax(bmx, fabs(V.betap[q]));
  }
  for (int q = threadIdx.x; q < nc; q += kMbThreads) {
    dmax = fmax(dmax, fabs(V.bcp[q] - V.bc[q]));
    bmx = fmax(bmx, fabs(V.bcp[q]));
  }
  const int same = __syncthreads_or(diff) ? 0 : 1;
  dmax = bmax(dmax, s);
  bmx = bmax(bmx, s);
  for (int q = threadIdx.x; q < k; q += kMbThreads) V.beta[V.S[q]] = 0.0;
  __syncthreads();
  for (int q = threadIdx.x; q < k; q += kMbThreads) {
    V.beta[V.Sp[q]] = V.betap[q];
    V.S[q] = V.Sp[q];
  }
  for (int q = threadIdx.x; q < nc; q += kMbThreads) V.bc[q] = V.bcp[q];
  if (threadIdx.x == 0) {
    fs->same = same;
    fs->dmax = dmax;
    fs->bmax = bmx;
    fs->conv = same && dmax <= tol * fmax(1.0, bmx);
  }
}

// Control state after k_commit_den (grid T). Mode 1: the committed solves count one more iteration,
// their column caches trade roles (the proposal's cache now holds the columns of S), and they stop
// when converged or at max_iter. Then the step size mu = ||g_{S u C}||^2 / ||A_{S u C} g_{S u C}||^2 of
// those still iterating; a zero denominator means the gradient vanishes on S u C: nothing can move,
// the solve ends there (converged).
__global__ __launch_bounds__(kMbThreads) void k_mu(SolveSet Q, int32_t mode, int32_t max_iter) {
  const int t = blockIdx.x;
  if (!fs_selected(Q.fs + t, mode == 0 ? kPhaseFresh : kPhaseGo)) return;
  __shared__ Stage s;
  const View V = view(Q, t);
  FitState* fs = V.fs;
  if (mode == 1) {
    __syncthreads();  // every thread has read the selection flags
    if (threadIdx.x == 0) {
      fs->iter += 1;
      fs->go = 0;
      fs->xcur ^= 1;
      if (fs->conv) {
        fs->active = 0;
        fs->status = IHT_OK;
      } else if (fs->iter >= max_iter) {
        fs->active = 0;
        fs->status = IHT_NOT_CONVERGED;
      }
      s.flag = fs->active;
    }
    __syncthreads();
    if (!s.flag) return;
  }
  const double den = sum_partials(Q.pmu + (int64_t)t * Q.nb, Q.nb, 1, 0, s);
  double nm = 0.0;
  for (int q = threadIdx.x; q < V.k; q += kMbThreads) {
    const double gq = V.g[V.S[q]];
    nm += gq * gq;
  }
  for (int q = threadIdx.x; q < V.nc; q += kMbThreads) nm += V.gc[q] * V.gc[q];
  const double num = bsum(nm, s);
  if (threadIdx.x == 0) {
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
}

// Exact gradient on the support of an accepted proposal (matrix-core fits): g_j = sum_i x_st(i, j) rq_i
// for the columns of S+, held decoded in the proposal's cache, one wave per column in a fixed order.
// The matrix-core pass leaves every g_j within fs.gerr of this; the step size, the support's values
// in the next proposal and the convergence test then see the FP64 values, as after a FP64 pass.
__global__ __launch_bounds__(256) void k_exact_support(SolveSet Q, const double* __restrict__ rq) {
  const int t = blockIdx.y;
  if (!fs_selected(Q.fs + t, kPhaseGo)) return;
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= Q.ks[t]) return;
  const int cp = 1 - Q.fs[t].xcur;
  const double* col = Q.X + (((int64_t)t * 2 + cp) * Q.kmax + q) * Q.n_pad;
  const double* r = rq + (int64_t)t * Q.n_pad;
  double a0 = 0.0, a1 = 0.0;
  int64_t i = lane;
  for (; i + 64 < Q.n; i += 128) {
    a0 += col[i] * r[i];
    a1 += col[i + 64] * r[i + 64];
  }
  if (i < Q.n) a0 += col[i] * r[i];
  const double a = wsum(a0 + a1);
  if (lane == 0) Q.g[(int64_t)t * Q.p + Q.Sp[(int64_t)t * Q.kmax + q]] = a;
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
  if (!fs_selected(Q.fs + blockIdx.x, kPhaseRetire) || Q.fs[blockIdx.x].status != IHT_OK) return;
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

// Outputs of the solves being written out, into their rows (support ascending and beta_S padded
// to ld with -1 / 0; beta_cov; the loss trace entries 0 .. iter when trace is not NULL).
__global__ void k_output(SolveSet Q, const OutRow* __restrict__ rows) {
  if (!fs_selected(Q.fs + blockIdx.x, kPhaseRetire)) return;
  const View V = view(Q, blockIdx.x);
  const OutRow o = rows[blockIdx.x];
  const bool valid = V.fs->nonfinite == 0;  // a solve rejected at the start never had a support
  for (int64_t q = threadIdx.x; q < o.ld; q += blockDim.x) {
    const bool in = valid && q < V.k;
    o.support[q] = in ? V.S[q] : -1;
    o.beta_S[q] = in ? V.beta[V.S[q]] : 0.0;
  }
  if (o.beta_cov)
    for (int q = threadIdx.x; q < V.nc; q += blockDim.x) o.beta_cov[q] = valid ? V.bc[q] : 0.0;
  if (o.trace)
    for (int q = threadIdx.x; q <= V.fs->iter; q += blockDim.x) o.trace[q] = V.trace[q];
}

// fs[t].fresh (field 0) or fs[t].retire (field 1) = value for the solves with flags[t] != 0 (all
// solves if flags is NULL).
__global__ void k_mark(FitState* __restrict__ fs, int32_t T, const int32_t* __restrict__ flags, int32_t field,
                       int32_t value) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || (flags && !flags[t])) return;
  if (field == 0)
    fs[t].fresh = value;
  else
    fs[t].retire = value;
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

hipError_t solve_init(const SolveSet& Q, int32_t max_iter, const int32_t* admit, hipStream_t st) {
  const unsigned bx = (unsigned)std::min<int64_t>((Q.p + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_beta, dim3(bx, (unsigned)Q.T), dim3(256), 0, st, Q, admit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_init, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, max_iter, admit);
  return hipGetLastError();
}

hipError_t solve_residual0(const SolveSet& Q, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<false>, dim3((unsigned)Q.nb, (unsigned)Q.T), dim3(kMbThreads), 0, st, Q, kPhaseInit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_decide<false>, dim3((unsigned)Q.T), dim3(kMbThreads), 0, st, Q, kPhaseInit, 0.0, 0);
  return hipGetLastError();
}

hipError_t solve_decode(const uint8_t* tiled, const SolveSet& Q, int32_t which, int32_t phase, hipStream_t st) {
  const dim3 grid((unsigned)((Q.n_pad + 255) / 256), (unsigned)((Q.kmax + kDecodeCols - 1) / kDecodeCols), (unsigned)Q.T);
  hipLaunchKernelGGL(k_decode, grid, dim3(256), 0, st, tiled, Q, which, phase);
  return hipGetLastError();
}

hipError_t solve_check_residual(const SolveSet& Q, int32_t phase, double c, int32_t max_backtrack, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<true>, dim3((unsigned)Q.nb, (unsigned)Q.T), dim3(kMbThreads), 0, st, Q, phase);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_decide<true>, dim3((unsigned)Q.T), dim3(kMbThreads), 0, st, Q, phase, c, max_backtrack);
  return hipGetLastError();
}

hipError_t solve_commit_mu(const SolveSet& Q, int32_t mode, double tol, int32_t max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_commit_den, dim3((unsigned)Q.nb, (unsigned)Q.T), dim3(kMbThreads), 0, st, Q, mode, tol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mu, dim3((unsigned)Q.T), dim3(kMbThreads), 0, st, Q, mode, max_iter);
  return hipGetLastError();
}

hipError_t solve_shrink(const SolveSet& Q, double shrink, hipStream_t st) {
  hipLaunchKernelGGL(k_shrink, dim3((unsigned)Q.T), dim3(64), 0, st, Q, shrink);
  return hipGetLastError();
}

hipError_t solve_exact_support(const SolveSet& Q, const double* rq, hipStream_t st) {
  hipLaunchKernelGGL(k_exact_support, dim3((unsigned)((Q.kmax + 3) / 4), (unsigned)Q.T), dim3(256), 0, st, Q, rq);
  return hipGetLastError();
}

hipError_t solve_polish(const SolveSet& Q, double tol, int32_t max_steps, hipStream_t st) {
  hipLaunchKernelGGL(k_polish, dim3((unsigned)Q.T), dim3(kThreads), 0, st, Q, tol, max_steps);
  return hipGetLastError();
}

hipError_t solve_output(const SolveSet& Q, const OutRow* rows, hipStream_t st) {
  hipLaunchKernelGGL(k_output, dim3((unsigned)Q.T), dim3(256), 0, st, Q, rows);
  return hipGetLastError();
}

hipError_t solve_mark(const SolveSet& Q, const int32_t* flags, int32_t field, int32_t value, hipStream_t st) {
  hipLaunchKernelGGL(k_mark, dim3((unsigned)((Q.T + 255) / 256)), dim3(256), 0, st, Q.fs, Q.T, flags, field, value);
  return hipGetLastError();
}

hipError_t solve_slots(const FitState* fs, int32_t T, int32_t phase, int32_t* slots, int32_t* count, hipStream_t st) {
  hipLaunchKernelGGL(k_slots, dim3(1), dim3(64), 0, st, fs, T, phase, slots, count);
  return hipGetLastError();
}

}  // namespace iht

// ---------------------------------------------------------------------------- prediction and cross-validation

namespace iht {
namespace {

// Prediction of subject i by a fitted model: sum_q x_st(i, sup[q]) b[q] with the standardisation u,
// v (a missing dosage is mean-imputed, i.e. 0 after standardising; entries of sup outside [0, p)
// are skipped and reported through *bad), plus the unpenalised columns times bc.
__device__ __forceinline__ double predict_subject(const uint8_t* __restrict__ tiled, int64_t n, int64_t p, int64_t p_pad,
                                                  int64_t i, const int64_t* __restrict__ sup,
                                                  const double* __restrict__ b, int32_t k, const double* __restrict__ u,
                                                  const double* __restrict__ v, const Unpen& U,
                                                  const double* __restrict__ bc, bool* bad) {
  const int64_t tile = i / kTileSubjects;
  const int grp = (int)((i % kTileSubjects) >> 2);
  const int sh = 2 * (int)(i & 3);
  double pred = 0.0;
  for (int32_t q = 0; q < k; ++q) {
    const int64_t j = sup[q];
    if (j < 0 || j >= p) {
      *bad = true;
      continue;
    }
    const int bt = (grp - (int)(j & (kSegBytes - 1))) & (kSegBytes - 1);
    const int code = (tiled[(tile * p_pad + j) * kSegBytes + bt] >> sh) & 3;
    const double x = (code == 1) ? 0.0 : v[j] * ((code == 0 ? 0.0 : (double)(code - 1)) - u[j]);
    pred += x * b[q];
  }
  for (int c = 0; c < U.cz + U.icpt; ++c) pred += ucol(U, n, c, i) * bc[c];
  return pred;
}

// out[i] = prediction of every subject i < n; err bit 0 is set if the support held an index outside [0, p).
__global__ __launch_bounds__(256) void k_predict(const uint8_t* __restrict__ tiled, int64_t n, int64_t p, int64_t p_pad,
                                                 const int64_t* __restrict__ sup, const double* __restrict__ b, int32_t k,
                                                 const double* __restrict__ u, const double* __restrict__ v, Unpen U,
                                                 const double* __restrict__ bc, double* __restrict__ out,
                                                 uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  bool bad = false;
  out[i] = predict_subject(tiled, n, p, p_pad, i, sup, b, k, u, v, U, bc, &bad);
  if (bad) atomicOr(err, 1u);
}

// Held-out squared errors (Methods, "Model selection"): solve t = f * r + a was fitted on the
// subjects outside fold f; every subject i of fold f is predicted with the solve's model,
// standardised with its training u, v, and (y_i - prediction)^2 is summed per block in a fixed order.
__global__ __launch_bounds__(256) void k_cv_sqerr(const uint8_t* __restrict__ tiled, int64_t n, int64_t p, int64_t p_pad,
                                                  const uint8_t* __restrict__ folds, int32_t r, const BatchSolve* __restrict__ sv,
                                                  const int32_t* __restrict__ ks, const int64_t* __restrict__ support,
                                                  const double* __restrict__ beta_S, int64_t ldk,
                                                  const double* __restrict__ beta_cov, int64_t ldc, Unpen U,
                                                  const double* __restrict__ y, double* __restrict__ part) {
  const int t = blockIdx.y;
  const int f = t / r;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (i < n && folds[i] == f) {
    bool bad = false;  // the supports come from the solver: always inside [0, p)
    const double d = y[i] - predict_subject(tiled, n, p, p_pad, i, support + (int64_t)t * ldk, beta_S + (int64_t)t * ldk,
                                            ks[t], sv[t].u, sv[t].v, U, beta_cov + (int64_t)t * ldc, &bad);
    e2 = d * d;
  }
  __shared__ double sh[40];
  e2 = ssum(e2, sh);
  if (threadIdx.x == 0) part[(int64_t)t * gridDim.x + blockIdx.x] = e2;
}

// mse[a * q + f] = (sum of fold f's block partials of solve f * r + a, in block order) / |fold f|;
// then k_best = the k of least mean MSE over the folds (the first in ks on an exact tie).
__global__ __launch_bounds__(64) void k_cv_finish(const double* __restrict__ part, int32_t nblk, int32_t q, int32_t r,
                                                  const int64_t* __restrict__ fold_count, const int32_t* __restrict__ ks,
                                                  double* __restrict__ mse, int32_t* __restrict__ k_best) {
  if (threadIdx.x != 0) return;
  for (int f = 0; f < q; ++f)
    for (int a = 0; a < r; ++a) {
      const double* P = part + (int64_t)(f * r + a) * nblk;
      double s = 0.0;
      for (int b = 0; b < nblk; ++b) s += P[b];
      mse[(int64_t)a * q + f] = s / (double)fold_count[f];
    }
  double best = 0.0;
  for (int a = 0; a < r; ++a) {
    double s = 0.0;
    for (int f = 0; f < q; ++f) s += mse[(int64_t)a * q + f];
    s /= (double)q;
    if (a == 0 || s < best) {
      best = s;
      *k_best = ks[a];
    }
  }
}

}  // namespace

hipError_t cv_heldout_mse(const uint8_t* tiled, const Layout& L, const uint8_t* folds, int32_t q, int32_t r,
                          const BatchSolve* sv, const int32_t* ks_solve, const int32_t* ks_path, const int64_t* support,
                          const double* beta_S, int64_t ldk, const double* beta_cov, int64_t ldc, const Unpen& U,
                          const double* y, const int64_t* fold_count, double* part, double* mse, int32_t* k_best,
                          hipStream_t st) {
  const int32_t nblk = (int32_t)((L.n + 255) / 256);
  hipLaunchKernelGGL(k_cv_sqerr, dim3((unsigned)nblk, (unsigned)(q * r)), dim3(256), 0, st, tiled, L.n, L.p, L.p_pad, folds, r, sv,
                     ks_solve, support, beta_S, ldk, beta_cov, ldc, U, y, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cv_finish, dim3(1), dim3(64), 0, st, part, nblk, q, r, fold_count, ks_path, mse, k_best);
  return hipGetLastError();
}

hipError_t launch_predict(const uint8_t* tiled, const Layout& L, const int64_t* support, const double* beta_S, int32_t k,
                          const double* u, const double* v, const Unpen& U, const double* beta_cov, double* out,
                          uint32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_predict, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, tiled, L.n, L.p, L.p_pad, support,
                     beta_S, k, u, v, U, beta_cov, out, err);
  return hipGetLastError();
}

}  // namespace iht
