// iht_api.hip -- host runtime behind include/iht.h: handles, argument checks, the solve loop.
//
// The solve loop follows Methods, eq. (ihta) with the normalised step and the omega rule of
// "IHT step sizes". All arithmetic runs in the device kernels; the host only orders launches and
// reads back the flags that decide the next launch (support moved? step accepted? converged?).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "iht.h"
#include "iht_batch.h"
#include "iht_internal.h"

using namespace iht;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? IHT_ENOMEM : IHT_EDEVICE;
}

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, std::max<size_t>(b, 256));
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

Layout make_layout(int64_t n, int64_t p) {
  Layout L;
  L.n = n;
  L.p = p;
  L.ntiles = (n + kTileSubjects - 1) / kTileSubjects;
  L.n_pad = L.ntiles * kTileSubjects;
  L.p_pad = (p + kSnpAlign - 1) / kSnpAlign * kSnpAlign;
  return L;
}

// Device work area for top-k; counters and histogram start zeroed and are self-resetting.
struct TopkArea {
  DevBuf small;  // hist | counters | state | sel
  DevBuf cand;
  int64_t cap = 0;
  TopkWork tw{};
  int ensure(int64_t p, hipStream_t st) {
    const size_t small_bytes = kTopkBins0 * 4 + 8 * 4 + 8 * 4 + kTopkMaxK * 4;
    if (!small.p) {
      HIPCHK(small.ensure(small_bytes));
      HIPCHK(launch_zero_u32(small.as<uint32_t>(), (int32_t)(small_bytes / 4), st));
    }
    if (p > cap) {
      HIPCHK(cand.ensure(topk_cand_capacity_bytes(p)));
      cap = p;
    }
    uint32_t* b = small.as<uint32_t>();
    tw.hist = b;
    tw.counters = b + kTopkBins0;
    tw.state = b + kTopkBins0 + 8;
    tw.sel = reinterpret_cast<int32_t*>(b + kTopkBins0 + 16);
    tw.cand_key = cand.as<uint64_t>();
    tw.cand_idx = reinterpret_cast<int32_t*>(cand.as<char>() + (size_t)cap * sizeof(uint64_t));
    return IHT_OK;
  }
};

}  // namespace

// One solve's device state (grown on demand, reused by later solves on the same genotype handle).
namespace {
struct FitWork {
  DevBuf beta, g, partial, r, S, Sp, betap, Xs, Xp, bc, bcp, gc, fs, bt;
  TopkArea topk;
};
}  // namespace

struct iht_geno {
  int device = 0;
  Layout L{};
  DevBuf tiled;
  // scratch for iht_gradient (centred residual, partial sums, scalars) and for iht_fit
  DevBuf partial, state;
  FitWork fit;
  DevBuf batch_r8, batch_scale, batch_rsum, batch_sv;  // iht_gradient_batch work areas
};

struct iht_stats {
  const iht_geno* geno = nullptr;
  int64_t nT = 0;
  DevBuf u, v, mask, mask_bits;
};

extern "C" {

void iht_opts_default(iht_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_iter = 200;
  o->max_backtrack = 50;
  o->c = 0.01;
  o->shrink = 0.5;
  o->precision = IHT_FP64;
}

const char* iht_last_error(void) { return g_last_error.c_str(); }

const char* iht_status_str(int s) {
  switch (s) {
    case IHT_OK: return "ok";
    case IHT_NOT_CONVERGED: return "not converged (max_iter reached)";
    case IHT_STALLED: return "stalled (backtracking budget exhausted)";
    case IHT_EINVAL: return "invalid argument";
    case IHT_ENOMEM: return "device out of memory";
    case IHT_EDEVICE: return "device error";
    case IHT_ENONFINITE: return "non-finite input";
    case IHT_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int iht_geno_create(const uint8_t* bed, int64_t n, int64_t p, int64_t row_bytes, int32_t flags, void* stream, iht_geno** out) {
  if (!out) return fail(IHT_EINVAL, "iht_geno_create: out is NULL");
  *out = nullptr;
  if (!bed) return fail(IHT_EINVAL, "iht_geno_create: bed is NULL");
  if (n < 1 || p < 1 || n > (int64_t(1) << 24) || p > (int64_t(1) << 28) - kSnpAlign)
    return fail(IHT_EINVAL, "iht_geno_create: n or p out of range");
  if (row_bytes < (n + 3) / 4) return fail(IHT_EINVAL, "iht_geno_create: row_bytes < ceil(n/4)");
  if (flags != IHT_HOST_PTR && flags != IHT_DEVICE_PTR) return fail(IHT_EINVAL, "iht_geno_create: bad flags");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_geno* G = new (std::nothrow) iht_geno();
  if (!G) return fail(IHT_ENOMEM, "iht_geno_create: host allocation");
  int rc = IHT_OK;
  do {
    hipError_t e = hipGetDevice(&G->device);
    if (e != hipSuccess) { rc = hip_fail(e, "hipGetDevice"); break; }
    G->L = make_layout(n, p);
    const size_t tiled_bytes = (size_t)G->L.ntiles * (size_t)G->L.p_pad * kSegBytes;
    e = G->tiled.ensure(tiled_bytes);
    if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(tiled)"); break; }
    const uint8_t* src = bed;
    DevBuf staging;
    if (flags == IHT_HOST_PTR) {
      e = staging.ensure((size_t)p * (size_t)row_bytes);
      if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(staging)"); break; }
      e = hipMemcpyAsync(staging.p, bed, (size_t)p * (size_t)row_bytes, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) { rc = hip_fail(e, "hipMemcpyAsync(bed)"); break; }
      src = staging.as<uint8_t>();
    }
    e = launch_retile(src, row_bytes, G->L, G->tiled.as<uint8_t>(), st);
    if (e != hipSuccess) { rc = hip_fail(e, "retile launch"); break; }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) { rc = hip_fail(e, "retile"); break; }
  } while (0);
  if (rc != IHT_OK) {
    delete G;
    return rc;
  }
  *out = G;
  return IHT_OK;
}

int iht_geno_destroy(iht_geno* g) {
  delete g;
  return IHT_OK;
}

int iht_geno_shape(const iht_geno* g, int64_t* n, int64_t* p) {
  if (!g) return fail(IHT_EINVAL, "iht_geno_shape: NULL handle");
  if (n) *n = g->L.n;
  if (p) *p = g->L.p;
  return IHT_OK;
}

int iht_stats_create(const iht_geno* g, const uint8_t* subset, void* stream, iht_stats** out) {
  if (!out) return fail(IHT_EINVAL, "iht_stats_create: out is NULL");
  *out = nullptr;
  if (!g) return fail(IHT_EINVAL, "iht_stats_create: NULL geno");
  const Layout& L = g->L;
  std::vector<double> mask(L.n_pad, 0.0);
  std::vector<uint32_t> bits(L.ntiles, 0);
  int64_t nT = 0;
  for (int64_t i = 0; i < L.n; ++i) {
    const uint8_t m = subset ? subset[i] : 1;
    if (m > 1) return fail(IHT_EINVAL, "iht_stats_create: subset entries must be 0 or 1");
    if (m) {
      mask[i] = 1.0;
      bits[i / kTileSubjects] |= uint32_t(1) << (i % kTileSubjects);
      ++nT;
    }
  }
  if (nT < 1) return fail(IHT_EINVAL, "iht_stats_create: empty subject set");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_stats* S = new (std::nothrow) iht_stats();
  if (!S) return fail(IHT_ENOMEM, "iht_stats_create: host allocation");
  S->geno = g;
  S->nT = nT;
  int rc = IHT_OK;
  do {
    hipError_t e;
    if ((e = S->u.ensure(L.p * 8)) != hipSuccess || (e = S->v.ensure(L.p * 8)) != hipSuccess ||
        (e = S->mask.ensure(L.n_pad * 8)) != hipSuccess || (e = S->mask_bits.ensure(L.ntiles * 4)) != hipSuccess) {
      rc = hip_fail(e, "hipMalloc(stats)");
      break;
    }
    if ((e = hipMemcpyAsync(S->mask.p, mask.data(), L.n_pad * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(S->mask_bits.p, bits.data(), L.ntiles * 4, hipMemcpyHostToDevice, st)) != hipSuccess) {
      rc = hip_fail(e, "hipMemcpyAsync(mask)");
      break;
    }
    if ((e = launch_stats(g->tiled.as<uint8_t>(), L, S->mask_bits.as<uint32_t>(), nT, S->u.as<double>(), S->v.as<double>(),
                          st)) != hipSuccess) {
      rc = hip_fail(e, "stats launch");
      break;
    }
    // the host vectors are freed on return: wait for the copies
    if ((e = hipStreamSynchronize(st)) != hipSuccess) {
      rc = hip_fail(e, "stats");
      break;
    }
  } while (0);
  if (rc != IHT_OK) {
    delete S;
    return rc;
  }
  *out = S;
  return IHT_OK;
}

int iht_stats_destroy(iht_stats* s) {
  delete s;
  return IHT_OK;
}

int iht_stats_read(const iht_stats* s, double* u, double* v, void* stream) {
  if (!s) return fail(IHT_EINVAL, "iht_stats_read: NULL handle");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t b = (size_t)s->geno->L.p * 8;
  if (u) HIPCHK(hipMemcpyAsync(u, s->u.p, b, hipMemcpyDeviceToDevice, st));
  if (v) HIPCHK(hipMemcpyAsync(v, s->v.p, b, hipMemcpyDeviceToDevice, st));
  return IHT_OK;
}

int iht_gradient(const iht_geno* g, const iht_stats* s, const double* r, double* grad, int32_t precision, void* stream) {
  if (!g || !s || !r || !grad) return fail(IHT_EINVAL, "iht_gradient: NULL argument");
  if (s->geno != g) return fail(IHT_EINVAL, "iht_gradient: stats belong to another genotype handle");
  if (precision != IHT_FP64 && precision != IHT_FP32) return fail(IHT_EINVAL, "iht_gradient: bad precision");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_geno* G = const_cast<iht_geno*>(g);
  const Layout& L = g->L;
  HIPCHK(G->state.ensure(sizeof(FitState)));
  const size_t pb = gradient_partial_bytes(L);
  if (pb) HIPCHK(G->partial.ensure(pb));
  FitState* fs = G->state.as<FitState>();
  HIPCHK(launch_gradient(g->tiled.as<uint8_t>(), L, r, s->mask.as<double>(), s->nT, s->u.as<double>(), s->v.as<double>(), fs,
                         precision, grad, G->partial.as<double>(), nullptr, st));
  return IHT_OK;
}

// Work area of iht_project: one per (thread, device), kept for the life of the process.
int iht_gradient_batch(const iht_geno* g, const iht_stats* const* stats, int32_t T, const double* R, double* G, void* stream) {
  if (!g || !stats || !R || !G) return fail(IHT_EINVAL, "iht_gradient_batch: NULL argument");
  if (T < 1 || T > 65536) return fail(IHT_EINVAL, "iht_gradient_batch: T out of range");
  std::vector<BatchSolve> sv((size_t)T);
  for (int32_t t = 0; t < T; ++t) {
    if (!stats[t]) return fail(IHT_EINVAL, "iht_gradient_batch: NULL stats handle");
    if (stats[t]->geno != g) return fail(IHT_EINVAL, "iht_gradient_batch: stats belong to another genotype handle");
    sv[t] = BatchSolve{stats[t]->u.as<double>(), stats[t]->v.as<double>(), stats[t]->mask.as<double>(), stats[t]->nT};
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_geno* Gh = const_cast<iht_geno*>(g);
  const Layout& L = g->L;
  const int32_t Tp = batch_t_pad(T);
  HIPCHK(Gh->batch_r8.ensure(batch_r8_bytes(L, T)));
  HIPCHK(Gh->batch_scale.ensure((size_t)Tp * 8));
  HIPCHK(Gh->batch_rsum.ensure((size_t)Tp * 8));
  HIPCHK(Gh->batch_sv.ensure((size_t)T * sizeof(BatchSolve)));
  HIPCHK(hipMemcpyAsync(Gh->batch_sv.p, sv.data(), (size_t)T * sizeof(BatchSolve), hipMemcpyHostToDevice, st));
  HIPCHK(launch_gradient_batch(g->tiled.as<uint8_t>(), L, R, T, Gh->batch_sv.as<BatchSolve>(), Gh->batch_r8.as<int8_t>(),
                               Gh->batch_scale.as<double>(), Gh->batch_rsum.as<double>(), G, L.p, st));
  // the host copy of the per-solve table must outlive the copy
  HIPCHK(hipStreamSynchronize(st));
  return IHT_OK;
}

static TopkArea* project_area() {
  static thread_local std::vector<TopkArea*> areas;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  if ((size_t)dev >= areas.size()) areas.resize(dev + 1, nullptr);
  if (!areas[dev]) areas[dev] = new (std::nothrow) TopkArea();
  return areas[dev];
}

int iht_project(const double* w, int64_t p, int32_t k, int64_t* support, double* w_out, void* stream) {
  if (!w || !support) return fail(IHT_EINVAL, "iht_project: NULL argument");
  if (p < 1 || p > (int64_t(1) << 31) - 1) return fail(IHT_EINVAL, "iht_project: p out of range");
  if (k < 1 || k > p || k > IHT_MAX_K) return fail(IHT_EINVAL, "iht_project: k out of range");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TopkArea* Ap = project_area();
  if (!Ap) return fail(IHT_ENOMEM, "iht_project: work area");
  TopkArea& A = *Ap;
  int rc = A.ensure(p, st);
  if (rc) return rc;
  HIPCHK(launch_zero_u32(A.tw.state + 3, 1, st));
  DevBuf vals;
  HIPCHK(vals.ensure((size_t)k * 8));
  HIPCHK(launch_topk_w(w, p, k, A.tw, support, vals.as<double>(), st));
  if (w_out) {
    HIPCHK(launch_fill(w_out, p, 0.0, st));
    HIPCHK(launch_scatter(support, vals.as<double>(), k, w_out, st));
  }
  uint32_t err = 0;
  HIPCHK(hipMemcpyAsync(&err, A.tw.state + 3, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err & 1u) return fail(IHT_ENONFINITE, "iht_project: non-finite entry in w");
  if (err & 2u) return fail(IHT_EDEVICE, "iht_project: internal top-k count mismatch");
  return IHT_OK;
}

int iht_fit(const iht_geno* g, const iht_stats* s, const double* y, const float* Z, int32_t cz, int32_t intercept, int32_t k,
            const iht_opts* opts, int64_t* support, double* beta_S, double* beta_cov, double* loss_trace, int32_t* n_iter,
            void* stream) {
  iht_opts o;
  iht_opts_default(&o);
  if (opts) o = *opts;
  if (!g || !s || !y || !support || !beta_S || !loss_trace || !n_iter) return fail(IHT_EINVAL, "iht_fit: NULL argument");
  if (s->geno != g) return fail(IHT_EINVAL, "iht_fit: stats belong to another genotype handle");
  const Layout& L = g->L;
  const int32_t icpt = intercept ? 1 : 0;
  const int32_t nc = cz + icpt;
  if (cz < 0 || (cz > 0 && !Z) || nc > kMaxUnpenalized) return fail(IHT_EINVAL, "iht_fit: bad covariates");
  if (nc > 0 && !beta_cov) return fail(IHT_EINVAL, "iht_fit: beta_cov is NULL");
  if (k < 1 || k > L.p || k > IHT_MAX_K) return fail(IHT_EINVAL, "iht_fit: k out of range");
  if (o.max_iter < 0 || o.max_backtrack < 0 || !(o.c > 0.0 && o.c < 1.0) || !(o.shrink > 0.0 && o.shrink < 1.0) ||
      !(o.tol >= 0.0) || (o.precision != IHT_FP64 && o.precision != IHT_FP32))
    return fail(IHT_EINVAL, "iht_fit: bad options");
  *n_iter = 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  FitWork& W = const_cast<iht_geno*>(g)->fit;
  const size_t kb = (size_t)k;
  HIPCHK(W.beta.ensure(L.p * 8));
  HIPCHK(W.g.ensure(L.p * 8));
  const size_t pb = gradient_partial_bytes(L);
  if (pb) HIPCHK(W.partial.ensure(pb));
  HIPCHK(W.r.ensure(L.n_pad * 8));
  HIPCHK(W.S.ensure(kb * 8));
  HIPCHK(W.Sp.ensure(kb * 8));
  HIPCHK(W.betap.ensure(kb * 8));
  HIPCHK(W.Xs.ensure(kb * L.n_pad * 8));
  HIPCHK(W.Xp.ensure(kb * L.n_pad * 8));
  HIPCHK(W.bc.ensure(kMaxUnpenalized * 8));
  HIPCHK(W.bcp.ensure(kMaxUnpenalized * 8));
  HIPCHK(W.gc.ensure(kMaxUnpenalized * 8));
  HIPCHK(W.fs.ensure(sizeof(FitState)));
  HIPCHK(W.bt.ensure(3 * kb * 8));
  if (int rc = W.topk.ensure(L.p, st)) return rc;

  double* beta = W.beta.as<double>();
  double* gr = W.g.as<double>();
  double* bc = W.bc.as<double>();
  double* bcp = W.bcp.as<double>();
  double* gc = W.gc.as<double>();
  FitState* fs = W.fs.as<FitState>();
  int64_t* S = W.S.as<int64_t>();
  int64_t* Sp = W.Sp.as<int64_t>();
  double* Xs = W.Xs.as<double>();
  double* Xp = W.Xp.as<double>();
  const double* mask = s->mask.as<double>();
  const double* u = s->u.as<double>();
  const double* v = s->v.as<double>();
  const uint8_t* tiled = g->tiled.as<uint8_t>();
  const Unpen U{Z, cz, icpt};
  FitState h{};

  auto read_state = [&]() -> int {
    HIPCHK(hipMemcpyAsync(&h, fs, sizeof(FitState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return IHT_OK;
  };

  // Initialisation: beta = 0, r = y on T, g = A^T r, S = top-k |g|.
  HIPCHK(launch_fill(beta, L.p, 0.0, st));
  HIPCHK(launch_fill(bc, kMaxUnpenalized, 0.0, st));
  HIPCHK(launch_zero_u32(W.topk.tw.state + 3, 1, st));
  HIPCHK(launch_check_finite(y, Z, L.n, cz, mask, fs, st));
  HIPCHK(launch_residual(y, Xs, W.betap.as<double>(), 0, U, bc, mask, L, W.r.as<double>(), gc, loss_trace, 0, fs, nullptr, st));
  HIPCHK(launch_gradient(tiled, L, W.r.as<double>(), mask, s->nT, u, v, fs, o.precision, gr, W.partial.as<double>(), nullptr, st));
  HIPCHK(launch_fill(&fs->mu, 1, 1.0, st));  // top-k of |0 + 1*g| = |g|
  HIPCHK(launch_topk_step(beta, gr, &fs->mu, L.p, k, W.topk.tw, S, nullptr, st));
  HIPCHK(launch_decode_cols(tiled, L, S, k, u, v, mask, Xs, st));
  if (int rc = read_state()) return rc;
  if (h.nonfinite) return fail(IHT_ENONFINITE, "iht_fit: non-finite y or Z inside the subject set");

  // One iteration is enqueued speculatively: step size, proposal, backtracking test, and then the
  // residual/loss, gradient and commit kernels gated on the device flag fs->go (proposal accepted
  // or support unchanged). One host synchronisation per iteration reads the flags; only when the
  // proposal needed backtracking does the host run the halving loop and re-enqueue the gated tail.
  const int32_t* go = &fs->go;
  int status = IHT_NOT_CONVERGED;
  int32_t m = 0;
  uint32_t terr = 0;
  for (; m < o.max_iter; ++m) {
    HIPCHK(launch_mu(Xs, S, k, gr, U, gc, mask, L, fs, st));
    HIPCHK(launch_topk_step(beta, gr, &fs->mu, L.p, k, W.topk.tw, Sp, W.betap.as<double>(), st));
    HIPCHK(launch_decode_cols(tiled, L, Sp, k, u, v, mask, Xp, st));
    HIPCHK(launch_bt_check(S, Xs, Sp, Xp, W.betap.as<double>(), k, beta, U, bc, gc, bcp, o.c, mask, L, fs, W.bt.as<double>(),
                           st));
    HIPCHK(launch_residual(y, Xp, W.betap.as<double>(), k, U, bcp, mask, L, W.r.as<double>(), gc, loss_trace, m + 1, fs, go,
                           st));
    HIPCHK(launch_gradient(tiled, L, W.r.as<double>(), mask, s->nT, u, v, fs, o.precision, gr, W.partial.as<double>(), go, st));
    HIPCHK(launch_commit(S, Sp, W.betap.as<double>(), k, beta, bc, bcp, nc, o.tol, fs, go, st));
    if (int rc = read_state()) return rc;
    if (h.den_zero) {
      status = IHT_OK;
      break;
    }
    if (!h.go) {
      int nbt = 0;
      bool stalled = false;
      while (!h.same && !h.accept) {
        if (nbt == o.max_backtrack) {
          stalled = true;
          break;
        }
        HIPCHK(launch_shrink(fs, o.shrink, st));
        ++nbt;
        HIPCHK(launch_topk_step(beta, gr, &fs->mu, L.p, k, W.topk.tw, Sp, W.betap.as<double>(), st));
        HIPCHK(launch_decode_cols(tiled, L, Sp, k, u, v, mask, Xp, st));
        HIPCHK(launch_bt_check(S, Xs, Sp, Xp, W.betap.as<double>(), k, beta, U, bc, gc, bcp, o.c, mask, L, fs,
                               W.bt.as<double>(), st));
        if (int rc = read_state()) return rc;
      }
      if (stalled) {
        status = IHT_STALLED;
        break;
      }
      HIPCHK(launch_residual(y, Xp, W.betap.as<double>(), k, U, bcp, mask, L, W.r.as<double>(), gc, loss_trace, m + 1, fs, go,
                             st));
      HIPCHK(launch_gradient(tiled, L, W.r.as<double>(), mask, s->nT, u, v, fs, o.precision, gr, W.partial.as<double>(), go,
                             st));
      HIPCHK(launch_commit(S, Sp, W.betap.as<double>(), k, beta, bc, bcp, nc, o.tol, fs, go, st));
      if (int rc = read_state()) return rc;
    }
    std::swap(Xs, Xp);
    if (h.conv) {
      status = IHT_OK;
      ++m;
      break;
    }
  }
  HIPCHK(launch_output(S, k, beta, bc, nc, support, beta_S, beta_cov, st));
  HIPCHK(hipMemcpyAsync(&terr, W.topk.tw.state + 3, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (terr) return fail(IHT_EDEVICE, "iht_fit: internal top-k error");
  *n_iter = m;
  return status;
}

}  // extern "C"
