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
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "iht_host.h"

using namespace iht;

extern "C" {

void iht_opts_default(iht_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_iter = 200;
  o->max_backtrack = 50;
  o->c = 0.01;
  o->shrink = 0.5;
  o->precision = IHT_FP64;
  o->mixed_tol = 1e-6;
  o->polish_iter = 200;
  o->family = IHT_GAUSSIAN;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
}

size_t iht_workspace_bytes_batch(int64_t n, int64_t p, int32_t T, int32_t kmax, int32_t c, int32_t precision) {
  if (n < 1 || p < 1 || T < 1 || kmax < 1 || c < 0 || c > kMaxUnpenalized) return 0;
  return SolveWork::workspace_bytes(make_layout(n, p), T, kmax, c, precision == IHT_MIXED_I8);
}

size_t iht_workspace_bytes(int64_t n, int64_t p, int32_t k, int32_t c, int32_t precision) {
  return iht_workspace_bytes_batch(n, p, 1, k, c, precision);
}

const char* iht_last_error(void) { return last_error_text().c_str(); }

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

}  // extern "C"

namespace {

size_t tiled_bytes_of(const Layout& L) { return (size_t)L.ntiles * (size_t)L.p_pad * kSegBytes; }

// iht_geno_create and iht_geno_create_in: the re-tiled matrix in memory of the handle's own, or in
// the caller's dst (borrowed) when dst is not NULL.
int geno_make(const char* who, const uint8_t* bed, int64_t n, int64_t p, int64_t row_bytes, int32_t flags, void* dst,
              uint64_t dst_bytes, void* stream, iht_geno** out) {
  if (!out) return fail(IHT_EINVAL, std::string(who) + ": out is NULL");
  *out = nullptr;
  if (!bed) return fail(IHT_EINVAL, std::string(who) + ": bed is NULL");
  if (n < 1 || p < 1 || n > (int64_t(1) << 24) || p > (int64_t(1) << 28) - kSnpAlign)
    return fail(IHT_EINVAL, std::string(who) + ": n or p out of range");
  if (row_bytes < (n + 3) / 4) return fail(IHT_EINVAL, std::string(who) + ": row_bytes < ceil(n/4)");
  if (flags != IHT_HOST_PTR && flags != IHT_DEVICE_PTR) return fail(IHT_EINVAL, std::string(who) + ": bad flags");
  const Layout L0 = make_layout(n, p);
  if (dst) {
    if ((reinterpret_cast<uintptr_t>(dst) & 255u) != 0) return fail(IHT_EINVAL, std::string(who) + ": dst not 256-byte aligned");
    if (dst_bytes < tiled_bytes_of(L0))
      return fail(IHT_EINVAL, std::string(who) + ": dst holds " + std::to_string(dst_bytes) + " bytes, the matrix needs " +
                                  std::to_string(tiled_bytes_of(L0)));
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_geno* G = new (std::nothrow) iht_geno();
  if (!G) return fail(IHT_ENOMEM, std::string(who) + ": host allocation");
  int rc = IHT_OK;
  do {
    hipError_t e = hipGetDevice(&G->device);
    if (e != hipSuccess) { rc = hip_fail(e, "hipGetDevice"); break; }
    G->L = L0;
    if (dst) {
      G->tiled.borrow(dst, tiled_bytes_of(G->L));
    } else {
      e = G->tiled.ensure(tiled_bytes_of(G->L));
      if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(tiled)"); break; }
    }
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

}  // namespace

extern "C" {

int iht_geno_create(const uint8_t* bed, int64_t n, int64_t p, int64_t row_bytes, int32_t flags, void* stream, iht_geno** out) {
  return geno_make("iht_geno_create", bed, n, p, row_bytes, flags, nullptr, 0, stream, out);
}

uint64_t iht_geno_bytes(int64_t n, int64_t p) {
  if (n < 1 || p < 1 || n > (int64_t(1) << 24) || p > (int64_t(1) << 28) - kSnpAlign) return 0;
  return tiled_bytes_of(make_layout(n, p));
}

int iht_geno_create_in(const uint8_t* bed, int64_t n, int64_t p, int64_t row_bytes, void* dst, uint64_t dst_bytes,
                       void* stream, iht_geno** out) {
  if (!dst) {
    if (out) *out = nullptr;
    return fail(IHT_EINVAL, "iht_geno_create_in: dst is NULL");
  }
  return geno_make("iht_geno_create_in", bed, n, p, row_bytes, IHT_DEVICE_PTR, dst, dst_bytes, stream, out);
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

}  // extern "C"

namespace {

// u [p], v [p], the FP64 subject mask [n_pad], then the subject bits [ntiles]
size_t stats_bytes_of(const Layout& L) { return (size_t)(2 * L.p + L.n_pad) * 8 + (size_t)L.ntiles * 4; }

// iht_stats_create and iht_stats_create_in: the statistics in memory of the handle's own, or in the
// caller's dst (borrowed) when dst is not NULL.
int stats_make(const char* who, const iht_geno* g, const uint8_t* subset, void* dst, uint64_t dst_bytes, void* stream,
               iht_stats** out) {
  if (!out) return fail(IHT_EINVAL, std::string(who) + ": out is NULL");
  *out = nullptr;
  if (!g) return fail(IHT_EINVAL, std::string(who) + ": NULL geno");
  const Layout& L = g->L;
  if (dst) {
    if ((reinterpret_cast<uintptr_t>(dst) & 255u) != 0) return fail(IHT_EINVAL, std::string(who) + ": dst not 256-byte aligned");
    if (dst_bytes < stats_bytes_of(L))
      return fail(IHT_EINVAL, std::string(who) + ": dst holds " + std::to_string(dst_bytes) + " bytes, the statistics need " +
                                  std::to_string(stats_bytes_of(L)));
  }
  // the subject bits of a subset (the whole set is built on the device)
  std::vector<uint32_t> bits;
  int64_t nT = L.n;
  if (subset) {
    bits.assign(L.ntiles, 0u);
    nT = 0;
    for (int64_t i = 0; i < L.n; ++i) {
      const uint8_t m = subset[i];
      if (m > 1) return fail(IHT_EINVAL, std::string(who) + ": subset entries must be 0 or 1");
      if (m) {
        bits[i / kTileSubjects] |= uint32_t(1) << (i % kTileSubjects);
        ++nT;
      }
    }
    if (nT < 1) return fail(IHT_EINVAL, std::string(who) + ": empty subject set");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_stats* S = new (std::nothrow) iht_stats();
  if (!S) return fail(IHT_ENOMEM, std::string(who) + ": host allocation");
  S->geno = g;
  S->nT = nT;
  int rc = IHT_OK;
  do {
    const size_t fbytes = (size_t)(2 * L.p + L.n_pad) * 8;
    hipError_t e = hipSuccess;
    if (dst) {
      S->buf.borrow(dst, stats_bytes_of(L));
    } else if ((e = S->buf.ensure(stats_bytes_of(L))) != hipSuccess) {
      rc = hip_fail(e, "hipMalloc(stats)");
      break;
    }
    S->u = S->buf.as<double>();
    S->v = S->u + L.p;
    S->mask = S->v + L.p;
    S->mask_bits = reinterpret_cast<uint32_t*>(S->buf.as<char>() + fbytes);
    if (subset) {
      // pageable source: the copy has read it when the stream is synchronised below
      if ((e = hipMemcpyAsync(S->mask_bits, bits.data(), L.ntiles * 4, hipMemcpyHostToDevice, st)) != hipSuccess) {
        rc = hip_fail(e, "hipMemcpyAsync(subject bits)");
        break;
      }
    }
    if ((e = launch_subject_mask(L, subset != nullptr, S->mask_bits, S->mask, st)) != hipSuccess ||
        (e = launch_stats(g->tiled.as<uint8_t>(), L, S->mask_bits, nT, S->u, S->v, st)) != hipSuccess) {
      rc = hip_fail(e, "stats launch");
      break;
    }
    if (subset && (e = hipStreamSynchronize(st)) != hipSuccess) {
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

}  // namespace

extern "C" {

int iht_stats_create(const iht_geno* g, const uint8_t* subset, void* stream, iht_stats** out) {
  return stats_make("iht_stats_create", g, subset, nullptr, 0, stream, out);
}

uint64_t iht_stats_bytes(const iht_geno* g) { return g ? stats_bytes_of(g->L) : 0; }

int iht_stats_create_in(const iht_geno* g, const uint8_t* subset, void* dst, uint64_t dst_bytes, void* stream,
                        iht_stats** out) {
  if (!dst) {
    if (out) *out = nullptr;
    return fail(IHT_EINVAL, "iht_stats_create_in: dst is NULL");
  }
  return stats_make("iht_stats_create_in", g, subset, dst, dst_bytes, stream, out);
}

int iht_stats_destroy(iht_stats* s) {
  delete s;
  return IHT_OK;
}

int iht_stats_read(const iht_stats* s, double* u, double* v, void* stream) {
  if (!s) return fail(IHT_EINVAL, "iht_stats_read: NULL handle");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t b = (size_t)s->geno->L.p * 8;
  if (u) HIPCHK(hipMemcpyAsync(u, s->u, b, hipMemcpyDeviceToDevice, st));
  if (v) HIPCHK(hipMemcpyAsync(v, s->v, b, hipMemcpyDeviceToDevice, st));
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
  HIPCHK(G->partial.ensure(gradient_work_bytes(L)));
  FitState* fs = G->state.as<FitState>();
  HIPCHK(launch_gradient(g->tiled.as<uint8_t>(), L, r, s->mask, s->nT, s->u, s->v, fs,
                         precision, grad, G->partial.as<double>(), nullptr, st));
  return IHT_OK;
}

// Work area of iht_project: one per (thread, device), kept for the life of the process.
int iht_gradient_batch(const iht_geno* g, const iht_stats* const* stats, int32_t T, const double* R, double* G, void* stream) {
  if (!g || !stats || !R || !G) return fail(IHT_EINVAL, "iht_gradient_batch: NULL argument");
  if (T < 1 || T > 65535) return fail(IHT_EINVAL, "iht_gradient_batch: T out of range");
  if (g->L.n > kBatchMaxSubjects)
    return fail(IHT_EUNSUPPORTED, "iht_gradient_batch: n > " + std::to_string(kBatchMaxSubjects) + " subjects");
  std::vector<BatchSolve> sv((size_t)T);
  for (int32_t t = 0; t < T; ++t) {
    if (!stats[t]) return fail(IHT_EINVAL, "iht_gradient_batch: NULL stats handle");
    if (stats[t]->geno != g) return fail(IHT_EINVAL, "iht_gradient_batch: stats belong to another genotype handle");
    sv[t] = BatchSolve{stats[t]->u, stats[t]->v, stats[t]->mask, stats[t]->nT};
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
  HIPCHK(launch_gradient_batch(g->tiled.as<uint8_t>(), L, R, L.n, T, Gh->batch_sv.as<BatchSolve>(), nullptr, nullptr,
                               Gh->batch_r8.as<int8_t>(), Gh->batch_scale.as<double>(), Gh->batch_rsum.as<double>(), G, L.p,
                               st));
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

static int project(const char* who, const double* w, int64_t p, int32_t k, const int64_t* hint, int64_t* support,
                   double* w_out, void* stream) {
  if (!w || !support) return fail(IHT_EINVAL, std::string(who) + ": NULL argument");
  if (p < 1 || p > (int64_t(1) << 31) - 1) return fail(IHT_EINVAL, std::string(who) + ": p out of range");
  if (k < 1 || k > p || k > IHT_MAX_K) return fail(IHT_EINVAL, std::string(who) + ": k out of range");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TopkArea* Ap = project_area();
  if (!Ap) return fail(IHT_ENOMEM, std::string(who) + ": work area");
  TopkArea& A = *Ap;
  if (int rc = A.ensure(p, 1, st)) return rc;
  HIPCHK(launch_topk_clear_errors(A.small.as<uint32_t>(), 1, nullptr, st));
  DevBuf vals;
  HIPCHK(vals.ensure((size_t)k * 8));
  TopkJob J{};
  J.g = w;
  J.ld = p;
  J.k0 = k;
  J.kmax = k;
  J.out = support;
  J.ldo = k;
  J.vals = vals.as<double>();
  J.small = A.small.as<uint32_t>();
  J.cand_key = A.cand_key();
  J.cand_idx = A.cand_idx();
  J.cap = A.cap;
  J.prev = hint;
  J.ldprev = k;
  HIPCHK(launch_topk(J, p, 1, st));
  if (w_out) {
    HIPCHK(launch_fill(w_out, p, 0.0, st));
    HIPCHK(launch_scatter(support, vals.as<double>(), k, p, w_out, st));
  }
  uint32_t err = 0;
  HIPCHK(hipMemcpyAsync(&err, A.small.as<uint32_t>() + kTopkErrorWord, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err & 1u) return fail(IHT_ENONFINITE, std::string(who) + ": non-finite entry in w");
  if (err & 4u) return fail(IHT_EINVAL, std::string(who) + ": hint does not hold k distinct indices");
  if (err & 2u) return fail(IHT_EDEVICE, std::string(who) + ": internal top-k count mismatch");
  return IHT_OK;
}

int iht_project(const double* w, int64_t p, int32_t k, int64_t* support, double* w_out, void* stream) {
  return project("iht_project", w, p, k, nullptr, support, w_out, stream);
}

int iht_project_hint(const double* w, int64_t p, int32_t k, const int64_t* hint, int64_t* support, double* w_out,
                     void* stream) {
  if (!hint) return fail(IHT_EINVAL, "iht_project_hint: NULL argument");
  return project("iht_project_hint", w, p, k, hint, support, w_out, stream);
}


}  // extern "C"

// ------------------------------------------------------------------------------------------------
// The solve driver behind iht_fit and iht_fit_batch. The loop follows Methods, eq. (ihta) with the
// normalised step and the omega rule of "IHT step sizes" for every solve of the set at once; all
// arithmetic runs in the device kernels. Each iteration is enqueued speculatively (step size,
// proposal, backtracking test, then residual, gradient and commit for the solves whose proposal was
// accepted) and the host reads the solves' flags once; only when some solve needs a halving does it
// run further rounds for those solves.
namespace {

struct FitArgs {
  const iht_geno* g;
  const iht_stats* const* stats;
  int32_t T;
  const double* Y;
  int64_t ldy;
  Unpen U;
  const int32_t* ks;  // host
  iht_opts o;
  int64_t* support;
  double* beta_S;
  double* beta_cov;
  double* trace;
  int32_t* n_iter;  // host
  int32_t* status;  // host
  hipStream_t st;
};

int run_fit(const FitArgs& A) {
  const iht_geno* g = A.g;
  const int32_t T = A.T;
  int32_t kmax = 0;
  for (int32_t t = 0; t < T; ++t) kmax = std::max(kmax, A.ks[t]);
  const int32_t nc = A.U.cz + A.U.icpt;
  std::vector<BatchSolve> sv((size_t)T);
  std::vector<OutRow> rows((size_t)T);
  for (int32_t t = 0; t < T; ++t) {
    sv[t] = BatchSolve{A.stats[t]->u, A.stats[t]->v, A.stats[t]->mask, A.stats[t]->nT};
    rows[t] = OutRow{A.support + (size_t)t * kmax, A.beta_S + (size_t)t * kmax,
                     A.beta_cov ? A.beta_cov + (size_t)t * nc : nullptr, nullptr, kmax};
  }
  Engine E;
  // device state: the handle's own (allocated on first use, grown and reused), or the caller's workspace
  iht_geno* G = const_cast<iht_geno*>(g);
  SolveWork borrowed;
  SolveWork* W = A.o.workspace ? &borrowed : &G->fit;
  if (int rc = E.setup(g, W, &G->fit_stage, T, kmax, A.U, A.Y, A.ldy, A.trace, A.o, A.st, A.o.workspace,
                       (size_t)A.o.workspace_bytes))
    return rc;
  if (int rc = E.admit(A.ks, sv.data(), nullptr)) return rc;
  for (int32_t turn = 0; turn <= A.o.max_iter && E.count_active() > 0; ++turn)
    if (int rc = E.turn()) return rc;
  if (int rc = E.retire(nullptr, rows.data())) return rc;
  int worst = IHT_OK;
  for (int32_t t = 0; t < T; ++t) {
    const FitState& f = E.state(t);
    if (E.topk_error(t) && !f.nonfinite)
      return fail(IHT_EDEVICE, "internal top-k error (solve " + std::to_string(t) + ", flags " +
                                   std::to_string(E.topk_error(t)) + ")");
    A.n_iter[t] = f.iter;
    A.status[t] = f.status;
    if (f.status < 0)
      worst = std::min(worst, f.status);
    else if (worst >= 0)
      worst = std::max(worst, f.status);
  }
  return worst;
}

}  // namespace

extern "C" {

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
  if (int rc = check_opts(o, "iht_fit")) return rc;
  *n_iter = 0;
  int32_t status = IHT_OK;
  const iht_stats* const stats[1] = {s};
  FitArgs A{g, stats, 1, y, L.n, Unpen{Z, cz, icpt}, &k, o, support, beta_S, nc ? beta_cov : nullptr, loss_trace, n_iter,
            &status, reinterpret_cast<hipStream_t>(stream)};
  const int rc = run_fit(A);
  if (rc == IHT_ENONFINITE) return fail(IHT_ENONFINITE, "iht_fit: non-finite y or Z inside the subject set");
  return rc;
}

int iht_fit_batch(const iht_geno* g, const iht_stats* const* stats, int32_t T, const double* Y, int64_t ldy, const float* Z,
                  int32_t cz, int32_t intercept, const int32_t* ks, const iht_opts* opts, int64_t* support, double* beta_S,
                  double* beta_cov, double* loss_trace, int32_t* n_iter, int32_t* status, void* stream) {
  iht_opts o;
  iht_opts_default(&o);
  if (opts) o = *opts;
  if (!g || !stats || !Y || !ks || !support || !beta_S || !loss_trace || !n_iter || !status)
    return fail(IHT_EINVAL, "iht_fit_batch: NULL argument");
  if (T < 1 || T > 65535) return fail(IHT_EINVAL, "iht_fit_batch: T out of range");
  const Layout& L = g->L;
  if (ldy < L.n) return fail(IHT_EINVAL, "iht_fit_batch: ldy < n");
  const int32_t icpt = intercept ? 1 : 0;
  const int32_t nc = cz + icpt;
  if (cz < 0 || (cz > 0 && !Z) || nc > kMaxUnpenalized) return fail(IHT_EINVAL, "iht_fit_batch: bad covariates");
  if (nc > 0 && !beta_cov) return fail(IHT_EINVAL, "iht_fit_batch: beta_cov is NULL");
  for (int32_t t = 0; t < T; ++t) {
    if (!stats[t]) return fail(IHT_EINVAL, "iht_fit_batch: NULL stats handle");
    if (stats[t]->geno != g) return fail(IHT_EINVAL, "iht_fit_batch: stats belong to another genotype handle");
    if (ks[t] < 1 || ks[t] > L.p || ks[t] > IHT_MAX_K) return fail(IHT_EINVAL, "iht_fit_batch: k out of range");
  }
  if (int rc = check_opts(o, "iht_fit_batch")) return rc;
  for (int32_t t = 0; t < T; ++t) n_iter[t] = 0;
  FitArgs A{g, stats, T, Y, ldy, Unpen{Z, cz, icpt}, ks, o, support, beta_S, nc ? beta_cov : nullptr, loss_trace, n_iter,
            status, reinterpret_cast<hipStream_t>(stream)};
  const int rc = run_fit(A);
  if (rc == IHT_ENONFINITE) return fail(IHT_ENONFINITE, "iht_fit_batch: non-finite y or Z inside a solve's subject set");
  return rc;
}


int iht_cv(const iht_geno* g, const double* y, const float* Z, int32_t cz, int32_t intercept, const uint8_t* folds, int32_t q,
           const int32_t* ks, int32_t r, const iht_opts* opts, double* mse, int32_t* k_best, int64_t* support, double* beta_S,
           double* beta_cov, double* loss_trace, int32_t* n_iter, void* stream) {
  iht_opts o;
  iht_opts_default(&o);
  if (opts) o = *opts;
  o.workspace = nullptr;  // the training batch and the refit use the handle's own memory
  o.workspace_bytes = 0;
  if (!g || !y || !folds || !ks || !mse || !k_best || !support || !beta_S || !loss_trace || !n_iter)
    return fail(IHT_EINVAL, "iht_cv: NULL argument");
  const Layout& L = g->L;
  if (q < 2 || q > 64 || r < 1 || (int64_t)q * r > 65535) return fail(IHT_EINVAL, "iht_cv: q or r out of range");
  const int32_t icpt = intercept ? 1 : 0;
  const int32_t nc = cz + icpt;
  if (cz < 0 || (cz > 0 && !Z) || nc > kMaxUnpenalized) return fail(IHT_EINVAL, "iht_cv: bad covariates");
  if (nc > 0 && !beta_cov) return fail(IHT_EINVAL, "iht_cv: beta_cov is NULL");
  int32_t kmax = 0;
  for (int32_t a = 0; a < r; ++a) {
    if (ks[a] < 1 || ks[a] > L.p || ks[a] > IHT_MAX_K) return fail(IHT_EINVAL, "iht_cv: k out of range");
    kmax = std::max(kmax, ks[a]);
  }
  if (int rc = check_opts(o, "iht_cv")) return rc;
  if (o.family != IHT_GAUSSIAN) return fail(IHT_EUNSUPPORTED, "iht_cv: least squares only (held-out MSE)");
  std::vector<int64_t> count(q, 0);
  for (int64_t i = 0; i < L.n; ++i) {
    if (folds[i] >= q) return fail(IHT_EINVAL, "iht_cv: fold index >= q");
    count[folds[i]]++;
  }
  for (int32_t f = 0; f < q; ++f)
    if (count[f] == 0 || count[f] == L.n) return fail(IHT_EINVAL, "iht_cv: every fold and its complement must be non-empty");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  *n_iter = 0;

  // training statistics of each fold (the subjects outside it) and of the whole set
  std::vector<iht_stats*> fstats(q, nullptr);
  iht_stats* full = nullptr;
  auto release = [&]() {
    for (iht_stats* s : fstats) iht_stats_destroy(s);
    iht_stats_destroy(full);
  };
  std::vector<uint8_t> sub(L.n);
  for (int32_t f = 0; f < q; ++f) {
    for (int64_t i = 0; i < L.n; ++i) sub[i] = folds[i] != f ? 1 : 0;
    if (int rc = iht_stats_create(g, sub.data(), stream, &fstats[f])) {
      release();
      return rc;
    }
  }
  if (int rc = iht_stats_create(g, nullptr, stream, &full)) {
    release();
    return rc;
  }

  // the q x r training solves (solve f * r + a: fold f held out, model size ks[a]) in one batch, all
  // reading the same trait (row stride 0)
  const int32_t T = q * r;
  const size_t Tz = (size_t)T;
  std::vector<const iht_stats*> stats(Tz);
  std::vector<int32_t> kss(Tz);
  std::vector<BatchSolve> sv(Tz);
  for (int32_t f = 0; f < q; ++f)
    for (int32_t a = 0; a < r; ++a) {
      const int32_t t = f * r + a;
      stats[t] = fstats[f];
      kss[t] = ks[a];
      sv[t] = BatchSolve{fstats[f]->u, fstats[f]->v, fstats[f]->mask, fstats[f]->nT};
    }
  const int32_t nblk = (int32_t)((L.n + 255) / 256);
  DevBuf d_sup, d_bS, d_bc, d_trace, d_folds, d_count, d_ks_solve, d_ks_path, d_part, d_mse, d_kb, d_sv;
  std::vector<int32_t> it_t(Tz), st_t(Tz);
  int rc = IHT_OK;
  do {
    hipError_t e;
    if ((e = d_sup.ensure(Tz * kmax * 8)) != hipSuccess || (e = d_bS.ensure(Tz * kmax * 8)) != hipSuccess ||
        (e = d_bc.ensure(Tz * std::max(nc, 1) * 8)) != hipSuccess ||
        (e = d_trace.ensure(Tz * (size_t)(o.max_iter + 1) * 8)) != hipSuccess || (e = d_folds.ensure(L.n)) != hipSuccess ||
        (e = d_count.ensure((size_t)q * 8)) != hipSuccess || (e = d_ks_solve.ensure(Tz * 4)) != hipSuccess ||
        (e = d_ks_path.ensure((size_t)r * 4)) != hipSuccess || (e = d_part.ensure(Tz * nblk * 8)) != hipSuccess ||
        (e = d_mse.ensure((size_t)r * q * 8)) != hipSuccess || (e = d_kb.ensure(4)) != hipSuccess ||
        (e = d_sv.ensure(Tz * sizeof(BatchSolve))) != hipSuccess) {
      rc = hip_fail(e, "hipMalloc(cv)");
      break;
    }
    FitArgs A{g, stats.data(), T, y, 0, Unpen{Z, cz, icpt}, kss.data(), o, d_sup.as<int64_t>(), d_bS.as<double>(),
              nc ? d_bc.as<double>() : nullptr, d_trace.as<double>(), it_t.data(), st_t.data(), st};
    rc = run_fit(A);
    if (rc < 0) break;
    // held-out errors, the MSE table and the chosen size; the copies go to the caller's stream and
    // their host arrays stay alive until the stream is synchronised below
    if ((e = hipMemcpyAsync(d_folds.p, folds, L.n, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_count.p, count.data(), (size_t)q * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_ks_solve.p, kss.data(), Tz * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_ks_path.p, ks, (size_t)r * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_sv.p, sv.data(), Tz * sizeof(BatchSolve), hipMemcpyHostToDevice, st)) != hipSuccess) {
      rc = hip_fail(e, "hipMemcpyAsync(cv)");
      break;
    }
    if ((e = cv_heldout_mse(g->tiled.as<uint8_t>(), L, d_folds.as<uint8_t>(), q, r, d_sv.as<BatchSolve>(),
                            d_ks_solve.as<int32_t>(), d_ks_path.as<int32_t>(), d_sup.as<int64_t>(), d_bS.as<double>(), kmax,
                            d_bc.as<double>(), std::max(nc, 1), Unpen{Z, cz, icpt}, y, d_count.as<int64_t>(),
                            d_part.as<double>(), d_mse.as<double>(), d_kb.as<int32_t>(), st)) != hipSuccess) {
      rc = hip_fail(e, "cv launch");
      break;
    }
    if ((e = hipMemcpyAsync(mse, d_mse.p, (size_t)r * q * 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(k_best, d_kb.p, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      rc = hip_fail(e, "cv results");
      break;
    }
    // the refit on every subject with the chosen size
    int32_t status = IHT_OK;
    const iht_stats* s1[1] = {full};
    FitArgs B{g, s1, 1, y, L.n, Unpen{Z, cz, icpt}, k_best, o, support, beta_S, nc ? beta_cov : nullptr, loss_trace, n_iter,
              &status, st};
    rc = run_fit(B);
  } while (0);
  release();
  if (rc == IHT_ENONFINITE) return fail(IHT_ENONFINITE, "iht_cv: non-finite y or Z");
  return rc;
}

int iht_predict(const iht_geno* g, const iht_stats* s, const int64_t* support, const double* beta_S, int32_t k,
                const float* Z, int32_t cz, int32_t intercept, const double* beta_cov, double* out, void* stream) {
  if (!g || !s || !out || (k > 0 && (!support || !beta_S))) return fail(IHT_EINVAL, "iht_predict: NULL argument");
  if (s->geno != g) return fail(IHT_EINVAL, "iht_predict: stats belong to another genotype handle");
  const Layout& L = g->L;
  if (k < 0 || k > L.p) return fail(IHT_EINVAL, "iht_predict: k out of range");
  const int32_t icpt = intercept ? 1 : 0;
  const int32_t nc = cz + icpt;
  if (cz < 0 || (cz > 0 && !Z) || nc > kMaxUnpenalized || (nc > 0 && !beta_cov))
    return fail(IHT_EINVAL, "iht_predict: bad covariates");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  iht_geno* G = const_cast<iht_geno*>(g);
  HIPCHK(G->pred_err.ensure(4));
  HIPCHK(launch_zero_u32(G->pred_err.as<uint32_t>(), 1, st));
  HIPCHK(launch_predict(g->tiled.as<uint8_t>(), L, support, beta_S, k, s->u, s->v, Unpen{Z, cz, icpt}, beta_cov, out,
                        G->pred_err.as<uint32_t>(), st));
  uint32_t err = 0;
  HIPCHK(hipMemcpyAsync(&err, G->pred_err.p, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err) return fail(IHT_EINVAL, "iht_predict: support index outside [0, p)");
  return IHT_OK;
}

int iht_batch_tuning(const iht_geno* g, int32_t T, int32_t* snps_per_block) {
  if (!g || !snps_per_block) return fail(IHT_EINVAL, "iht_batch_tuning: NULL argument");
  if (T < 1 || T > 65535) return fail(IHT_EINVAL, "iht_batch_tuning: T out of range");
  *snps_per_block = batch_tuned_snps(g->L, T);
  return IHT_OK;
}

}  // extern "C"
