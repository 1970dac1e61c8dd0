// iht_serve.hip -- a solve server with continuous batching over one resident genotype matrix.
//
// Requests (a subject set, 1..slots traits, a model size per trait) queue on the host and are
// admitted, in arrival order, whenever enough solve slots and one block of per-subject-set
// statistics are free; the slot state and the statistics blocks are allocated once, inside the
// caller's device-memory budget, so serving allocates nothing. Each step admits what fits (the
// admitted traits' statistics pass and initial state run beside the slots already iterating), runs
// one turn of the engine over every iterating slot, and writes out the solves that finished,
// straight into the request's output buffers. A solve's arithmetic depends only on its own slot
// state, so its result is the same alone and in any mix of other requests.
#include <hip/hip_runtime.h>

#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "iht_host.h"

using namespace iht;

// The server replays each turn's speculative iterations from a HIP graph (int8 matrix-core path).
#ifndef IHT_SERVER_GRAPHS
#define IHT_SERVER_GRAPHS 1
#endif

namespace {

struct Request {
  int64_t id = 0;
  std::vector<uint32_t> bits;  // subject bits [ntiles], empty = every subject
  int64_t nT = 0;
  const double* Y = nullptr;
  int64_t ldy = 0;
  int32_t T = 0;
  std::vector<int32_t> ks;
  int32_t kmax = 0;
  int64_t* support = nullptr;
  double* beta_S = nullptr;
  double* beta_cov = nullptr;
  double* trace = nullptr;
  int32_t* n_iter = nullptr;
  int32_t* status = nullptr;
  int32_t block = -1;  // statistics block while admitted
  int32_t left = 0;    // traits not yet written out
  bool done = false;
};

// u [p], v [p], the FP64 subject mask [n_pad], the subject bits [ntiles] of one subject set
struct StatsBlock {
  double* u = nullptr;
  double* v = nullptr;
  double* mask = nullptr;
  uint32_t* bits = nullptr;
  bool busy = false;
};

// bytes of one block, rounded up so that every block starts 256-byte aligned
size_t stats_block_bytes(const Layout& L) {
  return ((size_t)(2 * L.p + L.n_pad) * 8 + (size_t)L.ntiles * 4 + 255) / 256 * 256;
}

}  // namespace

struct iht_server {
  const iht_geno* g = nullptr;
  hipStream_t st = nullptr;
  iht_opts o{};
  Unpen U{};
  int32_t slots = 0, kmax = 0;
  int64_t budget = 0;
  SolveWork W;
  SolveStage P;
  Engine E;
  DevBuf Y;          // [slots][n] traits of the admitted solves
  DevBuf trace;      // [slots][max_iter + 1] loss traces until written out
  DevBuf pool;       // statistics blocks
  PinnedBuf bits_h;  // [blocks][ntiles] subject bits on their way to the device
  std::vector<StatsBlock> blocks;
  std::vector<int64_t> owner;     // request index of each slot, -1 = free
  std::vector<int32_t> trait;     // trait of each slot within its request
  std::vector<int32_t> ks;        // model size of each slot (1 when free)
  std::vector<BatchSolve> sv;     // subject set of each slot
  std::vector<Request> requests;  // every request ever submitted, by id
  std::deque<int64_t> queue;      // submitted, not yet admitted
  int64_t running = 0, completed = 0, turns = 0, device_bytes = 0;
  int32_t busy = 0;
};

namespace {

// Admits queued requests in arrival order while the one at the head fits.
int admit_queued(iht_server* S) {
  const Layout& L = S->g->L;
  std::vector<uint8_t> admit((size_t)S->slots, 0);
  bool any = false;
  while (!S->queue.empty()) {
    Request& R = S->requests[(size_t)S->queue.front()];
    if (R.T > S->slots - S->busy) break;
    int32_t b = -1;
    for (size_t i = 0; i < S->blocks.size(); ++i)
      if (!S->blocks[i].busy) {
        b = (int32_t)i;
        break;
      }
    if (b < 0) break;
    S->queue.pop_front();
    StatsBlock& B = S->blocks[(size_t)b];
    B.busy = true;
    R.block = b;
    // the subject set's statistics (a pinned row per block: free again only after the request ends)
    const bool have = !R.bits.empty();
    if (have) {
      uint32_t* row = reinterpret_cast<uint32_t*>(S->bits_h.p) + (size_t)b * L.ntiles;
      std::memcpy(row, R.bits.data(), (size_t)L.ntiles * 4);
      HIPCHK(hipMemcpyAsync(B.bits, row, (size_t)L.ntiles * 4, hipMemcpyHostToDevice, S->st));
    }
    HIPCHK(launch_subject_mask(L, have, B.bits, B.mask, S->st));
    HIPCHK(launch_stats(S->g->tiled.as<uint8_t>(), L, B.bits, R.nT, B.u, B.v, S->st));
    std::vector<uint32_t>().swap(R.bits);  // copied to the pinned row: a finished request keeps no bits
    // its traits into free slots
    int32_t j = 0;
    for (int32_t t = 0; t < S->slots && j < R.T; ++t) {
      if (S->owner[t] >= 0) continue;
      S->owner[t] = R.id;
      S->trait[t] = j;
      S->ks[t] = R.ks[j];
      S->sv[t] = BatchSolve{B.u, B.v, B.mask, R.nT};
      HIPCHK(hipMemcpyAsync(S->Y.as<double>() + (size_t)t * L.n, R.Y + (size_t)j * R.ldy, (size_t)L.n * 8,
                            hipMemcpyDeviceToDevice, S->st));
      admit[t] = 1;
      ++j;
    }
    S->busy += R.T;
    R.left = R.T;
    ++S->running;
    any = true;
  }
  if (!any) return IHT_OK;
  return S->E.admit(S->ks.data(), S->sv.data(), admit.data());
}

// Writes out the solves that stopped iterating, and completes the requests whose traits are all out.
int retire_finished(iht_server* S, int32_t* completed) {
  std::vector<uint8_t> flags((size_t)S->slots, 0);
  std::vector<OutRow> rows((size_t)S->slots, OutRow{nullptr, nullptr, nullptr, nullptr, 0});
  const int32_t nc = S->U.cz + S->U.icpt;
  const int64_t ldt = (int64_t)S->o.max_iter + 1;
  bool any = false;
  for (int32_t t = 0; t < S->slots; ++t) {
    if (S->owner[t] < 0 || S->E.state(t).active != 0) continue;
    const Request& R = S->requests[(size_t)S->owner[t]];
    const int32_t j = S->trait[t];
    rows[t] = OutRow{R.support + (size_t)j * R.kmax, R.beta_S + (size_t)j * R.kmax,
                     nc ? R.beta_cov + (size_t)j * nc : nullptr, R.trace + (size_t)j * ldt, R.kmax};
    flags[t] = 1;
    any = true;
  }
  if (!any) return IHT_OK;
  if (int rc = S->E.retire(flags.data(), rows.data())) return rc;
  for (int32_t t = 0; t < S->slots; ++t) {
    if (!flags[t]) continue;
    const FitState& f = S->E.state(t);
    if (S->E.topk_error(t) && !f.nonfinite)
      return fail(IHT_EDEVICE, "iht_server_step: internal top-k error (request " + std::to_string(S->owner[t]) + ")");
    Request& R = S->requests[(size_t)S->owner[t]];
    const int32_t j = S->trait[t];
    R.n_iter[j] = f.iter;
    R.status[j] = f.status;
    S->owner[t] = -1;
    S->ks[t] = 1;
    --S->busy;
    if (--R.left == 0) {
      R.done = true;
      std::vector<int32_t>().swap(R.ks);
      S->blocks[(size_t)R.block].busy = false;
      R.block = -1;
      --S->running;
      ++S->completed;
      ++*completed;
    }
  }
  return IHT_OK;
}

}  // namespace

extern "C" {

int iht_server_create(const iht_geno* g, int32_t slots, int32_t kmax, int64_t hbm_budget, const float* Z, int32_t cz,
                      int32_t intercept, const iht_opts* opts, void* stream, iht_server** out) {
  if (!out) return fail(IHT_EINVAL, "iht_server_create: out is NULL");
  *out = nullptr;
  if (!g) return fail(IHT_EINVAL, "iht_server_create: NULL geno");
  iht_opts o;
  iht_opts_default(&o);
  if (opts) o = *opts;
  o.workspace = nullptr;  // the server allocates its state at creation, inside its budget
  o.workspace_bytes = 0;
  const Layout& L = g->L;
  if (slots < 1 || slots > 65535) return fail(IHT_EINVAL, "iht_server_create: slots out of range");
  if (kmax < 1 || kmax > L.p || kmax > IHT_MAX_K) return fail(IHT_EINVAL, "iht_server_create: kmax out of range");
  const int32_t icpt = intercept ? 1 : 0;
  if (cz < 0 || (cz > 0 && !Z) || cz + icpt > kMaxUnpenalized) return fail(IHT_EINVAL, "iht_server_create: bad covariates");
  if (int rc = check_opts(o, "iht_server_create")) return rc;
  if (o.max_iter < 1) return fail(IHT_EINVAL, "iht_server_create: max_iter must be >= 1");
  iht_server* S = new (std::nothrow) iht_server();
  if (!S) return fail(IHT_ENOMEM, "iht_server_create: host allocation");
  S->g = g;
  S->st = reinterpret_cast<hipStream_t>(stream);
  S->o = o;
  S->U = Unpen{Z, cz, icpt};
  S->slots = slots;
  S->kmax = kmax;
  S->budget = hbm_budget;
  auto bail = [&](int rc) {
    (void)hipStreamSynchronize(S->st);
    delete S;
    return rc;
  };
  hipError_t e;
  if ((e = S->Y.ensure((size_t)slots * (size_t)L.n * 8)) != hipSuccess ||
      (e = S->trace.ensure((size_t)slots * (size_t)(o.max_iter + 1) * 8)) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(server slots)"));
  if (int rc = S->E.setup(g, &S->W, &S->P, slots, kmax, S->U, S->Y.as<double>(), L.n, S->trace.as<double>(), o, S->st))
    return bail(rc);
  S->E.use_graphs(IHT_SERVER_GRAPHS != 0);
  const int64_t slot_bytes = S->W.device_bytes() + (int64_t)S->Y.bytes + (int64_t)S->trace.bytes;
  const int64_t block_bytes = (int64_t)stats_block_bytes(L);
  if (hbm_budget < slot_bytes + block_bytes)
    return bail(fail(IHT_ENOMEM, "iht_server_create: the budget holds less than the slot state (" +
                                     std::to_string(slot_bytes) + " bytes) plus one subject set's statistics (" +
                                     std::to_string(block_bytes) + " bytes)"));
  const int64_t nblocks = std::min<int64_t>(slots, (hbm_budget - slot_bytes) / block_bytes);
  if ((e = S->pool.ensure((size_t)(nblocks * block_bytes))) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(server statistics)"));
  if ((e = S->bits_h.ensure((size_t)nblocks * (size_t)L.ntiles * 4)) != hipSuccess)
    return bail(hip_fail(e, "hipHostMalloc(server subject bits)"));
  S->blocks.resize((size_t)nblocks);
  for (int64_t b = 0; b < nblocks; ++b) {
    char* base = S->pool.as<char>() + b * block_bytes;
    StatsBlock& B = S->blocks[(size_t)b];
    B.u = reinterpret_cast<double*>(base);
    B.v = B.u + L.p;
    B.mask = B.v + L.p;
    B.bits = reinterpret_cast<uint32_t*>(B.mask + L.n_pad);
  }
  S->owner.assign((size_t)slots, -1);
  S->trait.assign((size_t)slots, 0);
  S->ks.assign((size_t)slots, 1);
  // free slots point at a valid (unused) block; every kernel skips them
  S->sv.assign((size_t)slots, BatchSolve{S->blocks[0].u, S->blocks[0].v, S->blocks[0].mask, 1});
  S->device_bytes = slot_bytes + nblocks * block_bytes;
  if ((e = hipStreamSynchronize(S->st)) != hipSuccess) return bail(hip_fail(e, "iht_server_create"));
  *out = S;
  return IHT_OK;
}

int iht_server_submit(iht_server* S, const uint8_t* subset, const double* Y, int64_t ldy, int32_t T, const int32_t* ks,
                      int64_t* support, double* beta_S, double* beta_cov, double* loss_trace, int32_t* n_iter,
                      int32_t* status, int64_t* id) {
  if (!S || !Y || !ks || !support || !beta_S || !loss_trace || !n_iter || !status || !id)
    return fail(IHT_EINVAL, "iht_server_submit: NULL argument");
  const Layout& L = S->g->L;
  const int32_t nc = S->U.cz + S->U.icpt;
  if (nc > 0 && !beta_cov) return fail(IHT_EINVAL, "iht_server_submit: beta_cov is NULL");
  if (T < 1 || T > S->slots) return fail(IHT_EINVAL, "iht_server_submit: T must be in [1, slots]");
  if (ldy < L.n) return fail(IHT_EINVAL, "iht_server_submit: ldy < n");
  Request R;
  R.ks.assign(ks, ks + T);
  for (int32_t j = 0; j < T; ++j) {
    if (ks[j] < 1 || ks[j] > S->kmax || ks[j] > L.p) return fail(IHT_EINVAL, "iht_server_submit: k out of range");
    R.kmax = std::max(R.kmax, ks[j]);
  }
  R.nT = L.n;
  if (subset) {
    R.bits.assign((size_t)L.ntiles, 0u);
    R.nT = 0;
    for (int64_t i = 0; i < L.n; ++i) {
      if (subset[i] > 1) return fail(IHT_EINVAL, "iht_server_submit: subset entries must be 0 or 1");
      if (subset[i]) {
        R.bits[(size_t)(i / kTileSubjects)] |= uint32_t(1) << (i % kTileSubjects);
        ++R.nT;
      }
    }
    if (R.nT < 1) return fail(IHT_EINVAL, "iht_server_submit: empty subject set");
  }
  R.id = (int64_t)S->requests.size();
  R.Y = Y;
  R.ldy = ldy;
  R.T = T;
  R.support = support;
  R.beta_S = beta_S;
  R.beta_cov = beta_cov;
  R.trace = loss_trace;
  R.n_iter = n_iter;
  R.status = status;
  for (int32_t j = 0; j < T; ++j) n_iter[j] = 0;
  S->requests.push_back(std::move(R));
  S->queue.push_back(S->requests.back().id);
  *id = S->requests.back().id;
  return IHT_OK;
}

int iht_server_step(iht_server* S, int32_t* completed) {
  if (!S || !completed) return fail(IHT_EINVAL, "iht_server_step: NULL argument");
  *completed = 0;
  if (int rc = admit_queued(S)) return rc;
  if (S->E.count_active() > 0) {
    if (int rc = S->E.turn()) return rc;
    ++S->turns;
  }
  return retire_finished(S, completed);
}

int iht_server_poll(const iht_server* S, int64_t id, int32_t* done) {
  if (!S || !done) return fail(IHT_EINVAL, "iht_server_poll: NULL argument");
  if (id < 0 || id >= (int64_t)S->requests.size()) return fail(IHT_EINVAL, "iht_server_poll: unknown request id");
  *done = S->requests[(size_t)id].done ? 1 : 0;
  return IHT_OK;
}

int iht_server_info(const iht_server* S, iht_server_info_t* info) {
  if (!S || !info) return fail(IHT_EINVAL, "iht_server_info: NULL argument");
  info->slots = S->slots;
  info->slots_busy = S->busy;
  info->stats_blocks = (int32_t)S->blocks.size();
  info->queued = (int64_t)S->queue.size();
  info->running = S->running;
  info->completed = S->completed;
  info->turns = S->turns;
  info->device_bytes = S->device_bytes;
  return IHT_OK;
}

int iht_server_destroy(iht_server* S) {
  if (!S) return IHT_OK;
  (void)hipStreamSynchronize(S->st);
  delete S;
  return IHT_OK;
}

}  // extern "C"
