// iht_engine.hip -- the solve loop over a set of slots (Methods, eq. (ihta) with the normalised
// step and the omega rule of "IHT step sizes"). Used by iht_fit / iht_fit_batch (all slots admitted
// at once, retired at once) and by the solve server (slots admitted and retired between turns).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "iht_host.h"

namespace iht {

namespace {
size_t align16(size_t b) { return (b + 15) / 16 * 16; }
}  // namespace

int check_opts(const iht_opts& o, const char* who) {
  if (o.max_iter < 0 || o.max_backtrack < 0 || !(o.c > 0.0 && o.c < 1.0) || !(o.shrink > 0.0 && o.shrink < 1.0) ||
      !(o.tol >= 0.0) || !(o.mixed_tol >= 0.0) || o.polish_iter < 0 ||
      (o.precision != IHT_FP64 && o.precision != IHT_FP32 && o.precision != IHT_MIXED_I8) ||
      (o.family != IHT_GAUSSIAN && o.family != IHT_LOGISTIC))
    return fail(IHT_EINVAL, std::string(who) + ": bad options");
  if (o.family == IHT_LOGISTIC && o.precision != IHT_FP64)
    return fail(IHT_EUNSUPPORTED, std::string(who) + ": the logistic family runs in IHT_FP64 only");
  return IHT_OK;
}

int check_kmax(const iht_opts& o, int32_t kmax, const char* who) {
  if (o.precision == IHT_MIXED_I8 && kmax > kCertifyMaxK)
    return fail(IHT_EUNSUPPORTED, std::string(who) + ": IHT_MIXED_I8 takes k <= " + std::to_string(kCertifyMaxK));
  return IHT_OK;
}

std::vector<std::pair<DevBuf*, size_t>> SolveWork::plan(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed) {
  const size_t Tz = (size_t)T, kz = (size_t)kmax;
  const size_t nb = (size_t)solve_subject_blocks(L.n), pst = (size_t)solve_partial_stride(nc);
  std::vector<std::pair<DevBuf*, size_t>> P = {
      {&beta, Tz * L.p * 8},
      {&g, Tz * L.p * 8},
      {&partial, gradient_work_bytes(L)},
      {&r, Tz * L.n_pad * 8},
      {&rc, Tz * L.n_pad * 8},
      {&S, Tz * kz * 8},
      {&Sp, Tz * kz * 8},
      {&betap, Tz * kz * 8},
      {&X, Tz * 2 * kz * L.n_pad * 8},
      {&bc, Tz * kMaxUnpenalized * 8},
      {&bcp, Tz * kMaxUnpenalized * 8},
      {&gc, Tz * kMaxUnpenalized * 8},
      {&fs, Tz * sizeof(FitState)},
      {&part, Tz * nb * pst * 8},
      {&pmu, Tz * nb * 8},
      {&ysum, Tz * kYsumStride * 8},
      {&pw, Tz * 3 * (kz + kMaxUnpenalized) * 8},
      {&ks, Tz * 4},
      {&sv, Tz * sizeof(BatchSolve)},
      {&flags, Tz * 4},
      {&rows, Tz * sizeof(OutRow)},
  };
  if (mixed) {
    P.push_back({&r8, batch_r8_bytes(L, T)});
    P.push_back({&scale, (size_t)batch_t_pad(T) * 8});
    P.push_back({&rsum, (size_t)batch_t_pad(T) * 8});
    P.push_back({&slots, Tz * 4});
    P.push_back({&count, 4});
    P.push_back({&rg, Tz * L.n_pad * 8});
    P.push_back({&gmax, Tz * (size_t)batch_gmax_ld(L) * 8});
  }
  P.push_back({&topk.small, TopkArea::small_bytes(T)});
  P.push_back({&topk.cand, TopkArea::cand_bytes(L.p, T)});
  return P;
}

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

size_t SolveWork::workspace_bytes(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed) {
  SolveWork W;
  size_t s = 0;
  for (const auto& e : W.plan(L, T, kmax, nc, mixed)) s += align256(e.second);
  return s;
}

int SolveWork::provide(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed, void* ws, size_t ws_bytes,
                       hipStream_t st) {
  const auto P = plan(L, T, kmax, nc, mixed);
  if (!ws) {
    for (size_t i = 0; i + 2 < P.size(); ++i) HIPCHK(P[i].first->ensure(P[i].second));
    return topk.ensure(L.p, T, st);
  }
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(IHT_EINVAL, "workspace not 256-byte aligned");
  size_t need = 0;
  for (const auto& e : P) need += align256(e.second);
  if (ws_bytes < need)
    return fail(IHT_EINVAL, "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need) + " bytes");
  char* at = static_cast<char*>(ws);
  for (size_t i = 0; i + 2 < P.size(); ++i) {
    P[i].first->borrow(at, P[i].second);
    at += align256(P[i].second);
  }
  char* small_p = at;
  char* cand_p = at + align256(P[P.size() - 2].second);
  return topk.borrow(small_p, cand_p, L.p, T, st);
}

int64_t SolveWork::device_bytes() const {
  const DevBuf* b[] = {&beta, &g,    &partial, &r,     &rc,   &S,     &Sp,    &betap, &X,     &bc,
                       &bcp,  &gc,   &fs,      &part,  &pmu,  &ysum,  &pw,    &ks,    &sv,    &flags,
                       &rows, &r8,   &scale,   &rsum,  &slots, &count, &rg,   &gmax, &topk.small, &topk.cand};
  int64_t s = 0;
  for (const DevBuf* d : b) s += (int64_t)d->bytes;
  return s;
}

Engine::~Engine() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (cap_st_) (void)hipStreamDestroy(cap_st_);
}

int Engine::setup(const iht_geno* g, SolveWork* Wp, SolveStage* Pp, int32_t T, int32_t kmax, const Unpen& U,
                  const double* Y, int64_t ldy, double* trace, const iht_opts& o, hipStream_t st, void* ws,
                  size_t ws_bytes) {
  g_ = g;
  W_ = Wp;
  P_ = Pp;
  SolveWork& W = *Wp;
  SolveStage& PS = *Pp;
  L_ = g->L;
  const Layout& L = L_;
  o_ = o;
  st_ = st;
  T_ = T;
  kmax_ = kmax;
  nc_ = U.cz + U.icpt;
  mixed_ = o.precision == IHT_MIXED_I8;
  if (int rc = check_kmax(o, kmax, "engine")) return rc;
  if (mixed_ && L.n > kBatchMaxSubjects)
    return fail(IHT_EUNSUPPORTED, "IHT_MIXED_I8 takes n <= " + std::to_string(kBatchMaxSubjects) + " subjects");
  if (exec_) (void)hipGraphExecDestroy(exec_);
  exec_ = nullptr;
  // the matrix-core path follows the FP64 iteration exactly (certified projection, FP64 gradient on
  // the support), so it stops by the same rule; the FP32 pass stops at mixed_tol and is refined
  tol_main_ = o.precision == IHT_FP32 ? std::max(o.tol, o.mixed_tol) : o.tol;
  const size_t Tz = (size_t)T;
  if (int rc = W.provide(L, T, kmax, nc_, mixed_, ws, ws_bytes, st)) return rc;
  const int32_t nb = solve_subject_blocks(L.n), pst = solve_partial_stride(nc_);
  // pinned areas: FitStates; ks, subject sets, flags, output rows, top-k error words
  HIPCHK(PS.host.ensure(Tz * sizeof(FitState)));
  const size_t o_sv = align16(Tz * 4), o_fl = o_sv + align16(Tz * sizeof(BatchSolve));
  const size_t o_rows = o_fl + align16(Tz * 4), o_err = o_rows + align16(Tz * sizeof(OutRow));
  HIPCHK(PS.stage.ensure(o_err + Tz * 4));
  h_ = reinterpret_cast<FitState*>(PS.host.p);
  std::memset(h_, 0, Tz * sizeof(FitState));
  ks_h_ = reinterpret_cast<int32_t*>(PS.stage.p);
  sv_h_ = reinterpret_cast<BatchSolve*>(PS.stage.p + o_sv);
  flags_h_ = reinterpret_cast<int32_t*>(PS.stage.p + o_fl);
  rows_h_ = reinterpret_cast<OutRow*>(PS.stage.p + o_rows);
  terr_ = reinterpret_cast<uint32_t*>(PS.stage.p + o_err);
  launch_.assign(Tz, 0);

  SolveSet& Q = Q_;
  Q = SolveSet{};
  Q.T = T;
  Q.kmax = kmax;
  Q.n = L.n;
  Q.n_pad = L.n_pad;
  Q.p = L.p;
  Q.p_pad = L.p_pad;
  Q.sv = W.sv.as<BatchSolve>();
  Q.ks = W.ks.as<int32_t>();
  Q.Y = Y;
  Q.ldy = ldy;
  Q.U = U;
  Q.beta = W.beta.as<double>();
  Q.g = W.g.as<double>();
  Q.r = W.r.as<double>();
  Q.rc = W.rc.as<double>();
  Q.S = W.S.as<int64_t>();
  Q.Sp = W.Sp.as<int64_t>();
  Q.betap = W.betap.as<double>();
  Q.X = W.X.as<double>();
  Q.bc = W.bc.as<double>();
  Q.bcp = W.bcp.as<double>();
  Q.gc = W.gc.as<double>();
  Q.fs = W.fs.as<FitState>();
  Q.trace = trace;
  Q.ldt = (int64_t)o.max_iter + 1;
  Q.nb = nb;
  Q.pst = pst;
  Q.part = W.part.as<double>();
  Q.pmu = W.pmu.as<double>();
  Q.ysum = W.ysum.as<double>();
  Q.pw = W.pw.as<double>();
  Q.family = o.family;

  TopkJob& J = J_;
  J = TopkJob{};
  J.beta = Q.beta;
  J.g = Q.g;
  J.ld = L.p;
  J.fs = Q.fs;
  J.ks = Q.ks;
  J.kmax = kmax;
  J.ldo = kmax;
  J.small = W.topk.small.as<uint32_t>();
  J.cand_key = W.topk.cand_key();
  J.cand_idx = W.topk.cand_idx();
  J.cap = W.topk.cap;
  if (mixed_) {  // the projection of the exact w from the matrix-core gradient
    J.certify = 1;
    J.tiled = g->tiled.as<uint8_t>();
    J.sv = Q.sv;
    J.rc = W.rg.as<double>();
    J.ldr = L.n_pad;
    J.n = L.n;
    J.p_pad = L.p_pad;
    J.ntiles = L.ntiles;
    J.gmax = W.gmax.as<uint64_t>();
    J.ldm = batch_gmax_ld(L);
  }
  // every slot starts idle (not fresh, not active, not retiring)
  HIPCHK(launch_zero_u32(reinterpret_cast<uint32_t*>(Q.fs), (int64_t)(Tz * sizeof(FitState) / 4), st));
  return IHT_OK;
}

int32_t Engine::count_active() const {
  int32_t c = 0;
  for (int32_t t = 0; t < T_; ++t) c += h_[t].active != 0 ? 1 : 0;
  return c;
}

int Engine::read_states() {
  HIPCHK(hipMemcpyAsync(h_, Q_.fs, (size_t)T_ * sizeof(FitState), hipMemcpyDeviceToHost, st_));
  HIPCHK(hipStreamSynchronize(st_));
  return IHT_OK;
}

// Copies host flags (NULL: none) into the device flag array; *dev = that array, or NULL for "all".
int Engine::upload_flags(const uint8_t* flags, const int32_t** dev) {
  if (!flags) {
    *dev = nullptr;
    return IHT_OK;
  }
  for (int32_t t = 0; t < T_; ++t) flags_h_[t] = flags[t] ? 1 : 0;
  HIPCHK(hipMemcpyAsync(W_->flags.p, flags_h_, (size_t)T_ * 4, hipMemcpyHostToDevice, st_));
  *dev = W_->flags.as<int32_t>();
  return IHT_OK;
}

// Gradient of the slots in `phase` (kPhaseInit: the admitted slots with finite inputs; kPhaseGo:
// those whose proposal was accepted). With per-slot passes only the slots in launch_ get a launch;
// each launch is gated on the slot's device flag.
int Engine::gradient(int32_t phase) {
  const uint8_t* tiled = g_->tiled.as<uint8_t>();
  SolveWork& W = *W_;
  if (mixed_) {
    HIPCHK(solve_slots(Q_.fs, T_, phase, W.slots.as<int32_t>(), W.count.as<int32_t>(), st_));
    HIPCHK(launch_gradient_batch(tiled, L_, Q_.r, L_.n_pad, T_, Q_.sv, W.slots.as<int32_t>(), W.count.as<int32_t>(),
                                 W.r8.as<int8_t>(), W.scale.as<double>(), W.rsum.as<double>(), Q_.g, L_.p, st_, Q_.fs,
                                 W.rg.as<double>(), W.gmax.as<uint64_t>()));
    // the accepted proposals' own entries exactly (the initial support is certified by its projection)
    if (phase == kPhaseGo) HIPCHK(solve_exact_support(Q_, W.rg.as<double>(), st_));
    return IHT_OK;
  }
  for (int32_t t = 0; t < T_; ++t) {
    if (!launch_[t]) continue;
    const BatchSolve& b = sv_h_[t];
    HIPCHK(launch_gradient(tiled, L_, Q_.r + (size_t)t * L_.n_pad, b.mask, b.nT, b.u, b.v, Q_.fs + t, o_.precision,
                           Q_.g + (size_t)t * L_.p, W.partial.as<double>(),
                           phase == kPhaseInit ? &Q_.fs[t].fresh : &Q_.fs[t].go, st_, Q_.rc + (size_t)t * L_.n_pad));
  }
  return IHT_OK;
}

// Proposal of the slots in `phase`: projection (warm-started by S), then the columns of S+, the
// backtracking test and (for the accepted ones) residual, loss and centred residual.
int Engine::propose(int32_t phase) {
  J_.phase = phase;
  J_.out = Q_.Sp;
  J_.vals = Q_.betap;
  J_.prev = Q_.S;  // the current support bounds the new k-th largest |w| from below
  J_.ldprev = kmax_;
  HIPCHK(launch_topk(J_, L_.p, T_, st_));
  HIPCHK(solve_decode(g_->tiled.as<uint8_t>(), Q_, 1, phase, st_));
  HIPCHK(solve_check_residual(Q_, phase, o_.c, o_.max_backtrack, st_));
  return IHT_OK;
}

int Engine::admit(const int32_t* ks, const BatchSolve* sv, const uint8_t* admit) {
  const size_t Tz = (size_t)T_;
  std::memcpy(ks_h_, ks, Tz * 4);
  std::memcpy(sv_h_, sv, Tz * sizeof(BatchSolve));
  HIPCHK(hipMemcpyAsync(W_->ks.p, ks_h_, Tz * 4, hipMemcpyHostToDevice, st_));
  HIPCHK(hipMemcpyAsync(W_->sv.p, sv_h_, Tz * sizeof(BatchSolve), hipMemcpyHostToDevice, st_));
  const int32_t* fl = nullptr;
  if (int rc = upload_flags(admit, &fl)) return rc;
  for (int32_t t = 0; t < T_; ++t) launch_[t] = (!admit || admit[t]) ? 1 : 0;

  // initial state: beta = 0, r = y on each subject set, g = A^T r, S = top-k |g| (mu = 1, beta = 0),
  // the first step size, then the first proposal
  HIPCHK(launch_topk_clear_errors(J_.small, T_, fl, st_));
  HIPCHK(solve_init(Q_, o_.max_iter, fl, st_));
  HIPCHK(solve_residual0(Q_, st_));
  if (int rc = gradient(kPhaseInit)) return rc;
  J_.phase = kPhaseInit;
  J_.out = Q_.S;
  J_.vals = nullptr;
  J_.prev = nullptr;
  HIPCHK(launch_topk(J_, L_.p, T_, st_));
  HIPCHK(solve_decode(g_->tiled.as<uint8_t>(), Q_, 0, kPhaseInit, st_));
  HIPCHK(solve_commit_mu(Q_, 0, tol_main_, o_.max_iter, st_));
  if (int rc = propose(kPhaseFresh)) return rc;
  HIPCHK(solve_mark(Q_, fl, 0, 0, st_));
  if (int rc = read_states()) return rc;
  for (int32_t t = 0; t < T_; ++t) launch_[t] = h_[t].active != 0 ? 1 : 0;
  return IHT_OK;
}

int Engine::turn() {
  auto count_bt = [&]() {
    int32_t c = 0;
    for (int32_t t = 0; t < T_; ++t) c += (h_[t].active != 0 && h_[t].need_bt != 0) ? 1 : 0;
    return c;
  };
  while (count_bt() > 0) {
    HIPCHK(solve_shrink(Q_, o_.shrink, st_));
    if (int rc = propose(kPhaseBacktrack)) return rc;
    if (int rc = read_states()) return rc;
  }
  if (graphs_ && mixed_) {
    if (!exec_)
      if (int rc = capture()) return rc;
    HIPCHK(hipGraphLaunch(exec_, st_));
  } else if (int rc = ahead()) {
    return rc;
  }
  if (int rc = read_states()) return rc;
  for (int32_t t = 0; t < T_; ++t) launch_[t] = h_[t].active != 0 ? 1 : 0;
  return IHT_OK;
}

// The speculative iterations of a turn: gradient of the accepted proposals, commit + next step
// size, next proposal; every launch gated per slot on the device flags.
int Engine::ahead() {
  for (int a = 0; a < kAhead; ++a) {
    if (int rc = gradient(kPhaseGo)) return rc;
    HIPCHK(solve_commit_mu(Q_, 1, tol_main_, o_.max_iter, st_));
    if (int rc = propose(kPhaseActive)) return rc;
  }
  return IHT_OK;
}

// Records ahead() into exec_ on the private stream (nothing runs while recording). The sequence
// holds kernel launches only (no memory set or copy nodes); their arguments are the engine's
// fixed buffers and the per-slot flags they read on the device.
int Engine::capture() {
  if (!cap_st_) HIPCHK(hipStreamCreateWithFlags(&cap_st_, hipStreamNonBlocking));
  hipStream_t user = st_;
  st_ = cap_st_;
  HIPCHK(hipStreamBeginCapture(cap_st_, hipStreamCaptureModeThreadLocal));
  const int rc = ahead();
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cap_st_, &graph);
  st_ = user;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
  const hipError_t ei = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    exec_ = nullptr;
    return hip_fail(ei, "hipGraphInstantiate");
  }
  return IHT_OK;
}

int Engine::retire(const uint8_t* flags, const OutRow* rows) {
  const size_t Tz = (size_t)T_;
  const int32_t* fl = nullptr;
  if (int rc = upload_flags(flags, &fl)) return rc;
  std::memcpy(rows_h_, rows, Tz * sizeof(OutRow));
  HIPCHK(hipMemcpyAsync(W_->rows.p, rows_h_, Tz * sizeof(OutRow), hipMemcpyHostToDevice, st_));
  HIPCHK(solve_mark(Q_, fl, 1, 1, st_));
  if (o_.precision == IHT_FP32 && o_.polish_iter > 0) HIPCHK(solve_polish(Q_, o_.tol, o_.polish_iter, st_));
  HIPCHK(solve_output(Q_, W_->rows.as<OutRow>(), st_));
  HIPCHK(solve_mark(Q_, fl, 1, 0, st_));
  HIPCHK(hipMemcpy2DAsync(terr_, 4, J_.small + kTopkErrorWord, (size_t)kTopkRowWords * 4, 4, Tz, hipMemcpyDeviceToHost,
                          st_));
  return read_states();
}

}  // namespace iht
