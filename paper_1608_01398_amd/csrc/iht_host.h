// iht_host.h -- host runtime pieces shared by the entry points, the solve engine and the solve
// server: error reporting, device buffers, the handle types, and the solve engine.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "iht.h"
#include "iht_batch.h"
#include "iht_internal.h"
#include "iht_solve.h"

namespace iht {

// The message behind iht_last_error (one per host thread).
inline std::string& last_error_text() {
  static thread_local std::string s;
  return s;
}

inline int fail(int code, const std::string& msg) {
  last_error_text() = msg;
  return code;
}

inline int hip_fail(hipError_t e, const char* what) {
  last_error_text() = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? IHT_ENOMEM : IHT_EDEVICE;
}

#define HIPCHK(expr)                                       \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return ::iht::hip_fail(e_, #expr); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;  // false: a view into memory the caller owns (a workspace); never freed here
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  // views b bytes at q (owned memory is released first)
  void borrow(void* q, size_t b) {
    release();
    p = q;
    bytes = b;
    owned = false;
  }
  // grows to at least b bytes (contents are lost when it grows); *fresh tells whether it did
  hipError_t ensure(size_t b, bool* fresh = nullptr) {
    if (fresh) *fresh = false;
    if (b <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, std::max<size_t>(b, 256));
    if (e == hipSuccess) {
      bytes = b;
      if (fresh) *fresh = true;
    }
    return e;
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

// Pinned host memory, grown on demand (contents are lost when it grows).
struct PinnedBuf {
  char* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(b, 256), hipHostMallocDefault);
    if (e == hipSuccess) bytes = b;
    return e;
  }
};

inline Layout make_layout(int64_t n, int64_t p) {
  Layout L;
  L.n = n;
  L.p = p;
  L.ntiles = (n + kTileSubjects - 1) / kTileSubjects;
  L.n_pad = L.ntiles * kTileSubjects;
  L.p_pad = (p + kSnpAlign - 1) / kSnpAlign * kSnpAlign;
  return L;
}

// Device work area for `rows` top-k problems over p entries. The per-row counters and histogram
// start zeroed and are self-resetting; the error words are cleared before each use.
struct TopkArea {
  DevBuf small;  // rows x kTopkRowWords
  DevBuf cand;   // rows x cap x (8 + 4) bytes
  int64_t cap = 0;
  int32_t rows = 0;
  static int64_t cap_for(int64_t p) { return std::max<int64_t>(p, 16384); }  // also holds the two-pass candidates
  static size_t small_bytes(int32_t nrows) { return (size_t)nrows * kTopkRowWords * 4; }
  static size_t cand_bytes(int64_t p, int32_t nrows) {
    return (size_t)nrows * (size_t)cap_for(p) * (sizeof(uint64_t) + sizeof(int32_t));
  }
  int ensure(int64_t p, int32_t nrows, hipStream_t st) {
    if (nrows > rows || !small.p) {
      bool fresh = false;
      HIPCHK(small.ensure(small_bytes(nrows), &fresh));
      if (fresh) HIPCHK(launch_zero_u32(small.as<uint32_t>(), (int64_t)nrows * kTopkRowWords, st));
      rows = nrows;
    }
    const int64_t want = cap_for(p);
    if (want > cap || (size_t)rows * (size_t)cap * 12 > cand.bytes) {
      cap = std::max(cap, want);
      HIPCHK(cand.ensure((size_t)rows * (size_t)cap * (sizeof(uint64_t) + sizeof(int32_t))));
    }
    return IHT_OK;
  }
  // views caller memory laid out by the plan below; the counters are cleared on the stream
  int borrow(void* small_p, void* cand_p, int64_t p, int32_t nrows, hipStream_t st) {
    small.borrow(small_p, small_bytes(nrows));
    cand.borrow(cand_p, cand_bytes(p, nrows));
    rows = nrows;
    cap = cap_for(p);
    HIPCHK(launch_zero_u32(small.as<uint32_t>(), (int64_t)nrows * kTopkRowWords, st));
    return IHT_OK;
  }
  uint64_t* cand_key() const { return cand.as<uint64_t>(); }
  int32_t* cand_idx() const {
    return reinterpret_cast<int32_t*>(cand.as<char>() + (size_t)rows * (size_t)cap * sizeof(uint64_t));
  }
};

// Device state of a set of solve slots: allocated by the library (grown on demand and reused) or
// carved out of a caller's workspace.
struct SolveWork {
  DevBuf beta, g, partial, r, rc, S, Sp, betap, X, bc, bcp, gc, fs, part, pmu, ysum, pw, ks, sv, flags, rows;
  DevBuf r8, scale, rsum, slots, count, rg;  // matrix-core pass work; rg: centred residual of each slot's gradient
  DevBuf gmax;  // matrix-core pass: largest |g| per 128 SNPs of each slot's gradient (the filter skips below it)
  TopkArea topk;

  // Every device buffer of T slots with model sizes up to kmax and nc unpenalised columns, with its
  // size (the top-k area's two buffers last). One list serves allocation, carving a workspace and
  // sizing one, so the three cannot disagree.
  std::vector<std::pair<DevBuf*, size_t>> plan(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed);
  // Bytes of a workspace that holds plan(...) (each buffer 256-byte aligned).
  static size_t workspace_bytes(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed);
  // Allocates (ws == NULL) or carves ws (ws_bytes >= workspace_bytes) into the plan's buffers.
  int provide(const Layout& L, int32_t T, int32_t kmax, int32_t nc, bool mixed, void* ws, size_t ws_bytes,
              hipStream_t st);
  int64_t device_bytes() const;
};

// Pinned host memory through which an engine exchanges the slots' small inputs and flags with the
// device (kept by the handle that owns the engine's memory).
struct SolveStage {
  PinnedBuf host;   // the slots' FitStates as last read
  PinnedBuf stage;  // ks, subject sets, flags, output rows and top-k error words
};

int check_opts(const iht_opts& o, const char* who);
// IHT_EUNSUPPORTED (with the message) when the precision cannot take model sizes up to kmax.
int check_kmax(const iht_opts& o, int32_t kmax, const char* who);

// The solve loop of Methods, eq. (ihta) with the normalised step and the omega rule of "IHT step
// sizes", over T slots sharing one genotype matrix. Every per-slot kernel is gated on the slot's
// device flags, so slots at different points of their solve share each launch; a slot is admitted
// (its initial state computed) without disturbing the others, advanced turn by turn, and retired
// (refined and written out) on its own. All arithmetic runs in the device kernels; the host only
// orders the launches and reads the slots' flags once per turn.
//
// A turn: halving rounds for the slots whose proposal was rejected, then kAhead speculative
// iterations [gradient of the accepted proposals, commit + next step size, next proposal (top-k
// warm-started by S), column decode, residual + backtracking test + decision]. A slot waiting for
// a halving would only repeat its proposal (same step size, same proposal, same rejection), so the
// speculative proposals skip it, as they skip the slots that finished: running ahead never changes
// a result.
class Engine {
 public:
  static constexpr int kAhead = 2;

  Engine() = default;
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine();
  // Replay the speculative part of each turn from a HIP graph (matrix-core gradient only: its
  // launch sequence does not depend on which slots are iterating). Captured at the first turn on a
  // private stream, replayed on the engine's stream; for engines that run many turns with the same
  // buffers (the solve server).
  void use_graphs(bool on) { graphs_ = on; }

  // Device state of T slots with model sizes up to kmax (allocated in W). Slot t reads its trait
  // at Y + t * ldy and keeps its loss trace at trace + t * (max_iter + 1).
  // The device state comes from W (allocated there, or carved from the workspace ws of ws_bytes
  // bytes when ws is not NULL), the pinned staging from P.
  int setup(const iht_geno* g, SolveWork* W, SolveStage* P, int32_t T, int32_t kmax, const Unpen& U, const double* Y,
            int64_t ldy, double* trace, const iht_opts& o, hipStream_t st, void* ws = nullptr, size_t ws_bytes = 0);
  // Admits the slots with admit[t] != 0 (every slot if admit is NULL): ks and sv (host [T]) give
  // every slot's model size and subject set; the admitted ones get beta = 0, the initial residual,
  // gradient, support and step size, and their first proposal. The other slots are untouched.
  // Ends with the states read.
  int admit(const int32_t* ks, const BatchSolve* sv, const uint8_t* admit);
  // One turn of every slot still iterating; ends with the states read.
  int turn();
  // Writes out the slots with flags[t] != 0 (every slot if NULL): the FP64 refinement after an
  // FP32 solve, then the outputs into rows[t] (host [T]). Ends with the states and the top-k error
  // words read.
  int retire(const uint8_t* flags, const OutRow* rows);

  const FitState& state(int32_t t) const { return h_[t]; }
  uint32_t topk_error(int32_t t) const { return terr_[t]; }
  int32_t count_active() const;
  int32_t slots() const { return T_; }
  int32_t kmax() const { return kmax_; }

 private:
  int gradient(int32_t phase);
  int propose(int32_t phase);
  int ahead();
  int capture();
  int read_states();
  int upload_flags(const uint8_t* flags, const int32_t** dev);

  const iht_geno* g_ = nullptr;
  SolveWork* W_ = nullptr;
  SolveStage* P_ = nullptr;
  Layout L_{};
  iht_opts o_{};
  hipStream_t st_ = nullptr;
  int32_t T_ = 0, kmax_ = 0, nc_ = 0;
  bool mixed_ = false;
  double tol_main_ = 0.0;
  SolveSet Q_{};
  TopkJob J_{};
  // pinned host views (inside W->host and W->stage)
  FitState* h_ = nullptr;
  int32_t* ks_h_ = nullptr;
  BatchSolve* sv_h_ = nullptr;
  int32_t* flags_h_ = nullptr;
  OutRow* rows_h_ = nullptr;
  uint32_t* terr_ = nullptr;
  std::vector<uint8_t> launch_;  // slots that get a per-slot gradient launch (FP64 / FP32 passes)
  bool graphs_ = false;
  hipStream_t cap_st_ = nullptr;     // private stream the graph is captured on
  hipGraphExec_t exec_ = nullptr;    // the kAhead iterations of a turn
};

}  // namespace iht

struct iht_geno {
  int device = 0;
  iht::Layout L{};
  iht::DevBuf tiled;
  // scratch for iht_gradient (centred residual, partial sums, scalars) and for iht_fit
  iht::DevBuf partial, state;
  iht::SolveWork fit;
  iht::SolveStage fit_stage;
  iht::DevBuf batch_r8, batch_scale, batch_rsum, batch_sv;  // iht_gradient_batch work areas
  iht::DevBuf pred_err;                                      // iht_predict's error word
};

struct iht_stats {
  const iht_geno* geno = nullptr;
  int64_t nT = 0;
  // one allocation: u [p], v [p], the FP64 subject mask [n_pad], then the subject bits [ntiles]
  iht::DevBuf buf;
  double* u = nullptr;
  double* v = nullptr;
  double* mask = nullptr;
  uint32_t* mask_bits = nullptr;
};
