// iht_noalloc.hip -- the gradient pass for callers that cannot allocate device memory (code under
// stream capture, tight serving loops, harnesses that forbid allocation).
//
// iht_gradient keeps its scratch (the centred residual, the split pass's partial sums and the
// centring scalars) in memory its genotype handle allocates on first use. This variant runs the
// same kernels on a fixed array in device global memory instead: one array per device, reserved
// when the code object is loaded and held until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol); the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "iht_host.h"

namespace iht {
namespace {

// Scratch layout: the centring scalars (a FitState), then the gradient work area of
// launch_gradient (centred residual [n_pad] FP64, then the partial sums of a split pass). A pass
// splits its subjects only while its SNP groups times the split stay within one wave of 256
// workgroups, so the partial sums never exceed 256 workgroups x their lanes x kPassMaxNS SNPs x
// 16 bytes, for any p.
constexpr size_t kScratchStateBytes = 256;
constexpr int64_t kNoallocMaxSubjects = 262144;
constexpr size_t kScratchWorkBytes =
    (size_t)kNoallocMaxSubjects * 8 + (size_t)256 * kPassThreads * kPassMaxNS * 16;
constexpr size_t kScratchBytes = kScratchStateBytes + kScratchWorkBytes;  // 18 MB + 256 B
static_assert(sizeof(FitState) <= kScratchStateBytes, "centring scalars fit their slot");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
int scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(IHT_EDEVICE, "iht_gradient_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IHT_OK;
}

}  // namespace
}  // namespace iht

using namespace iht;

extern "C" {

size_t iht_gradient_noalloc_max_bytes(void) { return kScratchWorkBytes; }

int iht_gradient_noalloc(const iht_geno* g, const iht_stats* s, const double* r, double* grad, int32_t precision,
                         void* stream) {
  if (!g || !s || !r || !grad) return fail(IHT_EINVAL, "iht_gradient_noalloc: NULL argument");
  if (s->geno != g) return fail(IHT_EINVAL, "iht_gradient_noalloc: stats belong to another genotype handle");
  if (precision != IHT_FP64 && precision != IHT_FP32) return fail(IHT_EINVAL, "iht_gradient_noalloc: bad precision");
  const Layout& L = g->L;
  const size_t need = gradient_work_bytes(L);
  if (need > kScratchWorkBytes)
    return fail(IHT_EINVAL, "iht_gradient_noalloc: this matrix needs " + std::to_string(need) +
                                " bytes of scratch, more than the fixed " + std::to_string(kScratchWorkBytes) +
                                " (at most 262,144 subjects)");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != g->device) return fail(IHT_EINVAL, "iht_gradient_noalloc: the handle lives on another device");
  void* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  FitState* fs = static_cast<FitState*>(base);
  double* work = reinterpret_cast<double*>(static_cast<char*>(base) + kScratchStateBytes);
  HIPCHK(launch_gradient(g->tiled.as<uint8_t>(), L, r, s->mask, s->nT, s->u, s->v, fs, precision, grad, work,
                         nullptr, reinterpret_cast<hipStream_t>(stream)));
  return IHT_OK;
}

}  // extern "C"
