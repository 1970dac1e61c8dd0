// iht_batch.hip -- batched gradient G = X_st^T R for T solves sharing one packed genotype matrix.
//
// For solve t on subject set T_t (Methods, eq. normal_grad; "Bandwidth optimization of IHT"):
//   G_jt = v_jt (A_jt - u_jt (R_t - B_jt)),  A = X0^T R~, B = M^T R~, R_t = sum_i R~_it,
// with X0 the dosages (missing -> 0), M the missing indicator and R~ the residual centred over T_t
// and quantised to three balanced int8 digits under a power-of-two scale s_t:
//   R~_it = s_t (q0 + q1 / 254 + q2 / 254^2),  q in [-127, 127].
// A and B are exact int32 sums computed on the matrix cores (v_mfma_i32_32x32x32_i8): dosages 0/1/2
// and flags 0/1 times the digits; the digit sums are combined in FP64. The only approximation is
// the quantisation of the residual (|R - R~| <= s_t / (2 * 254^2), s_t < max|R| / 63.5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "iht_batch.h"

namespace iht {
namespace {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));
typedef uint32_t v2u_b __attribute__((ext_vector_type(2)));

constexpr int kDigits = 3;
constexpr double kBase = 254.0;

__device__ double bsum(double x, double* sh) {
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

__device__ double bmax(double x, double* sh) {
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

// Position along the matrix-core K dimension of subject s (0..31) of a tile: inside each 16-subject
// half, subject 4e + q sits at 4q + e (the genotype operand below is built code plane by code
// plane; both operands use the same order, so the products are unchanged).
__device__ __forceinline__ int kpos(int s) { return (s & 16) | ((s & 3) << 2) | ((s >> 2) & 3); }

// One block per slot: centre the slot's residual over its subject set, choose the scale, write the
// digits and the exact digit sums. Slots at or past the live count are skipped: a matrix-core
// column only ever meets its own digits, so their contents never reach a live slot.
// R8 layout: [tile][slot block of 32][digit][half of the tile][slot in the block][16 subjects] int8:
// the 3 KB of one tile and slot block are contiguous (one direct-to-LDS copy per digit), and in LDS
// lane (slot, half) reads its 16 bytes at consecutive 16-byte offsets (no bank conflicts).
__global__ __launch_bounds__(1024) void k_quant(const double* __restrict__ R, int64_t ldr, int64_t n, int64_t n_pad, int32_t T,
                                                int32_t T_pad, const BatchSolve* __restrict__ sv,
                                                const int32_t* __restrict__ slots, const int32_t* __restrict__ count,
                                                int8_t* __restrict__ R8, double* __restrict__ scale,
                                                double* __restrict__ rsum, FitState* __restrict__ fs,
                                                double* __restrict__ rq) {
  __shared__ double sh[40];
  const int slot = blockIdx.x;
  const int live = count ? *count : T;
  if (slot >= live) return;
  const int t = slots ? slots[slot] : slot;
  const double* r = R + (int64_t)t * ldr;
  const double* mask = sv[t].mask;
  double s1 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s1 += (mask[i] != 0.0) ? r[i] : 0.0;
  const double mean = bsum(s1, sh) / (double)sv[t].nT;
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    if (mask[i] != 0.0) mx = fmax(mx, fabs(r[i] - mean));
  mx = bmax(mx, sh);
  // smallest power of two s with 127 s >= max|r - mean| (exact scaling, no overflow of q0)
  double s = 1.0;
  if (mx > 0.0) {
    int e;
    (void)frexp(mx / 127.0, &e);
    s = ldexp(1.0, e);
    if (127.0 * ldexp(1.0, e - 1) >= mx) s = ldexp(1.0, e - 1);
  }
  double sq[kDigits] = {0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n_pad; i += blockDim.x) {
    int q[kDigits] = {0, 0, 0};
    const bool in = i < n && mask[i] != 0.0;
    if (rq) rq[(int64_t)t * ldr + i] = in ? r[i] - mean : 0.0;
    if (in && mx > 0.0) {
      double x = (r[i] - mean) / s;  // |x| <= 127, exact division by a power of two
      const double q0 = rint(x);
      const double e0 = (x - q0) * kBase;  // |e0| <= 127
      const double q1 = rint(e0);
      const double e1 = (e0 - q1) * kBase;
      const double q2 = rint(e1);
      q[0] = (int)q0;
      q[1] = (int)q1;
      q[2] = (int)q2;
    }
#pragma unroll
    for (int d = 0; d < kDigits; ++d) {
      const int kp = kpos((int)(i & 31));
      R8[((((i >> 5) * (T_pad / 32) + slot / 32) * kDigits + d) * 2 + (kp >> 4)) * 512 + (slot % 32) * 16 + (kp & 15)] =
          (int8_t)q[d];
      sq[d] += (double)q[d];  // integer-valued, exact
    }
  }
  double tot[kDigits];
#pragma unroll
  for (int d = 0; d < kDigits; ++d) tot[d] = bsum(sq[d], sh);
  if (threadIdx.x == 0) {
    scale[slot] = s;
    rsum[slot] = s * ((tot[0] + tot[1] * (1.0 / kBase)) + tot[2] * (1.0 / (kBase * kBase)));
    // |r_i - mean - R~_i| <= s / (2 254^2) (plus far smaller rounding); a standardised column has
    // sum_T x^2 = |T|, so sum_T |x| <= |T| (Cauchy-Schwarz) and every G_j is within |T| s / (2 254^2)
    // of the exact X_st^T r, before the FP64 combination's own rounding: twice that bounds both.
    if (fs) fs[t].gerr = (double)sv[t].nT * s * (1.0 / (kBase * kBase));
  }
}

// Two-bit code -> dosage / missing flag, as byte tables for v_perm (selector bytes 0-3 pick bytes
// 0-3 of the table): code 0 -> (0, 0), 1 (missing) -> (0, 1), 2 -> (1, 0), 3 -> (2, 0).
constexpr uint32_t kDoseBytes = 0x02010000u;
constexpr uint32_t kMissBytes = 0x00000100u;
// s_waitcnt immediate of gfx9-family targets for "no vector-memory operation outstanding" (vmcnt
// bits 3:0 and 15:14 zero, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

// One 32-SNP group per wave. With one slot block its 6 accumulator tiles (96 registers) leave 128
// registers per wave, so 16 waves share a CU; with two slot blocks (192 accumulator registers, 8
// waves per CU) each decoded genotype operand serves twice the matrix-core work and the matrix is
// streamed half as often.
constexpr int kBlockSolves = 32;

// Block (bx, by): kBlockSnps SNPs from kBlockSnps bx x the kSB blocks of 32 slots from kSB by. Wave
// w owns SNPs [kBlockSnps bx + 32 w, + 32) as one 32-row dosage operand and one missing-flag
// operand, times the 3 digit column tiles of each slot block: 6 kSB accumulator tiles of 32x32
// int32. The block shape (SNPs per block, blocks per CU, slot blocks) is a template parameter; the
// launcher picks it per problem shape by timing (every shape computes the same exact sums).
template <int kBlockSnps, int kMinBlocks, int kSB>
__global__ __launch_bounds__(2 * kBlockSnps, kMinBlocks) void k_gradB(const uint2* __restrict__ tiled, int64_t p, int64_t p_pad,
                                                                     int32_t ntiles, const int8_t* __restrict__ R8, int32_t T,
                                                                     int32_t T_pad, const BatchSolve* __restrict__ sv,
                                                                     const int32_t* __restrict__ slots,
                                                                     const int32_t* __restrict__ count,
                                                                     const double* __restrict__ scale,
                                                                     const double* __restrict__ rsum, double* __restrict__ G,
                                                                     int64_t ldg, uint64_t* __restrict__ gmax, int64_t ldm) {
  constexpr int kWaves = kBlockSnps / 32;
  static_assert(kBlockSnps % kGmaxSnps == 0, "whole 128-SNP groups per block");
  const int live = count ? *count : T;
  const int nsb = T_pad / kBlockSolves;
  const int sb0 = (int)blockIdx.y * kSB;      // the block's first slot block
  if (sb0 * kBlockSolves >= live) return;     // no live slot in this block (uniform)
  const int nsbb = min(kSB, nsb - sb0);       // slot blocks that exist (uniform)
  // Operands in LDS, in a ring of four tiles, copied from global memory straight into LDS (no
  // registers): the three 1 KB digit planes of each of the block's slot blocks and the block's
  // packed genotype segments (8 bytes per SNP, 1 KB per copy). Copy c of a tile is issued by wave
  // c % kWaves. The loop takes two tiles per barrier: at the start of a step each wave issues its
  // copies of the next two tiles (into the two slots read in the previous step), then does the
  // matrix-core work of the current two, waits for its copies and meets the others at the barrier.
  // No register receives a global load inside the loop, and the loop is unrolled over the ring, so
  // the ring slots are constant offsets and the compiler can see that an LDS read of one slot does
  // not wait for the copies into the others.
  constexpr int kRing = 4;
  constexpr int kSegKB = kBlockSnps * 8 / 1024;  // genotype copies per tile (1 KB each)
  constexpr int kNC = kDigits * kSB + kSegKB;    // copies per tile
  __shared__ __attribute__((aligned(16))) int8_t rb[kRing][kSB][kDigits * 1024];
  __shared__ __attribute__((aligned(16))) uint2 sg_lds[kRing][kBlockSnps];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int kh = lane >> 5;  // k-half: subjects 16 kh .. 16 kh + 15 of the tile
  const int col = lane & 31;

  const int64_t jb = (int64_t)blockIdx.x * kBlockSnps;  // the block's first SNP
  const int64_t j0 = jb + 32 * w;
  const int64_t jA = j0 + col;  // this lane's SNP
  // un-rotation selector: group g of the tile sits in segment byte (g - j) mod 8; this lane needs
  // groups 4 kh .. 4 kh + 3 in order (v_perm over the segment {hi dword, lo dword}).
  const uint32_t rot = (uint32_t)(jA & 7);
  uint32_t sel = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) sel |= ((4u * kh + e - rot) & 7u) << (8 * e);

  // this wave's copies of tile t into ring slot S (p_pad is a multiple of every block's SNPs)
  auto stage = [&](int t, auto S) {
    constexpr int slot = decltype(S)::value;
#pragma unroll
    for (int i = 0; i < (kNC + kWaves - 1) / kWaves; ++i) {
      const int c = w + i * kWaves;
      if (c < kDigits * kSB) {
        const int sbk = c / kDigits, d = c % kDigits;
        if (sbk < nsbb) {
          const int8_t* src = R8 + (((int64_t)t * nsb + sb0 + sbk) * kDigits + d) * 1024 + lane * 16;
          __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(&rb[slot][sbk][d * 1024]), 16, 0,
                                           0);
        }
      } else if (c < kNC) {
        const int part = c - kDigits * kSB;
        const uint2* src = tiled + (int64_t)t * p_pad + jb + part * 128 + lane * 2;
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(&sg_lds[slot][part * 128]), 16, 0, 0);
      }
    }
  };
  v16i acc[kSB][2][kDigits];  // [slot block][dose|miss][digit]
#pragma unroll
  for (int b = 0; b < kSB; ++b)
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int d = 0; d < kDigits; ++d) acc[b][o][d] = v16i{};

  // the matrix-core work of the tile in ring slot U
  auto compute = [&](auto U) {
    constexpr int u = decltype(U)::value;
    // A operands: 4 packed bytes (16 subjects) of the SNP; code plane q (the q-th code of every
    // byte) gives the dosage and flag bytes of dword q
    v4i op[2];
    {
      const uint2 sg = sg_lds[u][32 * w + col];
      const uint32_t g4 = __builtin_amdgcn_perm(sg.y, sg.x, sel);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t codes = (g4 >> (2 * q)) & 0x03030303u;
        op[0][q] = (int32_t)__builtin_amdgcn_perm(0u, kDoseBytes, codes);
        op[1][q] = (int32_t)__builtin_amdgcn_perm(0u, kMissBytes, codes);
      }
    }
#pragma unroll
    for (int b = 0; b < kSB; ++b) {
      if (b > 0 && b >= nsbb) break;  // uniform: the block's last slot block does not exist
#pragma unroll
      for (int d = 0; d < kDigits; ++d) {
        const v4i bop = *reinterpret_cast<const v4i*>(&rb[u][b][d * 1024 + kh * 512 + col * 16]);
#pragma unroll
        for (int o = 0; o < 2; ++o)
          acc[b][o][d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(op[o], bop, acc[b][o][d], 0, 0, 0);
      }
    }
  };
  // tiles t, t + 1 of the ring slots U, U + 1 (t % kRing == U), with one barrier
  auto step = [&](int t, auto U) {
    constexpr int u = decltype(U)::value;
    if (t + 2 < ntiles) stage(t + 2, std::integral_constant<int, (u + 2) % kRing>{});
    if (t + 3 < ntiles) stage(t + 3, std::integral_constant<int, (u + 3) % kRing>{});
    compute(U);
    if (t + 1 < ntiles) compute(std::integral_constant<int, u + 1>{});
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    // LDS is the only memory the waves share in the loop: a barrier without a memory fence (the
    // compiler barriers keep LDS accesses on their side of it)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
  };

  stage(0, std::integral_constant<int, 0>{});
  if (ntiles > 1) stage(1, std::integral_constant<int, 1>{});
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  for (int t = 0; t < ntiles; t += kRing) {
    step(t, std::integral_constant<int, 0>{});
    if (t + 2 < ntiles) step(t + 2, std::integral_constant<int, 2>{});
  }

  // Epilogue: column col = slot (sb0 + b) 32 + col; rows of register r: 8 (r / 4) + 4 kh + (r % 4).
  // With gmax, the largest |G| of each 128-SNP group and slot (waves 4 g .. 4 g + 3 hold group g of
  // the block) is left for the projection's filter, which skips the groups below its threshold.
  __shared__ uint64_t gm[kWaves][kBlockSolves];
  const double i1 = 1.0 / kBase, i2 = 1.0 / (kBase * kBase);
#pragma unroll
  for (int b = 0; b < kSB; ++b) {
    const int sl = (sb0 + b) * kBlockSolves + col;
    const bool on = sl < live;  // (false for a slot block past the last)
    uint64_t mk = 0;
    if (on) {
      const int t = slots ? slots[sl] : sl;
      const double s = scale[sl], Rt = rsum[sl];
      const double* u = sv[t].u;
      const double* v = sv[t].v;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t j = j0 + 8 * (r / 4) + 4 * kh + (r % 4);
        if (j >= p) continue;
        const double A = s * (((double)acc[b][0][0][r] + (double)acc[b][0][1][r] * i1) + (double)acc[b][0][2][r] * i2);
        const double B = s * (((double)acc[b][1][0][r] + (double)acc[b][1][1][r] * i1) + (double)acc[b][1][2][r] * i2);
        const double gj = v[j] * (A - u[j] * (Rt - B));
        G[(int64_t)t * ldg + j] = gj;
        const uint64_t key = (uint64_t)__double_as_longlong(fabs(gj));
        mk = key > mk ? key : mk;
      }
    }
    if (gmax) {  // uniform
      const uint64_t o = __shfl_xor(mk, 32, 64);  // the other k-half of the same slot
      mk = o > mk ? o : mk;
      if (kh == 0) gm[w][col] = mk;
      __syncthreads();
      if ((w & 3) == 0 && kh == 0 && on) {
        uint64_t m = gm[w][col];
#pragma unroll
        for (int x = 1; x < 4; ++x) m = gm[w + x][col] > m ? gm[w + x][col] : m;
        const int t = slots ? slots[sl] : sl;
        gmax[(int64_t)t * ldm + jb / kGmaxSnps + w / 4] = m;
      }
      __syncthreads();  // gm is reused by the next slot block
    }
  }
}

}  // namespace

int32_t batch_t_pad(int32_t T) { return (T + kBlockSolves - 1) / kBlockSolves * kBlockSolves; }

size_t batch_r8_bytes(const Layout& L, int32_t T) { return (size_t)L.ntiles * kDigits * batch_t_pad(T) * 32; }

namespace {

// Block shapes of k_gradB the launcher chooses from: (SNPs per block, blocks per CU, slot blocks).
struct GradBShape {
  int snps;
  int sb;
  void (*kernel)(const uint2*, int64_t, int64_t, int32_t, const int8_t*, int32_t, int32_t, const BatchSolve*,
                 const int32_t*, const int32_t*, const double*, const double*, double*, int64_t, uint64_t*, int64_t);
};
const GradBShape kShapes[] = {{256, 1, &k_gradB<256, 2, 1>}, {128, 1, &k_gradB<128, 4, 1>}, {256, 2, &k_gradB<256, 1, 2>},
                              {128, 2, &k_gradB<128, 2, 2>}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

hipError_t launch_shape(int si, const uint8_t* tiled, const Layout& L, const int8_t* R8, int32_t T, int32_t T_pad,
                        const BatchSolve* sv, const int32_t* slots, const int32_t* count, const double* scale,
                        const double* rsum, double* G, int64_t ldg, hipStream_t st, uint64_t* gmax = nullptr) {
  const GradBShape& S = kShapes[si];
  const int32_t nsb = T_pad / kBlockSolves;
  const dim3 grid((unsigned)((L.p + S.snps - 1) / S.snps), (unsigned)((nsb + S.sb - 1) / S.sb));
  hipLaunchKernelGGL(S.kernel, grid, dim3(2 * S.snps), 0, st, reinterpret_cast<const uint2*>(tiled), L.p, L.p_pad,
                     (int32_t)L.ntiles, R8, T, T_pad, sv, slots, count, scale, rsum, G, ldg, gmax, batch_gmax_ld(L));
  return hipGetLastError();
}

// Autotuner: the first launch for a (device, tiles, padded p, padded T) shape times every block
// shape three times on the call's own inputs (HIP events on the call's stream; each run writes the
// same G) and keeps the one of least median time for the rest of the process. Not while the
// stream is being captured into a graph: the first shape is used then, untimed.
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int64_t, int32_t>, int> g_tuned;

int tuned_shape(const uint8_t* tiled, const Layout& L, const int8_t* R8, int32_t T, int32_t T_pad, const BatchSolve* sv,
                const int32_t* slots, const int32_t* count, const double* scale, const double* rsum, double* G,
                int64_t ldg, hipStream_t st) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, (int64_t)L.ntiles, L.p_pad, T_pad);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return 0;
  }
  // one untimed run of each shape (code load, caches), then kTuneReps timed runs of each, the shapes
  // interleaved so that clock drift falls on all of them alike; the median decides
  constexpr int kTuneReps = 3;
  float ms[kNumShapes][kTuneReps];
  bool ok[kNumShapes];
  for (int si = 0; si < kNumShapes; ++si)
    ok[si] = launch_shape(si, tiled, L, R8, T, T_pad, sv, slots, count, scale, rsum, G, ldg, st) == hipSuccess;
  for (int rep = 0; rep < kTuneReps; ++rep)
    for (int si = 0; si < kNumShapes; ++si) {
      if (!ok[si]) continue;
      ok[si] = hipEventRecord(e0, st) == hipSuccess &&
               launch_shape(si, tiled, L, R8, T, T_pad, sv, slots, count, scale, rsum, G, ldg, st) == hipSuccess &&
               hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
               hipEventElapsedTime(&ms[si][rep], e0, e1) == hipSuccess;
    }
  int best = 0;
  float best_ms = 0.0f;
  bool have = false;
  for (int si = 0; si < kNumShapes; ++si) {
    if (!ok[si]) continue;
    std::sort(ms[si], ms[si] + kTuneReps);
    const float med = ms[si][kTuneReps / 2];
    if (!have || med < best_ms) {
      best = si;
      best_ms = med;
      have = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

int32_t batch_tuned_snps(const Layout& L, int32_t T) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(dev, (int64_t)L.ntiles, L.p_pad, batch_t_pad(T)));
  return it == g_tuned.end() ? 0 : kShapes[it->second].snps;
}

hipError_t launch_gradient_batch(const uint8_t* tiled, const Layout& L, const double* R, int64_t ldr, int32_t T,
                                 const BatchSolve* sv, const int32_t* slots, const int32_t* count, int8_t* R8, double* scale,
                                 double* rsum, double* G, int64_t ldg, hipStream_t st, FitState* fs, double* rq,
                                 uint64_t* gmax) {
  const int32_t T_pad = batch_t_pad(T);
  hipLaunchKernelGGL(k_quant, dim3((unsigned)T_pad), dim3(1024), 0, st, R, ldr, L.n, L.n_pad, T, T_pad, sv, slots, count, R8,
                     scale, rsum, fs, rq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int si = tuned_shape(tiled, L, R8, T, T_pad, sv, slots, count, scale, rsum, G, ldg, st);
  return launch_shape(si, tiled, L, R8, T, T_pad, sv, slots, count, scale, rsum, G, ldg, st, gmax);
}

}  // namespace iht
