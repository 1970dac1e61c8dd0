// iht_device.hip -- gfx950 kernels around the gradient pass: the re-tile of the PLINK matrix into
// the device layout, the per-SNP standardisation statistics, the hard-threshold projection (top-k)
// and small fill/scatter helpers. The gradient pass itself is in iht_pass.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "iht_internal.h"

namespace iht {
namespace {

__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------------------------------
// Re-tile PLINK SNP-major rows into [tile][p_pad][8 B] with a per-SNP byte rotation.

// Block (bx, by): SNPs [32 bx, 32 bx + 32) x tiles [32 by, 32 by + 32), i.e. PLINK bytes
// [256 by, 256 by + 256) of 32 rows. The rows are staged in LDS with consecutive lanes reading
// consecutive bytes of a row; the segments are written with consecutive lanes on consecutive SNPs
// of one tile (256 contiguous bytes per tile). Pad SNPs (j >= p) and bits of subjects >= n are zero.
constexpr int kRetileSnps = 32;
constexpr int kRetileTiles = 32;
constexpr int kRetileBytes = kRetileTiles * kSegBytes;  // 256 PLINK bytes per row and block

__global__ __launch_bounds__(256) void k_retile(const uint8_t* __restrict__ raw, int64_t row, int64_t n, int64_t p,
                                                int64_t p_pad, int64_t ntiles, uint8_t* __restrict__ tiled) {
  __shared__ uint8_t st[kRetileSnps][kRetileBytes];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kRetileSnps;
  const int64_t c0 = (int64_t)blockIdx.y * kRetileBytes;  // first PLINK byte of the chunk
  const int64_t nbytes = (n + 3) / 4;                       // PLINK bytes that hold subjects
#pragma unroll 4
  for (int q = tid; q < kRetileSnps * kRetileBytes; q += 256) {
    const int r = q / kRetileBytes, o = q % kRetileBytes;
    const int64_t j = j0 + r, src = c0 + o;
    uint32_t val = 0;
    if (j < p && src < nbytes) {
      val = raw[j * row + src];
      const int64_t keep = n - src * 4;  // subjects of this byte that exist
      if (keep < 4) val &= (1u << (2 * keep)) - 1u;
    }
    st[r][o] = (uint8_t)val;
  }
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.y * kRetileTiles;
#pragma unroll
  for (int m = 0; m < (kRetileSnps * kRetileTiles) / 256; ++m) {
    const int q = tid + 256 * m;
    const int r = q % kRetileSnps, tl = q / kRetileSnps;
    const int64_t t = t0 + tl, j = j0 + r;
    if (t >= ntiles) continue;
    const int rot = (int)(j & (kSegBytes - 1));
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int b = 0; b < kSegBytes; ++b) w[b >> 2] |= (uint32_t)st[r][tl * kSegBytes + ((b + rot) & (kSegBytes - 1))] << (8 * (b & 3));
    *reinterpret_cast<uint2*>(tiled + (t * p_pad + j) * kSegBytes) = make_uint2(w[0], w[1]);
  }
}

// ------------------------------------------------------------------------------------------------
// Exact genotype class counts over the subject set -> u, v (Methods, "Bandwidth optimization of IHT").

// Bit q of m -> bit 2q: byte g of the result is the subject mask of 4-subject group g of a tile, on
// the low bits of the groups' 2-bit codes.
__device__ __forceinline__ uint64_t spread32(uint32_t m) {
  uint64_t x = m;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

// One SNP per thread, the tiles 8 at a time with their loads issued first. Each 2-bit code adds to
// one of het (10), hom (11) or missing (01); 00 adds nothing, which is also what the cleared bits
// of subjects past n hold, so with the whole subject set (FULL) no mask is applied. Otherwise the
// tile's subject bits are spread onto the codes' low bits and rotated by the SNP's byte rotation
// (byte b of the segment holds group (b + j) mod 8).
template <bool FULL>
__global__ __launch_bounds__(256) void k_stats(const uint2* __restrict__ tiled, int64_t p, int64_t p_pad, int64_t ntiles,
                                               const uint32_t* __restrict__ mask_bits, int64_t nT, double* __restrict__ u,
                                               double* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  const int rot8 = 8 * (int)(j & (kSegBytes - 1));
  uint32_t het = 0, hom = 0, mis = 0;
  constexpr int U = 8;
  for (int64_t t0 = 0; t0 < ntiles; t0 += U) {
    uint2 d[U];
#pragma unroll
    for (int e = 0; e < U; ++e) d[e] = (t0 + e < ntiles) ? tiled[(t0 + e) * p_pad + j] : make_uint2(0u, 0u);
#pragma unroll
    for (int e = 0; e < U; ++e) {
      uint32_t m0 = 0xFFFFFFFFu, m1 = 0xFFFFFFFFu;
      if (!FULL) {
        const uint64_t s64 = spread32(t0 + e < ntiles ? mask_bits[t0 + e] : 0u);
        const uint64_t seg = rot8 ? (s64 >> rot8) | (s64 << (64 - rot8)) : s64;
        m0 = (uint32_t)seg;
        m1 = (uint32_t)(seg >> 32);
      }
      const uint32_t lo0 = d[e].x & 0x55555555u, hi0 = (d[e].x >> 1) & 0x55555555u;
      const uint32_t lo1 = d[e].y & 0x55555555u, hi1 = (d[e].y >> 1) & 0x55555555u;
      het += __popc(hi0 & ~lo0 & m0) + __popc(hi1 & ~lo1 & m1);
      hom += __popc(hi0 & lo0 & m0) + __popc(hi1 & lo1 & m1);
      mis += __popc(lo0 & ~hi0 & m0) + __popc(lo1 & ~hi1 & m1);
    }
  }
  const int64_t nobs = nT - (int64_t)mis;
  if (nobs == 0) {
    u[j] = 0.0;
    v[j] = 0.0;
    return;
  }
  const int64_t s1 = (int64_t)het + 2 * (int64_t)hom;
  const int64_t s2 = (int64_t)het + 4 * (int64_t)hom;
  const int64_t num = nobs * s2 - s1 * s1;
  u[j] = __ddiv_rn((double)s1, (double)nobs);
  if (num == 0) {
    v[j] = 0.0;
    return;
  }
  const double var = __ddiv_rn((double)num, (double)(nobs * nT));
  v[j] = __ddiv_rn(1.0, __dsqrt_rn(var));
}

// ------------------------------------------------------------------------------------------------
// Top-k of |w| with ties to the lower index (the projection of eq. ihta).
// Level 0: 8192-bin histogram of key bits 62..50 (key = IEEE bits of |w|) -> threshold bucket.
// Collect: keys above the bucket are selected; keys in it are candidates. The last block finds the
// exact remainder among the candidates by radix select on the unique 96-bit key (|w| bits, ~index),
// then sorts the k indices ascending.

// Row t of a TopkJob: the values it ranks, its k and its work area.
struct TopkRow {
  const double* beta;  // NULL: w = g
  const double* g;
  double mu;
  int32_t k;
  TopkWork tw;
  int64_t* out;
  double* vals;
  __device__ double at(int64_t j) const { return beta ? __dadd_rn(beta[j], __dmul_rn(mu, g[j])) : g[j]; }
};

// false when row t is outside the job's phase (the whole block then returns).
__device__ __forceinline__ bool topk_row(const TopkJob& J, int t, TopkRow& R) {
  if (J.fs && !fs_selected(J.fs + t, J.phase)) return false;
  R.beta = J.beta ? J.beta + (int64_t)t * J.ld : nullptr;
  R.g = J.g + (int64_t)t * J.ld;
  R.mu = J.beta ? J.fs[t].mu : 0.0;
  R.k = J.ks ? J.ks[t] : J.k0;
  uint32_t* b = J.small + (int64_t)t * kTopkRowWords;
  R.tw.hist = b;
  R.tw.counters = b + kTopkBins0;
  R.tw.state = b + kTopkBins0 + 8;
  R.tw.sel = reinterpret_cast<int32_t*>(b + kTopkBins0 + 16);
  R.tw.cand_key = J.cand_key + (int64_t)t * J.cap;
  R.tw.cand_idx = J.cand_idx + (int64_t)t * J.cap;
  R.out = J.out + (int64_t)t * J.ldo;
  R.vals = J.vals ? J.vals + (int64_t)t * J.ldo : nullptr;
  return true;
}

__device__ __forceinline__ uint64_t abs_key(double w) { return (uint64_t)__double_as_longlong(fabs(w)); }
__device__ __forceinline__ double key_value(uint64_t key) { return __longlong_as_double((long long)key); }

// Bound on |w~_j - w_j| for the entries of a certified row off its exact support: the gradient's
// bound, times the step size when w = beta + mu g.
__device__ __forceinline__ double row_err(const TopkJob& J, int t, const TopkRow& R) {
  const double e = J.fs[t].gerr;
  return R.beta ? R.mu * e : e;
}

// (bucket, count above, count in bucket) of the need-th largest over nb bins held in LDS h,
// found by the first wave (per-lane bin sums, then a shuffle suffix scan); out[] is visible to the
// whole block after the closing barrier.
__device__ void find_bucket(const uint32_t* h, int nb, uint32_t need, uint32_t* out) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int per = nb / 64;
    uint32_t local = 0;
    for (int q = 0; q < per; ++q) local += h[lane * per + q];
    uint32_t incl = local;  // sum over lanes >= lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_down(incl, off, 64);
      if (lane + off < 64) incl += t;
    }
    uint32_t cum = incl - local;  // sum over lanes > lane (higher bins)
    if (cum < need && cum + local >= need) {
      for (int q = per - 1; q >= 0; --q) {
        const uint32_t c = h[lane * per + q];
        if (cum + c >= need) {
          out[0] = (uint32_t)(lane * per + q);
          out[1] = cum;
          out[2] = c;
          break;
        }
        cum += c;
      }
    }
  }
  __syncthreads();
}

// Total order of the projection: |w| descending, then index ascending ("a before b").
__device__ __forceinline__ bool key_before(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(1024) void k_topk_hist(TopkJob J, int64_t p, int64_t chunk) {
  TopkRow src;
  if (!topk_row(J, blockIdx.y, src)) return;
  const TopkWork& tw = src.tw;
  const int32_t k = src.k;
  __shared__ uint32_t h[kTopkBins0];
  __shared__ uint32_t res[4];
  __shared__ uint32_t ticket;
  for (int i = threadIdx.x; i < kTopkBins0; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * chunk, e = min(p, b + chunk);
  bool bad = false;
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
    const double w = src.at(j);
    bad |= !isfinite(w);
    atomicAdd(&h[(uint32_t)(abs_key(w) >> 50) & (kTopkBins0 - 1)], 1u);
  }
  if (bad) atomicOr(&tw.state[3], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kTopkBins0; i += blockDim.x)
    if (h[i]) atomicAdd(&tw.hist[i], h[i]);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) ticket = atomicAdd(&tw.counters[0], 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();
  for (int i = threadIdx.x; i < kTopkBins0; i += blockDim.x) {
    h[i] = atomic_load_u32(&tw.hist[i]);
    tw.hist[i] = 0u;
  }
  __syncthreads();
  find_bucket(h, kTopkBins0, (uint32_t)k, res);
  if (threadIdx.x == 0) {
    tw.state[0] = res[0];
    tw.state[1] = res[1];
    tw.state[2] = res[2];
    tw.counters[0] = 0u;
  }
}

constexpr int kCandLds = 2048;  // candidates ranked directly in LDS when there are at most this many

__global__ __launch_bounds__(1024) void k_topk_collect(TopkJob J, int64_t p, int64_t chunk) {
  TopkRow src;
  if (!topk_row(J, blockIdx.y, src)) return;
  const TopkWork& tw = src.tw;
  const int32_t k = src.k;
  int64_t* __restrict__ support = src.out;
  double* __restrict__ vals = src.vals;
  __shared__ int32_t sel[kTopkMaxK];
  __shared__ uint64_t ck[kCandLds];
  __shared__ int32_t ci[kCandLds];
  __shared__ uint32_t h[4096];
  __shared__ uint32_t res[4];
  __shared__ uint32_t ticket, nsel_l;
  const uint32_t bucket = tw.state[0];
  const int64_t b = (int64_t)blockIdx.x * chunk, e = min(p, b + chunk);
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
    const uint64_t key = abs_key(src.at(j));
    const uint32_t bin = (uint32_t)(key >> 50) & (kTopkBins0 - 1);
    if (bin > bucket) {
      const uint32_t pos = atomicAdd(&tw.counters[2], 1u);
      if (pos < (uint32_t)kTopkMaxK) tw.sel[pos] = (int32_t)j;
    } else if (bin == bucket) {
      const uint32_t pos = atomicAdd(&tw.counters[3], 1u);
      tw.cand_key[pos] = key;
      tw.cand_idx[pos] = (int32_t)j;
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) ticket = atomicAdd(&tw.counters[1], 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();

  // ---- last block: the `need` best candidates of the threshold bucket, then sort k indices ----
  const uint32_t n_above = atomic_load_u32(&tw.counters[2]);
  const uint32_t n_cand = atomic_load_u32(&tw.counters[3]);
  for (uint32_t q = threadIdx.x; q < n_above; q += blockDim.x)
    sel[q] = __hip_atomic_load(&tw.sel[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t need = (uint32_t)k - n_above;
  if (n_cand <= (uint32_t)kCandLds) {
    for (uint32_t q = threadIdx.x; q < n_cand; q += blockDim.x) {
      ck[q] = __hip_atomic_load(&tw.cand_key[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ci[q] = __hip_atomic_load(&tw.cand_idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // rank of each candidate in the total order; ranks are distinct, so the best `need` land in
    // sel[n_above + rank] without atomics
    for (uint32_t q = threadIdx.x; q < n_cand; q += blockDim.x) {
      const uint64_t kq = ck[q];
      const int32_t iq = ci[q];
      uint32_t rank = 0;
      for (uint32_t q2 = 0; q2 < n_cand; ++q2) rank += key_before(ck[q2], ci[q2], kq, iq) ? 1u : 0u;
      if (rank < need) sel[n_above + rank] = iq;
    }
  } else {
    // Radix select of the need-th best 96-bit key c = (|w| bits << 32) | ~index over candidates.
    typedef unsigned __int128 u128;
    u128 prefix = 0;
    uint32_t need_c = need;
    for (int L = 0; L < 8; ++L) {
      const int shift = 84 - 12 * L;
      for (int i = threadIdx.x; i < 4096; i += blockDim.x) h[i] = 0;
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < n_cand; q += blockDim.x) {
        const u128 c = ((u128)__hip_atomic_load(&tw.cand_key[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 32) |
                       (u128)(0xFFFFFFFFu - (uint32_t)__hip_atomic_load(&tw.cand_idx[q], __ATOMIC_RELAXED,
                                                                       __HIP_MEMORY_SCOPE_AGENT));
        if ((c >> (shift + 12)) == prefix) atomicAdd(&h[(uint32_t)(c >> shift) & 0xFFFu], 1u);
      }
      __syncthreads();
      find_bucket(h, 4096, need_c, res);
      prefix = (prefix << 12) | (u128)res[0];
      need_c -= res[1];
      __syncthreads();
    }
    if (threadIdx.x == 0) nsel_l = n_above;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < n_cand; q += blockDim.x) {
      const int32_t idx = __hip_atomic_load(&tw.cand_idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u128 c = ((u128)__hip_atomic_load(&tw.cand_key[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 32) |
                     (u128)(0xFFFFFFFFu - (uint32_t)idx);
      if (c >= prefix) {
        const uint32_t pos = atomicAdd(&nsel_l, 1u);
        if (pos < (uint32_t)kTopkMaxK) sel[pos] = idx;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && nsel_l != (uint32_t)k) atomicOr(&tw.state[3], 2u);
  }
  __syncthreads();
  // the k selected indices, ascending
  if (k <= 1024) {
    for (int q = threadIdx.x; q < k; q += blockDim.x) {
      const int32_t x = sel[q];
      int rank = 0;
      for (int q2 = 0; q2 < k; ++q2) rank += (sel[q2] < x) ? 1 : 0;
      const bool ok = x >= 0 && x < p && rank < k;  // always true when the counts agree
      if (!ok) atomicOr(&tw.state[3], 2u);
      if (rank < k) {
        support[rank] = ok ? x : 0;
        if (vals) vals[rank] = ok ? src.at(x) : 0.0;
      }
    }
  } else {
    int N = 1;
    while (N < k) N <<= 1;
    for (int q = threadIdx.x; q < N; q += blockDim.x)
      if (q >= k) sel[q] = 0x7FFFFFFF;
    __syncthreads();
    for (int size = 2; size <= N; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < N / 2; i += blockDim.x) {
          const int lo = 2 * i - (i & (stride - 1));
          const int hi = lo + stride;
          const bool asc = (lo & size) == 0;
          const int32_t a = sel[lo], c2 = sel[hi];
          if ((a > c2) == asc) {
            sel[lo] = c2;
            sel[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    for (int q = threadIdx.x; q < k; q += blockDim.x) {
      const int32_t x = sel[q];
      const bool ok = x >= 0 && x < p;  // always true when the counts agree
      if (!ok) atomicOr(&tw.state[3], 2u);
      support[q] = ok ? x : 0;
      if (vals) vals[q] = ok ? src.at(x) : 0.0;
    }
  }
  if (threadIdx.x == 0) {
    tw.counters[1] = 0u;
    tw.counters[2] = 0u;
    tw.counters[3] = 0u;
  }
}

// ------------------------------------------------------------------------------------------------
// Two-pass top-k for k <= kLocalMaxK (no global atomics, no fences). Pass 1: each block takes a
// chunk of the row, keeps its values in registers and marks its own k first entries in the total
// order (|w| descending, index ascending) by radix select on the unique 96-bit composite
// (|w| bits, ~index); it writes them to its kmax candidate slots (unused slots index -1). The row's
// k first entries are among the union of the blocks' k first. Pass 2: one block per row selects
// the k first of all candidates the same way and sorts them by index.

constexpr int kSelBits = 11;
constexpr int kSelBins = 1 << kSelBits;  // 2048: two bins per thread of a 1024-thread block
constexpr int kLocalMaxK = 512;
constexpr int kLocalEPT = 8;   // entries per thread in pass 1: chunks of 8192
constexpr int kFinalEPT = 8;   // candidates per thread in pass 2: up to 8192 per row
constexpr int64_t kSmallChunk = 256 * kLocalEPT;   // pass-1 chunk of a 256-thread block
constexpr int64_t kLargeChunk = 1024 * kLocalEPT;  // pass-1 chunk of a 1024-thread block
constexpr int64_t kRankMax = 256;  // pass-2 lists ranked pairwise; longer ones by radix selection
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 sel_comp(uint64_t key, int32_t idx) {
  return ((u128)key << 32) | (u128)(0xFFFFFFFFu - (uint32_t)idx);
}

// Sum of v over the threads >= tid (THREADS-thread block; sh holds THREADS / 64 words).
template <int THREADS>
__device__ __forceinline__ uint32_t block_suffix_sum(uint32_t v, uint32_t* sh) {
  constexpr int W = THREADS / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_down(x, off, 64);
    if (lane + off < 64) x += y;
  }
  if (lane == 0) sh[w] = x;
  __syncthreads();
  uint32_t add = 0;
  for (int w2 = w + 1; w2 < W; ++w2) add += sh[w2];
  __syncthreads();
  return x + add;
}

// Bit e of the result: entry e of this thread is among the k first valid entries of the block in
// the total order; idx_of(e) gives the entry's index (-1: no entry). Radix select on the composite,
// 11 bits at a time from the top (while the digit lies in the key, 64-bit arithmetic only),
// stopping as soon as the bucket holding the k-th entry is taken whole. Thread t owns the
// kSelBins / THREADS consecutive bins from BPT t. Needs 1 <= k <= number of valid entries, E <= 32.
template <int THREADS, int E, class IdxOf>
__device__ uint32_t block_select(const uint64_t (&key)[E], IdxOf idx_of, uint32_t k, uint32_t* hist, uint32_t* sh) {
  static_assert(E <= 32, "selection mask");
  constexpr int BPT = kSelBins / THREADS;  // 2 (1024 threads) or 8 (256 threads)
  constexpr int SH = THREADS / 64;         // sh[SH .. SH + 2] carry the chosen bin
  const int tid = threadIdx.x;
  u128 prefix = 0;
  uint32_t need = k;
  int s = 96;  // composite bits [s, 96) are fixed by prefix
  while (s > 0) {
    const int ns = s > kSelBits ? s - kSelBits : 0;
    const int nbits = s - ns;
    const uint32_t dmask = (1u << nbits) - 1u;
#pragma unroll
    for (int i = 0; i < BPT; ++i) hist[BPT * tid + i] = 0u;
    __syncthreads();
    if (ns >= 32) {  // digit and prefix inside the key
      const uint64_t pk = (uint64_t)prefix;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (idx_of(e) >= 0 && (s - 32 >= 64 ? 0ull : (key[e] >> (s - 32))) == pk)
          atomicAdd(&hist[(uint32_t)(key[e] >> (ns - 32)) & dmask], 1u);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int32_t ix = idx_of(e);
        if (ix >= 0) {
          const u128 c = sel_comp(key[e], ix);
          if ((c >> s) == prefix) atomicAdd(&hist[(uint32_t)(c >> ns) & dmask], 1u);
        }
      }
    }
    __syncthreads();
    uint32_t h[BPT], tot = 0;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      h[i] = hist[BPT * tid + i];
      tot += h[i];
    }
    const uint32_t incl = block_suffix_sum<THREADS>(tot, sh);  // entries in bins >= BPT tid
    const uint32_t excl = incl - tot;                          // entries in bins >= BPT (tid + 1)
    if (excl < need && incl >= need) {
      uint32_t acc = excl;
#pragma unroll
      for (int i = BPT - 1; i >= 0; --i) {
        if (acc < need && acc + h[i] >= need) {
          sh[SH] = (uint32_t)(BPT * tid + i);
          sh[SH + 1] = acc;
          sh[SH + 2] = h[i];
        }
        acc += h[i];
      }
    }
    __syncthreads();
    const uint32_t b = sh[SH], above = sh[SH + 1], cnt = sh[SH + 2];
    prefix = (prefix << nbits) | (u128)b;
    need -= above;
    s = ns;
    __syncthreads();  // everyone has read the chosen bin
    if (cnt == need) break;
  }
  uint32_t take = 0u;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t ix = idx_of(e);
    if (ix >= 0 && (sel_comp(key[e], ix) >> s) >= prefix) take |= 1u << e;
  }
  return take;
}

template <int THREADS, int EPT>
__global__ __launch_bounds__(THREADS) void k_topk_local(TopkJob J, int64_t p) {
  TopkRow src;
  if (!topk_row(J, blockIdx.y, src)) return;
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t sh[32];
  __shared__ uint32_t nout;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * (THREADS * EPT);
  auto idx_of = [&](int e) -> int32_t {
    const int64_t j = base + (int64_t)e * THREADS + tid;
    return j < p ? (int32_t)j : -1;
  };
  uint64_t key[EPT];
  bool bad = false;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int32_t j = idx_of(e);
    const double w = j >= 0 ? src.at(j) : 0.0;
    bad |= !isfinite(w);
    key[e] = abs_key(w);
  }
  if (bad) atomicOr(&src.tw.state[3], 1u);
  const int64_t nvalid = min((int64_t)(THREADS * EPT), p - base);
  uint32_t take = 0u;
  if (nvalid <= (int64_t)src.k) {
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (idx_of(e) >= 0) take |= 1u << e;
  } else {
    take = block_select<THREADS, EPT>(key, idx_of, (uint32_t)src.k, hist, sh);
  }
  if (tid == 0) nout = 0u;
  __syncthreads();
  uint64_t* ok = src.tw.cand_key + (int64_t)blockIdx.x * J.kmax;
  int32_t* oi = src.tw.cand_idx + (int64_t)blockIdx.x * J.kmax;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    if (take & (1u << e)) {
      const uint32_t pos = atomicAdd(&nout, 1u);  // < min(k, nvalid) <= kmax
      ok[pos] = key[e];
      oi[pos] = idx_of(e);
    }
  }
  __syncthreads();
  for (int q = (int)nout + tid; q < J.kmax; q += THREADS) oi[q] = -1;
}

// Bound for the filter of a solver row (beta and prev = its ascending support): the k-th largest
// key among the support's k entries and the first kBoundSlots - k entries of the row outside the
// support. These are distinct indices, so the bound is at most the row's k-th largest key (each of
// the k first, ties included, is at or above it) and at least the smallest key over the support.
// The sample makes it tight when some support entries are small (k above the number of effects):
// about k p / kBoundSlots entries of the row then pass the filter instead of nearly all of them.
// Written to state[4] (low word) and state[5] (high word); 0 (no bound) if fewer than k valid
// entries were seen. A row takes the sample only once one of its filters has let more than
// kLooseCandidates entries through (state[6], set by k_topk_final, cleared with the error word);
// until then the bound is the smallest key over the support, which costs k loads.
constexpr int kBoundEPT = 8;
constexpr int kBoundSlots = 1024 * kBoundEPT;
constexpr uint32_t kLooseCandidates = 1024;
static_assert(kBoundSlots > kLocalMaxK, "the sample must hold the support");

__global__ __launch_bounds__(1024) void k_topk_bound(TopkJob J, int64_t p) {
  TopkRow src;
  if (!topk_row(J, blockIdx.x, src)) return;
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t sh[32];
  __shared__ uint64_t shm[16];
  __shared__ uint32_t total;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = src.k;
  const int64_t* prev = J.prev + (int64_t)blockIdx.x * J.ldprev;
  if (src.tw.state[6] == 0u) {
    uint64_t tk = ~0ull;
    for (int q = tid; q < k; q += 1024) {
      const int64_t h = prev[q];
      const uint64_t kq = (h >= 0 && h < p) ? abs_key(src.at(h)) : (uint64_t)0;  // out of range: no bound
      tk = kq < tk ? kq : tk;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(tk, off, 64);
      tk = o < tk ? o : tk;
    }
    if (lane == 0) shm[w] = tk;
    __syncthreads();
    if (tid == 0) {
      uint64_t m = shm[0];
      for (int i = 1; i < 16; ++i) m = shm[i] < m ? shm[i] : m;
      src.tw.state[4] = (uint32_t)m;
      src.tw.state[5] = (uint32_t)(m >> 32);
    }
    return;
  }
  // the support in LDS for the membership searches (k <= kLocalMaxK on this path)
  __shared__ int64_t sprev[kLocalMaxK];
  for (int q = tid; q < k; q += 1024) sprev[q] = prev[q];
  __syncthreads();
  int32_t idx[kBoundEPT];
  uint64_t key[kBoundEPT];
  uint32_t nv = 0;
#pragma unroll
  for (int e = 0; e < kBoundEPT; ++e) {
    const int i = e * 1024 + tid;
    int64_t j;
    bool ok;
    double v = 0.0;
    if (i < k) {
      j = sprev[i];
      ok = j >= 0 && j < p;
      if (ok) v = src.at(j);
    } else {
      j = i - k;
      ok = j < p;
      if (ok) {  // skip the support's own indices
        int lo = 0, hi = k;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sprev[mid] < j)
            lo = mid + 1;
          else
            hi = mid;
        }
        ok = !(lo < k && sprev[lo] == j);
        if (ok) v = __dmul_rn(src.mu, src.g[j]);  // beta is zero off the support
      }
    }
    ok = ok && isfinite(v);
    idx[e] = ok ? (int32_t)j : -1;
    key[e] = abs_key(v);
    nv += ok ? 1u : 0u;
  }
  const uint32_t all = block_suffix_sum<1024>(nv, sh);
  if (tid == 0) total = all;
  __syncthreads();
  if (total < (uint32_t)k) {
    if (tid == 0) {
      src.tw.state[4] = 0u;
      src.tw.state[5] = 0u;
    }
    return;
  }
  const uint32_t take = block_select<1024, kBoundEPT>(key, [&](int e) { return idx[e]; }, (uint32_t)k, hist, sh);
  uint64_t mn = ~0ull;
#pragma unroll
  for (int e = 0; e < kBoundEPT; ++e)
    if ((take >> e) & 1u) mn = key[e] < mn ? key[e] : mn;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mn, off, 64);
    mn = o < mn ? o : mn;
  }
  if (lane == 0) shm[w] = mn;
  __syncthreads();
  if (tid == 0) {
    uint64_t m = shm[0];
    for (int i = 1; i < 16; ++i) m = shm[i] < m ? shm[i] : m;
    src.tw.state[4] = (uint32_t)m;
    src.tw.state[5] = (uint32_t)(m >> 32);
  }
}

// Pass 1 with a threshold (TopkJob::prev): the smallest key over the row's k distinct previous
// indices is at most the k-th largest key, so every entry at or above it is a candidate (a superset
// of the k first, ties included); for a solver row the tighter bound of k_topk_bound is used. Each wave appends its candidates to the row's list with one atomic add;
// the order of the list does not matter to pass 2.
__global__ __launch_bounds__(256) void k_topk_filter(TopkJob J, int64_t p, int32_t cpb) {
  TopkRow src;
  if (!topk_row(J, blockIdx.y, src)) return;
  __shared__ uint64_t shk[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t* prev = J.prev + (int64_t)blockIdx.y * J.ldprev;
  // (64-bit keys compared as integers throughout: no min() overload that could convert them)
  uint64_t tk = ~0ull;
  if (J.use_bound) {
    tk = (uint64_t)src.tw.state[4] | ((uint64_t)src.tw.state[5] << 32);
  } else {
    for (int q = tid; q < src.k; q += 256) {
      const int64_t h = prev[q];
      const uint64_t kq = (h >= 0 && h < p) ? abs_key(src.at(h)) : (uint64_t)0;  // out of range: no bound
      tk = kq < tk ? kq : tk;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(tk, off, 64);
      tk = o < tk ? o : tk;
    }
    if (lane == 0) shk[w] = tk;
    __syncthreads();
    tk = shk[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) tk = shk[i] < tk ? shk[i] : tk;
  }
  if (J.certify) {  // values off the exact support may be off by err: keep 2 err below the bound
    const double lo = __longlong_as_double((long long)tk) - 2.0 * row_err(J, blockIdx.y, src);
    tk = lo > 0.0 ? abs_key(lo) : 0ull;
  }
  // Appends this wave's `in` lanes to the row's candidate list: one atomic add per wave.
  auto append = [&](bool in, uint64_t key, int64_t j) {
    const uint64_t m = __ballot(in);
    if (m == 0ull) return;
    uint32_t at = 0u;
    if (lane == __ffsll((long long)m) - 1) at = atomicAdd(&src.tw.counters[4], (uint32_t)__popcll(m));
    at = __shfl(at, __ffsll((long long)m) - 1, 64);
    const uint32_t pos = at + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (in && (int64_t)pos < J.cap) {  // the count starts at 0 and cannot pass p <= cap
      src.tw.cand_key[pos] = key;
      src.tw.cand_idx[pos] = (int32_t)j;
    }
  };
  // With beta (w = beta + mu g), prev is the support of beta, ascending: beta is zero elsewhere, so
  // there w = mu g exactly and only g is read; the support's own entries are appended once, by the
  // row's first block, and skipped by the scan.
  const bool on_support = src.beta != nullptr;
  bool bad = false;
  if (on_support && blockIdx.x == 0) {
    for (int q0 = 0; q0 < src.k; q0 += 256) {
      const int q = q0 + tid;
      const double v = q < src.k ? src.at(prev[q]) : 0.0;
      bad |= !isfinite(v);
      append(q < src.k, abs_key(v), q < src.k ? prev[q] : 0);
    }
  }
  // chunks blockIdx.x * cpb .. + cpb - 1 of 2048 entries
  for (int cb = 0; cb < cpb; ++cb) {
    const int64_t base = ((int64_t)blockIdx.x * cpb + cb) * kSmallChunk;
    if (base >= p) break;  // uniform
    if (J.gmax && on_support) {
      // the chunk's largest |g| from the gradient pass (per 128 indices; each wave reads them):
      // when even |mu| times it is below the threshold, no entry of the chunk can pass (the FP64
      // product rounds monotonically)
      const int64_t g0 = base / kGmaxSnps;
      const int64_t ng = min((int64_t)(kSmallChunk / kGmaxSnps), (p + kGmaxSnps - 1) / kGmaxSnps - g0);
      uint64_t m = (lane < ng) ? J.gmax[(int64_t)blockIdx.y * J.ldm + g0 + lane] : 0ull;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
      }
      if (abs_key(__dmul_rn(fabs(src.mu), key_value(m))) < tk) continue;  // uniform
    }
    uint64_t key[kLocalEPT];
#pragma unroll
    for (int e = 0; e < kLocalEPT; ++e) {
      const int64_t j = base + (int64_t)e * 256 + tid;
      const double v = j < p ? (on_support ? __dmul_rn(src.mu, src.g[j]) : src.at(j)) : 0.0;
      bad |= !isfinite(v);
      key[e] = abs_key(v);
    }
#pragma unroll
    for (int e = 0; e < kLocalEPT; ++e) {
      const int64_t j = base + (int64_t)e * 256 + tid;
      bool in = j < p && key[e] >= tk;
      if (in && on_support) {  // rare: only entries at or above the bound search the support
        int lo = 0, hi = src.k;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (prev[mid] < j)
            lo = mid + 1;
          else
            hi = mid;
        }
        in = !(lo < src.k && prev[lo] == j);
      }
      append(in, key[e], j);
    }
  }
  if (bad) atomicOr(&src.tw.state[3], 1u);
}

// Radix select, by one block, of the k first of n candidates held in global memory (the same
// composite order as block_select): on return the selected ones are those whose composite >> s is
// >= prefix. Used when a filtered candidate list is too long for registers.
__device__ void select_global(const uint64_t* __restrict__ keys, const int32_t* __restrict__ idx, int64_t n, uint32_t k,
                              uint32_t* hist, uint32_t* sh, u128& prefix_out, int& s_out) {
  const int tid = threadIdx.x;
  u128 prefix = 0;
  uint32_t need = k;
  int s = 96;
  while (s > 0) {
    const int ns = s > kSelBits ? s - kSelBits : 0;
    const int nbits = s - ns;
    const uint32_t dmask = (1u << nbits) - 1u;
    hist[2 * tid] = 0u;
    hist[2 * tid + 1] = 0u;
    __syncthreads();
    for (int64_t q = tid; q < n; q += 1024) {
      const u128 c = sel_comp(keys[q], idx[q]);
      if ((c >> s) == prefix) atomicAdd(&hist[(uint32_t)(c >> ns) & dmask], 1u);
    }
    __syncthreads();
    const uint32_t h0 = hist[2 * tid], h1 = hist[2 * tid + 1];
    const uint32_t incl = block_suffix_sum<1024>(h0 + h1, sh);
    const uint32_t excl = incl - h0 - h1;
    if (excl < need && incl >= need) {
      if (excl + h1 >= need) {
        sh[16] = 2u * tid + 1u;
        sh[17] = excl;
        sh[18] = h1;
      } else {
        sh[16] = 2u * tid;
        sh[17] = excl + h1;
        sh[18] = h0;
      }
    }
    __syncthreads();
    const uint32_t b = sh[16], above = sh[17], cnt = sh[18];
    prefix = (prefix << nbits) | (u128)b;
    need -= above;
    s = ns;
    __syncthreads();
    if (cnt == need) break;
  }
  prefix_out = prefix;
  s_out = s;
}

// Pass 2, one block per row: the k first of the row's candidates (nb blocks x kmax slots, or the
// filtered list), sorted by index. With save (a certified row's first selection), the list length
// and the k-th largest key of the selection are left in counters[5], counters[6..7] for
// k_topk_exact, and the list is kept.
__global__ __launch_bounds__(1024) void k_topk_final(TopkJob J, int64_t p, int32_t nb, int32_t save) {
  TopkRow src;
  if (!topk_row(J, blockIdx.x, src)) return;
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t sh[32];
  __shared__ int32_t sel[kLocalMaxK];
  __shared__ uint32_t nsel;
  __shared__ unsigned long long kth;
  const int tid = threadIdx.x;
  const int k = src.k;
  int64_t total = (int64_t)nb * J.kmax;  // <= 1024 * kFinalEPT (checked at launch)
  if (J.prev) {
    // the count was formed by device-scope atomics: take it (and reset it) with one, so that no
    // cached copy of the word is read
    if (tid == 0) {
      const uint32_t c = atomicExch(&src.tw.counters[4], 0u);
      nsel = c;
      if ((int64_t)c < k) atomicOr(&src.tw.state[3], 4u);  // the bound came from repeated indices
      if (c > kLooseCandidates) src.tw.state[6] = 1u;      // later bounds of this row use the sample
    }
    __syncthreads();
    total = min((int64_t)nsel, J.cap);
    __syncthreads();  // every thread has read it before nsel is reused
  }
  if (tid == 0) {
    nsel = 0u;
    kth = ~0ull;
  }
  for (int q = tid; q < kLocalMaxK; q += 1024) sel[q] = 0;
  __syncthreads();
  if (total <= kRankMax || (total <= 1024 && total < k)) {  // (fewer than k: flagged below)
    // short lists (a warm-started projection): the exact rank of each candidate in the total order
    // (|w| descending, index ascending) against the others in LDS; the k of rank < k are the result.
    // Every thread reads the whole list, so the LDS traffic grows with its square: past kRankMax
    // entries the radix selection below is faster (a 1000-entry list reads 12 MB of LDS on one CU).
    uint64_t* ck = reinterpret_cast<uint64_t*>(hist);  // the histogram's 8 KB hold the 1024 keys
    __shared__ int32_t cidx[1024];
    if (tid < total) {
      ck[tid] = src.tw.cand_key[tid];
      cidx[tid] = src.tw.cand_idx[tid];
    }
    __syncthreads();
    if (tid < total && cidx[tid] >= 0) {
      const uint64_t kq = ck[tid];
      const int32_t iq = cidx[tid];
      int rank = 0;
      for (int q2 = 0; q2 < (int)total; ++q2) {
        const int32_t i2 = cidx[q2];
        rank += (i2 >= 0 && key_before(ck[q2], i2, kq, iq)) ? 1 : 0;
      }
      if (rank < k) {
        const uint32_t pos = atomicAdd(&nsel, 1u);
        if (pos < (uint32_t)kLocalMaxK) sel[pos] = iq;
      }
    }
  } else if (total <= 1024 * (int64_t)kFinalEPT) {
    uint64_t key[kFinalEPT];
    int32_t idx[kFinalEPT];
#pragma unroll
    for (int e = 0; e < kFinalEPT; ++e) {
      const int64_t q = tid + (int64_t)e * 1024;
      idx[e] = q < total ? src.tw.cand_idx[q] : -1;
      key[e] = idx[e] >= 0 ? src.tw.cand_key[q] : 0;
    }
    const uint32_t take = block_select<1024, kFinalEPT>(key, [&](int e) { return idx[e]; }, (uint32_t)k, hist, sh);
#pragma unroll
    for (int e = 0; e < kFinalEPT; ++e) {
      if (take & (1u << e)) {
        const uint32_t pos = atomicAdd(&nsel, 1u);
        if (pos < (uint32_t)kLocalMaxK) sel[pos] = idx[e];
      }
    }
  } else {
    u128 prefix;
    int s;
    select_global(src.tw.cand_key, src.tw.cand_idx, total, (uint32_t)k, hist, sh, prefix, s);
    for (int64_t q = tid; q < total; q += 1024) {
      const int32_t ix = src.tw.cand_idx[q];
      if ((sel_comp(src.tw.cand_key[q], ix) >> s) >= prefix) {
        const uint32_t pos = atomicAdd(&nsel, 1u);
        if (pos < (uint32_t)kLocalMaxK) sel[pos] = ix;
      }
    }
  }
  __syncthreads();
  if (nsel != (uint32_t)k) {
    // cannot happen for a valid job (flagged; the caller reports an error): the output still gets
    // k valid indices, so that nothing downstream indexes with an unset entry
    if (tid == 0) atomicOr(&src.tw.state[3], 2u);
    for (int q = tid; q < k; q += 1024) {
      src.out[q] = q;
      if (src.vals) src.vals[q] = 0.0;
    }
    return;
  }
  // the k selected indices, ascending (indices are distinct)
  for (int q = tid; q < k; q += 1024) {
    const int32_t x = sel[q];
    int rank = 0;
    for (int q2 = 0; q2 < k; ++q2) rank += (sel[q2] < x) ? 1 : 0;
    const bool ok = x >= 0 && x < p && rank < k;  // always true when the counts agree
    if (!ok) atomicOr(&src.tw.state[3], 2u);
    if (rank < k) {
      const double w = ok ? src.at(x) : 0.0;
      src.out[rank] = ok ? x : 0;
      if (src.vals) src.vals[rank] = w;
      if (save) atomicMin(&kth, (unsigned long long)abs_key(w));
    }
  }
  if (save) {
    __syncthreads();
    if (tid == 0) {
      (void)atomicExch(&src.tw.counters[5], (uint32_t)total);
      (void)atomicExch(&src.tw.counters[6], (uint32_t)kth);
      (void)atomicExch(&src.tw.counters[7], (uint32_t)(kth >> 32));
    }
  }
}

// Certified selection, between the two final selections of a certified row: every entry of the
// row's filtered list whose value lies within 2 err below the approximate k-th largest (and, when the
// values at prev are exact, is off prev) gets its exact gradient in FP64, g_j = sum_i x_st(i, j)
// rc_i over the decoded standardised column (missing and outside the subject set: 0), written to g
// and to the list's key. Every entry left approximate is then below the exact k-th largest, so the
// second selection returns the projection of the exact w. One wave per entry to evaluate; the list
// length is restored for the second selection.
__global__ __launch_bounds__(256) void k_topk_exact(TopkJob J, int64_t p) {
  TopkRow src;
  const int t = blockIdx.y;
  if (!topk_row(J, t, src)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t cnt = atomic_load_u32(&src.tw.counters[5]);
  const uint64_t kkey = (uint64_t)atomic_load_u32(&src.tw.counters[6]) | ((uint64_t)atomic_load_u32(&src.tw.counters[7]) << 32);
  const double lo = key_value(kkey) - 2.0 * row_err(J, t, src);
  const int64_t* prev = J.prev + (int64_t)t * J.ldprev;
  // the row's support in LDS for the membership searches (k <= kLocalMaxK on certified rows)
  __shared__ int64_t sprev[kLocalMaxK];
  if (J.prev_exact) {
    for (int q = threadIdx.x; q < src.k; q += blockDim.x) sprev[q] = prev[q];
    __syncthreads();
  }
  const BatchSolve sv = J.sv[t];
  const double* rc = J.rc + (int64_t)t * J.ldr;
  double* g = const_cast<double*>(src.g);
  const int64_t len = min((int64_t)cnt, J.cap);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + w) * 64; c0 < len; c0 += waves * 64) {
    const int64_t pos = c0 + lane;
    int32_t j = -1;
    bool need = false;
    if (pos < len) {
      j = src.tw.cand_idx[pos];
      need = j >= 0 && j < p && key_value(src.tw.cand_key[pos]) >= lo;
      if (need && J.prev_exact) {  // warm row: values on the support are exact already
        int a = 0, b = src.k;
        while (a < b) {
          const int mid = (a + b) >> 1;
          if (sprev[mid] < j)
            a = mid + 1;
          else
            b = mid;
        }
        need = !(a < src.k && sprev[a] == j);
      }
    }
    uint64_t m = __ballot(need);
    while (m) {
      const int bl = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int32_t jj = __shfl(j, bl, 64);
      const double uj = sv.u[jj], vj = sv.v[jj];
      const int rot = jj & (kSegBytes - 1);
      // lane l takes tiles l, l + 64, ...: one 8-byte segment (32 subjects) per tile; byte b of the
      // segment holds 4-subject group (b + rot) mod 8. Subjects past n have code 0 and rc 0.
      const uint2* seg = reinterpret_cast<const uint2*>(J.tiled) + jj;
      double a = 0.0;
      for (int64_t t = lane; t < J.ntiles; t += 64) {
        const uint2 d = seg[t * J.p_pad];
        const double* rt = rc + t * kTileSubjects;
#pragma unroll
        for (int b = 0; b < kSegBytes; ++b) {
          const uint32_t byte = ((b < 4 ? d.x : d.y) >> (8 * (b & 3))) & 0xFFu;
          const int grp = (b + rot) & (kSegBytes - 1);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int code = (int)((byte >> (2 * q)) & 3u);
            const double x = code == 1 ? 0.0 : vj * ((code == 0 ? 0.0 : (double)(code - 1)) - uj);
            a += x * rt[4 * grp + q];
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
      if (lane == 0) {
        g[jj] = a;
        src.tw.cand_key[c0 + bl] = abs_key(src.at(jj));
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) (void)atomicExch(&src.tw.counters[4], cnt);
}

// Subject mask of a stats handle: mask[i] = bit i of the tile bits (given), or every subject i < n
// (bits written too).
__global__ void k_subject_mask(int32_t have_bits, uint32_t* __restrict__ bits, double* __restrict__ mask, int64_t n,
                               int64_t n_pad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  if (have_bits) {
    mask[i] = (bits[i / kTileSubjects] >> (i % kTileSubjects)) & 1u ? 1.0 : 0.0;
    return;
  }
  mask[i] = i < n ? 1.0 : 0.0;
  if (i % kTileSubjects == 0) {
    const int64_t left = n - i;  // subjects of this tile
    bits[i / kTileSubjects] = left >= kTileSubjects ? 0xFFFFFFFFu : (left > 0 ? (1u << left) - 1u : 0u);
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0u;
}

__global__ void k_topk_clear_errors(uint32_t* __restrict__ small, int32_t rows, const int32_t* __restrict__ flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < rows && (!flags || flags[t])) {  // words that kernels update with device-scope atomics are cleared with one
    (void)atomicExch(&small[t * kTopkRowWords + kTopkErrorWord], 0u);
    (void)atomicExch(&small[t * kTopkRowWords + kTopkBins0 + 4], 0u);  // filtered-candidate count
    (void)atomicExch(&small[t * kTopkRowWords + kTopkBins0 + 8 + 6], 0u);  // the row's sampled-bound flag
  }
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = val;
}

__global__ void k_scatter(const int64_t* __restrict__ idx, const double* __restrict__ vals, int32_t k, int64_t p,
                          double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < k) {
    const int64_t j = idx[q];
    if (j >= 0 && j < p) out[j] = vals[q];
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// Launchers

hipError_t launch_retile(const uint8_t* raw, int64_t row_bytes, const Layout& L, uint8_t* tiled, hipStream_t st) {
  const dim3 grid((unsigned)(L.p_pad / kRetileSnps), (unsigned)((L.ntiles + kRetileTiles - 1) / kRetileTiles));
  hipLaunchKernelGGL(k_retile, grid, dim3(256), 0, st, raw, row_bytes, L.n, L.p, L.p_pad, L.ntiles, tiled);
  return hipGetLastError();
}

hipError_t launch_stats(const uint8_t* tiled, const Layout& L, const uint32_t* mask_bits, int64_t nT, double* u, double* v,
                        hipStream_t st) {
  const int64_t blocks = (L.p + 255) / 256;
  if (nT == L.n)  // the whole subject set: no mask
    hipLaunchKernelGGL(k_stats<true>, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<const uint2*>(tiled), L.p,
                       L.p_pad, L.ntiles, mask_bits, nT, u, v);
  else
    hipLaunchKernelGGL(k_stats<false>, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<const uint2*>(tiled), L.p,
                       L.p_pad, L.ntiles, mask_bits, nT, u, v);
  return hipGetLastError();
}

hipError_t launch_topk(const TopkJob& J, int64_t p, int32_t rows, hipStream_t st) {
  // two-pass selection when every row's candidates fit pass 2: chunks of 2048 (256-thread blocks,
  // enough of them to fill the chip) when they do, else of 8192
  const int64_t cap2 = 1024 * (int64_t)kFinalEPT;
  const int64_t nb_s = (p + kSmallChunk - 1) / kSmallChunk;
  const int64_t nb_l = (p + kLargeChunk - 1) / kLargeChunk;
  // A certified row's filtered list is selected from twice: first by the approximate values, then,
  // after k_topk_exact has made the entries near the k-th largest exact, by those.
  // chunks per filter block: one while the launch has at most 8192 blocks, else enough (up to 8) to
  // keep it near that; most blocks of a many-row launch read little (the summary skip) or nothing
  // (gated rows), and their dispatch alone costs time
  const int64_t cpb = std::min<int64_t>(8, std::max<int64_t>(1, (nb_s * rows + 8191) / 8192));
  auto filter_final = [&](const TopkJob& Jf) -> hipError_t {
    hipLaunchKernelGGL(k_topk_filter, dim3((unsigned)((nb_s + cpb - 1) / cpb), (unsigned)rows), dim3(256), 0, st, Jf, p,
                       (int32_t)cpb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_final, dim3((unsigned)rows), dim3(1024), 0, st, Jf, p, 0, Jf.certify);
    e = hipGetLastError();
    if (e != hipSuccess || !Jf.certify) return e;
    hipLaunchKernelGGL(k_topk_exact, dim3(8u, (unsigned)rows), dim3(256), 0, st, Jf, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_final, dim3((unsigned)rows), dim3(1024), 0, st, Jf, p, 0, 0);
    return hipGetLastError();
  };
  if (J.certify && !(J.fs && J.kmax <= kLocalMaxK && J.cap >= p)) return hipErrorInvalidValue;
  if (J.prev && J.kmax <= kLocalMaxK && J.cap >= p) {
    TopkJob Jf = J;
    Jf.use_bound = J.beta != nullptr ? 1 : 0;  // solver rows: prev is beta's ascending support
    Jf.prev_exact = Jf.use_bound;               // whose gradient entries a certified row keeps exact
    if (Jf.use_bound) {
      hipLaunchKernelGGL(k_topk_bound, dim3((unsigned)rows), dim3(1024), 0, st, Jf, p);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return filter_final(Jf);
  }
  // a certified cold row: the approximate top-k below, then a filter with it as the hint
  TopkJob Jc = J;
  Jc.prev = J.out;
  Jc.ldprev = J.ldo;
  Jc.prev_exact = 0;  // approximate values (with beta, every beta entry is 0 on a cold row)
  if (J.kmax <= kLocalMaxK && nb_s * J.kmax <= cap2 && nb_s * J.kmax <= J.cap) {
    hipLaunchKernelGGL((k_topk_local<256, kLocalEPT>), dim3((unsigned)nb_s, (unsigned)rows), dim3(256), 0, st, J, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_final, dim3((unsigned)rows), dim3(1024), 0, st, J, p, (int32_t)nb_s, 0);
    e = hipGetLastError();
    return (e != hipSuccess || !J.certify) ? e : filter_final(Jc);
  }
  if (J.kmax <= kLocalMaxK && nb_l * J.kmax <= cap2 && nb_l * J.kmax <= J.cap) {
    hipLaunchKernelGGL((k_topk_local<1024, kLocalEPT>), dim3((unsigned)nb_l, (unsigned)rows), dim3(1024), 0, st, J, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_final, dim3((unsigned)rows), dim3(1024), 0, st, J, p, (int32_t)nb_l, 0);
    e = hipGetLastError();
    return (e != hipSuccess || !J.certify) ? e : filter_final(Jc);
  }
  // histogram path (large k or very long rows): about 2048 blocks over all rows, 4096 to 65536
  // entries per block; a certified row then filters with its result as the hint, as above
  int64_t chunk = 4096;
  while (chunk < 65536 && (p + chunk - 1) / chunk * rows > 2048) chunk <<= 1;
  const dim3 grid((unsigned)((p + chunk - 1) / chunk), (unsigned)rows);
  hipLaunchKernelGGL(k_topk_hist, grid, dim3(1024), 0, st, J, p, chunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_topk_collect, grid, dim3(1024), 0, st, J, p, chunk);
  e = hipGetLastError();
  return (e != hipSuccess || !J.certify) ? e : filter_final(Jc);
}

hipError_t launch_subject_mask(const Layout& L, bool have_bits, uint32_t* bits, double* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_subject_mask, dim3((unsigned)((L.n_pad + 255) / 256)), dim3(256), 0, st, (int32_t)have_bits, bits, mask,
                     L.n, L.n_pad);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* x, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

hipError_t launch_topk_clear_errors(uint32_t* small, int32_t rows, const int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_topk_clear_errors, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, small, rows, flags);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double val, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, val);
  return hipGetLastError();
}

hipError_t launch_scatter(const int64_t* idx, const double* vals, int32_t k, int64_t p, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, idx, vals, k, p, out);
  return hipGetLastError();
}

}  // namespace iht
