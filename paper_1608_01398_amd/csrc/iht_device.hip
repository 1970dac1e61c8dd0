// iht_device.hip -- gfx950 kernels of the IHT hot path.
//
// Hot loop (gradient pass, Methods: eq. normal_grad with on-the-fly standardisation):
//   g_j = v_j * ( D_j - u_j * (R - M_j) ),   D_j = sum_i dose_ij r_i,   M_j = sum_{i missing} r_i,
// with r the residual centred over the subject set (R = sum r, ~0). This is X_st^T r written with the
// paper's identity X_st = X diag(v) - 1 u^T diag(v) (Methods, "Bandwidth optimization of IHT") and
// mean-imputed missing entries (x~ = u_j, so they contribute 0). Centring is exact in real
// arithmetic because every standardised column sums to zero over the subject set.
//
// D_j and M_j come from a table in LDS built per subject tile from the residual: for each group of
// 4 subjects and each of the 256 possible packed bytes, (sum of dose*r, sum of missing*r). One
// 16-byte LDS lookup then replaces the decode and 4 multiply-adds of 4 genotypes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "iht_internal.h"

namespace iht {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 stream_load(const uint4* p) {
  const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(x.x, x.y, x.z, x.w);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint2 stream_load2(const uint2* p) {
  const u32x2 x = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
  return make_uint2(x.x, x.y);
}

__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic block sum over 1024 threads (wave tree, then the 16 wave totals in order).
__device__ double block_sum(double x, double* sh) {
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

__device__ __forceinline__ uint32_t spread_nibble(uint32_t m) {  // bit q -> bit 2q
  return (m & 1u) | ((m & 2u) << 1) | ((m & 4u) << 2) | ((m & 8u) << 3);
}

__global__ __launch_bounds__(256) void k_stats(const uint2* __restrict__ tiled, int64_t p, int64_t p_pad, int64_t ntiles,
                                               const uint32_t* __restrict__ mask_bits, int64_t nT, double* __restrict__ u,
                                               double* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  const int rot = (int)(j & (kSegBytes - 1));
  uint32_t het = 0, hom = 0, mis = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const uint32_t m32 = mask_bits[t];
    const uint2 d = tiled[t * p_pad + j];
    const uint32_t dw[2] = {d.x, d.y};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      uint32_t mm = 0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int grp = (4 * q + bb + rot) & (kSegBytes - 1);
        mm |= spread_nibble((m32 >> (4 * grp)) & 15u) << (8 * bb);
      }
      const uint32_t lo = dw[q] & 0x55555555u, hi = (dw[q] >> 1) & 0x55555555u;
      het += __popc(hi & ~lo & mm);
      hom += __popc(hi & lo & mm);
      mis += __popc(lo & ~hi & mm);
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
// The gradient pass.

// LDS table: one 256-byte row per packed byte value v (0..255), 64 KB in all. FP64 rows hold
// [buffer 0: 8 groups x (T, M) 16 B][buffer 1: same]; FP32 rows hold [buffer 0 copy 0: 8 x 8 B]
// [buffer 0 copy 1][buffer 1 copy 0][buffer 1 copy 1]. The buffer is an immediate offset (+128).
// At every lookup step the 8 (FP64, 16-byte reads) or 16 (FP32, two copies) lanes served together
// read 8 different groups, which tile all 32 banks: no conflicts for any data.
template <bool F32>
struct Tab;
template <>
struct Tab<false> {
  static constexpr uint32_t kGroupShift = 4;
  __device__ static uint32_t slot_base(int lane) { return 0u; }
};
template <>
struct Tab<true> {
  static constexpr uint32_t kGroupShift = 3;
  __device__ static uint32_t slot_base(int lane) { return (uint32_t)((lane >> 3) & 1) * 64u; }
};

__device__ __forceinline__ double dose_of(int c) { return c == 3 ? 2.0 : (c == 2 ? 1.0 : 0.0); }
__device__ __forceinline__ double miss_of(int c) { return c == 1 ? 1.0 : 0.0; }

// Builder thread: group gb = tid % 8 and byte values v = tid / 8 + (threads / 8) m. Entries are
// T(v) = sum_k dose(c_k(v)) r_k and M(v) = sum_k [c_k(v) missing] r_k over the group's 4 subjects,
// summed in subject order. 512 threads: 4 values per thread (the 4th subject's code varies);
// 1024 threads: 2 values (the high bit of the 4th subject's code varies).
template <bool F32, int THREADS>
__device__ __forceinline__ void build_entries(char* lds, int buf, int gb, int vb, const double (&r)[4]) {
  static_assert(THREADS == 512 || THREADS == 1024, "builder mapping");
  constexpr int EPT = 2048 / THREADS;
  const int c0 = vb & 3, c1 = (vb >> 2) & 3, c2 = (vb >> 4) & 3;
  const double T6 = (dose_of(c0) * r[0] + dose_of(c1) * r[1]) + dose_of(c2) * r[2];
  const double M6 = (miss_of(c0) * r[0] + miss_of(c1) * r[1]) + miss_of(c2) * r[2];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int v = vb + (THREADS / 8) * m;
    const int c3 = v >> 6;
    const double T = (c3 == 0 || c3 == 1) ? T6 : T6 + dose_of(c3) * r[3];
    const double M = (c3 == 1) ? M6 + r[3] : M6;
    char* row = lds + (v << 8) + buf * 128;
    if constexpr (F32) {
      const float2 e = make_float2((float)T, (float)M);
      *reinterpret_cast<float2*>(row + (gb << 3)) = e;
      *reinterpret_cast<float2*>(row + 64 + (gb << 3)) = e;
    } else {
      *reinterpret_cast<double2*>(row + (gb << 4)) = make_double2(T, M);
    }
  }
}

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) v2d_t lds_double2;
typedef __attribute__((address_space(3))) v2f_t lds_float2;

// Lookups and rotation-invariant tile sum of one SNP's 8-byte segment (buffer BUF).
// The pairings {b, b+4}, {b, b+2}, {0, 1} of byte positions map to the same pairings of subject
// groups for every rotation, and + is commutative, so the tile sum depends only on the column's
// bytes: identical columns give bitwise identical gradients.
template <bool F32>
__device__ __forceinline__ void tile_sum(const char* lds, const uint32_t (&offs)[2], const uint2 d, double& accT,
                                         double& accM) {
  using acc_t = typename std::conditional<F32, float, double>::type;
  acc_t PT[4], PM[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    acc_t vt[2], vm[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = c + 4 * h;
      const uint32_t dw = h ? d.y : d.x;
      // byte0 = slot offset of step b, byte1 = packed value, bytes 2-3 = 0
      const uint32_t sel = (4u + (uint32_t)c) | ((uint32_t)c << 8) | (0x0Cu << 16) | (0x0Cu << 24);
      // the table starts at LDS address 0, so the perm result is the LDS address itself
      const uint32_t addr = __builtin_amdgcn_perm(offs[h], dw, sel);
      if constexpr (F32) {
        const v2f_t e = *reinterpret_cast<const lds_float2*>((size_t)addr);
        vt[h] = e.x;
        vm[h] = e.y;
      } else {
        const v2d_t e = *reinterpret_cast<const lds_double2*>((size_t)addr);
        vt[h] = e.x;
        vm[h] = e.y;
      }
      (void)b;
    }
    PT[c] = vt[0] + vt[1];
    PM[c] = vm[0] + vm[1];
  }
  accT += (double)((PT[0] + PT[2]) + (PT[1] + PT[3]));
  accM += (double)((PM[0] + PM[2]) + (PM[1] + PM[3]));
}

constexpr int kRing = 4;               // tiles of packed data held in registers (prefetch distance 3)
constexpr int kMaxTilesPerBlock = 376;  // residual staged in LDS: 376 * 32 * 8 B next to the 64 KB table

typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// Packed bytes of tile t for the lane's NS SNPs: one buffer resource per tile (scalar base), one
// 32-bit lane offset. Tiles past the block's range get a zero-size resource: the loads return zeros
// without touching memory (and those tiles have all-zero tables).
template <int NS>
__device__ __forceinline__ void load_tile(uint2 (&d)[NS], const uint2* __restrict__ tiled, int64_t p_pad, uint32_t voff,
                                          int t, int t1) {
  const bool real = t < t1;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint2*>(tiled + (int64_t)(real ? t : 0) * p_pad), 0, real ? 0x7FFFFFFF : 0, 0x00020000);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const v2u x = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + (uint32_t)(s * kPassThreads * 8), 0, 2 /* nt */);
    d[s] = make_uint2(x.x, x.y);
  }
}

template <int NS, bool F32>
__global__ __launch_bounds__(kPassThreads, 1) void k_pass(const uint2* __restrict__ tiled, int64_t p, int64_t p_pad, int32_t ntiles,
                                                  int32_t tps, int64_t n, const double* __restrict__ r,
                                                  const double* __restrict__ mask, int64_t nT, const double* __restrict__ u,
                                                  const double* __restrict__ v, FitState* __restrict__ fs,
                                                  double* __restrict__ g, double2* __restrict__ partial,
                                                  const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  // The table sits at LDS address 0 (this kernel has no static LDS), so a v_perm result is the
  // full lookup address; the residual of the block's subjects and the reduction scratch follow it.
  extern __shared__ __attribute__((aligned(16))) uint4 dyn_lds[];
  char* lds = reinterpret_cast<char*>(dyn_lds);               // 256 rows x 256 B table
  double* red = reinterpret_cast<double*>(lds + 65536);      // 40 doubles of reduction scratch
  double* rl = red + 40;                                      // centred residual of this block's subjects
  constexpr uint32_t GS = Tab<F32>::kGroupShift;

  const int tid = threadIdx.x;
  const int t0 = blockIdx.y * tps;
  const int t1 = min(ntiles, t0 + tps);
  const int64_t i0 = (int64_t)t0 * kTileSubjects;
  const int64_t nsub = (int64_t)(t1 - t0) * kTileSubjects;

  const int64_t jb = (int64_t)blockIdx.x * (kPassThreads * NS) + tid;
  const uint32_t voff = (uint32_t)(jb * 8);
  // first tiles in flight before anything else
  uint2 d[kRing][NS];
#pragma unroll
  for (int q = 0; q < kRing - 1; ++q) load_tile<NS>(d[q], tiled, p_pad, voff, t0 + q, t1);

  // Centre the residual over the subject set: X_st^T 1_T = 0, so the gradient is unchanged and the
  // table entries stay small. R = sum of the centred residual (~0) enters the epilogue.
  double mean, R;
  {
    double s1 = 0.0;
    for (int64_t i = tid; i < n; i += kPassThreads) s1 += (mask[i] != 0.0) ? r[i] : 0.0;
    mean = block_sum(s1, red) / (double)nT;
    double s2 = 0.0;
    for (int64_t i = tid; i < n; i += kPassThreads) s2 += (mask[i] != 0.0) ? r[i] - mean : 0.0;
    R = block_sum(s2, red);
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) {
      fs->mean = mean;
      fs->Rsum = R;
    }
    for (int64_t q = tid; q < nsub; q += kPassThreads) {
      const int64_t i = i0 + q;
      rl[q] = (i < n && mask[i] != 0.0) ? r[i] - mean : 0.0;
    }
  }

  const uint32_t rot = (uint32_t)tid & 7u;  // == j & 7 for every SNP slot of this lane
  // offs[B][h] byte c = offset inside a table row of step b = c + 4h in LDS buffer B:
  // B * 128 + copy base + (group (b + rot) mod 8) * entry size.
  uint32_t offs[2][2];
#pragma unroll
  for (int B = 0; B < 2; ++B)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t o = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        o |= ((uint32_t)B * 128u + Tab<F32>::slot_base(tid) + ((((uint32_t)(c + 4 * h) + rot) & 7u) << GS)) << (8 * c);
      offs[B][h] = o;
    }
  const int gb = tid & 7, vb = tid >> 3;

  // residuals of builder group gb in tile t (zero past the block's range -> all-zero table)
  auto group_r = [&](int t, double (&rr)[4]) {
    const bool live = t < t1;
    const int q = live ? (t - t0) * kTileSubjects + gb * 4 : 0;
    const double4 x = *reinterpret_cast<const double4*>(rl + q);
    rr[0] = live ? x.x : 0.0;
    rr[1] = live ? x.y : 0.0;
    rr[2] = live ? x.z : 0.0;
    rr[3] = live ? x.w : 0.0;
  };

  double accT[NS], accM[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    accT[s] = 0.0;
    accM[s] = 0.0;
  }
  __syncthreads();  // residual staged
  {
    double rr[4];
    group_r(t0, rr);
    build_entries<F32, kPassThreads>(lds, 0, gb, vb, rr);
  }
  __syncthreads();

  // Tile t uses ring slot (t - t0) % 4 and LDS buffer (t - t0) % 2, both compile-time in the
  // unrolled body. Each step prefetches tile t+3, builds the table of tile t+1 and consumes tile t.
  // Tiles past t1 (at most 3 in the last trip) have all-zero tables and add exact zeros.
  const int trips = (t1 - t0 + kRing - 1) / kRing;
  for (int trip = 0; trip < trips; ++trip) {
#pragma unroll
    for (int uu = 0; uu < kRing; ++uu) {
      const int t = t0 + trip * kRing + uu;
      load_tile<NS>(d[(uu + kRing - 1) % kRing], tiled, p_pad, voff, t + kRing - 1, t1);
      {
        double rr[4];
        group_r(t + 1, rr);
        build_entries<F32, kPassThreads>(lds, (uu + 1) & 1, gb, vb, rr);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        tile_sum<F32>(lds, offs[uu & 1], d[uu][s], accT[s], accM[s]);
#if IHT_PASS_SNP_BARRIER
        __builtin_amdgcn_sched_barrier(0);
#endif
      }
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
    }
  }

#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int64_t j = jb + s * kPassThreads;
    if (j < p) {
      if (partial) {
        partial[(int64_t)blockIdx.y * p_pad + j] = make_double2(accT[s], accM[s]);
      } else {
        g[j] = v[j] * (accT[s] - u[j] * (R - accM[s]));
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_pass_finalize(const double2* __restrict__ partial, int32_t split, int64_t p,
                                                       int64_t p_pad, const double* __restrict__ u,
                                                       const double* __restrict__ v, const FitState* __restrict__ fs,
                                                       double* __restrict__ g, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  double D = 0.0, M = 0.0;
  for (int s = 0; s < split; ++s) {
    const double2 e = partial[(int64_t)s * p_pad + j];
    D += e.x;
    M += e.y;
  }
  g[j] = v[j] * (D - u[j] * (fs->Rsum - M));
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
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 sel_comp(uint64_t key, int32_t idx) {
  return ((u128)key << 32) | (u128)(0xFFFFFFFFu - (uint32_t)idx);
}

// Sum of v over the threads >= tid (1024-thread block; sh holds 16 words).
__device__ __forceinline__ uint32_t block_suffix_sum(uint32_t v, uint32_t* sh) {
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
  for (int w2 = w + 1; w2 < 16; ++w2) add += sh[w2];
  __syncthreads();
  return x + add;
}

// Bit e of the result: entry e of this thread is among the k first valid entries of the block in
// the total order; idx_of(e) gives the entry's index (-1: no entry). Radix select on the composite,
// 11 bits at a time from the top (while the digit lies in the key, 64-bit arithmetic only),
// stopping as soon as the bucket holding the k-th entry is taken whole. Needs 1 <= k <= number of
// valid entries, E <= 32.
template <int E, class IdxOf>
__device__ uint32_t block_select(const uint64_t (&key)[E], IdxOf idx_of, uint32_t k, uint32_t* hist, uint32_t* sh) {
  static_assert(E <= 32, "selection mask");
  const int tid = threadIdx.x;
  u128 prefix = 0;
  uint32_t need = k;
  int s = 96;  // composite bits [s, 96) are fixed by prefix
  while (s > 0) {
    const int ns = s > kSelBits ? s - kSelBits : 0;
    const int nbits = s - ns;
    const uint32_t dmask = (1u << nbits) - 1u;
    hist[2 * tid] = 0u;
    hist[2 * tid + 1] = 0u;
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
    const uint32_t h0 = hist[2 * tid], h1 = hist[2 * tid + 1];
    const uint32_t incl = block_suffix_sum(h0 + h1, sh);  // entries in bins >= 2 tid
    const uint32_t excl = incl - h0 - h1;                   // entries in bins >= 2 tid + 2
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
    __syncthreads();  // everyone has read sh[16..18]
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

template <int EPT>
__global__ __launch_bounds__(1024) void k_topk_local(TopkJob J, int64_t p) {
  TopkRow src;
  if (!topk_row(J, blockIdx.y, src)) return;
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t sh[32];
  __shared__ uint32_t nout;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * (1024 * EPT);
  auto idx_of = [&](int e) -> int32_t {
    const int64_t j = base + (int64_t)e * 1024 + tid;
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
  const int64_t nvalid = min((int64_t)(1024 * EPT), p - base);
  uint32_t take = 0u;
  if (nvalid <= (int64_t)src.k) {
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (idx_of(e) >= 0) take |= 1u << e;
  } else {
    take = block_select<EPT>(key, idx_of, (uint32_t)src.k, hist, sh);
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
  for (int q = (int)nout + tid; q < J.kmax; q += 1024) oi[q] = -1;
}

__global__ __launch_bounds__(1024) void k_topk_final(TopkJob J, int64_t p, int32_t nb) {
  TopkRow src;
  if (!topk_row(J, blockIdx.x, src)) return;
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t sh[32];
  __shared__ int32_t sel[kLocalMaxK];
  __shared__ uint32_t nsel;
  const int tid = threadIdx.x;
  const int64_t total = (int64_t)nb * J.kmax;  // <= 1024 * kFinalEPT (checked at launch)
  uint64_t key[kFinalEPT];
  int32_t idx[kFinalEPT];
#pragma unroll
  for (int e = 0; e < kFinalEPT; ++e) {
    const int64_t q = tid + (int64_t)e * 1024;
    idx[e] = q < total ? src.tw.cand_idx[q] : -1;
    key[e] = idx[e] >= 0 ? src.tw.cand_key[q] : 0;
  }
  const int k = src.k;
  const uint32_t take = block_select<kFinalEPT>(key, [&](int e) { return idx[e]; }, (uint32_t)k, hist, sh);
  if (tid == 0) nsel = 0u;
  for (int q = tid; q < kLocalMaxK; q += 1024) sel[q] = 0;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kFinalEPT; ++e) {
    if (take & (1u << e)) {
      const uint32_t pos = atomicAdd(&nsel, 1u);
      if (pos < (uint32_t)kLocalMaxK) sel[pos] = idx[e];
    }
  }
  __syncthreads();
  if (tid == 0 && nsel != (uint32_t)k) atomicOr(&src.tw.state[3], 2u);
  // the k selected indices, ascending (indices are distinct)
  for (int q = tid; q < k; q += 1024) {
    const int32_t x = sel[q];
    int rank = 0;
    for (int q2 = 0; q2 < k; ++q2) rank += (sel[q2] < x) ? 1 : 0;
    const bool ok = x >= 0 && x < p && rank < k;  // always true when the counts agree
    if (!ok) atomicOr(&src.tw.state[3], 2u);
    if (rank < k) {
      src.out[rank] = ok ? x : 0;
      if (src.vals) src.vals[rank] = ok ? src.at(x) : 0.0;
    }
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0u;
}

__global__ void k_topk_clear_errors(uint32_t* __restrict__ small, int32_t rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < rows) small[t * kTopkRowWords + kTopkErrorWord] = 0u;
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = val;
}

__global__ void k_scatter(const int64_t* __restrict__ idx, const double* __restrict__ vals, int32_t k,
                          double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < k) out[idx[q]] = vals[q];
}

// ------------------------------------------------------------------------------------------------
// Pass geometry: NS SNPs per lane and `split` subject ranges per SNP block, chosen so one launch
// fills the 256 CUs about once (one 1024-thread workgroup per CU: 128 KB of LDS each).
struct PassGeom {
  int ns;
  int split;
  int tps;
  int64_t groups;
};

PassGeom pass_geometry(const Layout& L, int precision) {
  const int cand64[3] = {4, 2, 1}, cand32[3] = {4, 2, 1};
  const int* cand = precision == 1 ? cand32 : cand64;
  const int ncand = 3;
  const int64_t min_split = (L.ntiles + kMaxTilesPerBlock - 1) / kMaxTilesPerBlock;
  PassGeom G{1, 1, (int)L.ntiles, 0};
  for (int ci = 0; ci < ncand; ++ci) {
    const int ns = cand[ci];
    const int64_t groups = (L.p + (int64_t)kPassThreads * ns - 1) / ((int64_t)kPassThreads * ns);
    if (groups * 2 >= 256 || ns == 1 || (groups >= 64 && L.ntiles >= 8)) {
      int64_t split = std::max<int64_t>(1, 256 / groups);
      split = std::min<int64_t>(split, L.ntiles);
      split = std::max<int64_t>(split, min_split);
      const int tps = (int)((L.ntiles + split - 1) / split);
      split = (L.ntiles + tps - 1) / tps;
      G = PassGeom{ns, (int)split, tps, groups};
      break;
    }
  }
  return G;
}

size_t pass_lds_bytes(const PassGeom& G) { return 65536 + 40 * sizeof(double) + (size_t)G.tps * kTileSubjects * sizeof(double); }

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
  hipLaunchKernelGGL(k_stats, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<const uint2*>(tiled), L.p, L.p_pad,
                     L.ntiles, mask_bits, nT, u, v);
  return hipGetLastError();
}

size_t gradient_partial_bytes(const Layout& L) {
  size_t b = 0;
  for (int prec = 0; prec < 2; ++prec) {
    const PassGeom G = pass_geometry(L, prec);
    if (G.split > 1) b = std::max(b, (size_t)G.split * (size_t)L.p_pad * sizeof(double2));
  }
  return b;
}

template <int NS, bool F32>
static void launch_pass_one(dim3 grid, size_t lds, hipStream_t st, const uint2* tiled, const Layout& L, int tps, const double* r,
                            const double* mask, int64_t nT, const double* u, const double* v, FitState* fs, double* g,
                            double2* partial, const int32_t* gate) {
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass<NS, F32>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536 + 40 * (int)sizeof(double) + kMaxTilesPerBlock * kTileSubjects * (int)sizeof(double));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_pass<NS, F32>), grid, dim3(kPassThreads), lds, st, tiled, L.p, L.p_pad, (int32_t)L.ntiles, tps, L.n, r,
                     mask, nT, u, v, fs, g, partial, gate);
}

template <int NS>
static void launch_pass_ns(bool f32, dim3 grid, size_t lds, hipStream_t st, const uint2* tiled, const Layout& L, int tps,
                           const double* r, const double* mask, int64_t nT, const double* u, const double* v, FitState* fs,
                           double* g, double2* partial, const int32_t* gate) {
  if (!f32) {
    launch_pass_one<NS, false>(grid, lds, st, tiled, L, tps, r, mask, nT, u, v, fs, g, partial, gate);
    return;
  }
  launch_pass_one<NS, true>(grid, lds, st, tiled, L, tps, r, mask, nT, u, v, fs, g, partial, gate);
}

hipError_t launch_gradient(const uint8_t* tiled, const Layout& L, const double* r, const double* mask, int64_t nT,
                           const double* u, const double* v, FitState* fs, int precision, double* g, double* partial,
                           const int32_t* gate, hipStream_t st) {
  const PassGeom G = pass_geometry(L, precision);
  const dim3 grid((unsigned)G.groups, (unsigned)G.split);
  double2* part = (G.split > 1) ? reinterpret_cast<double2*>(partial) : nullptr;
  const bool f32 = precision == 1;
  const uint2* t4 = reinterpret_cast<const uint2*>(tiled);
  const size_t lds = pass_lds_bytes(G);
  if (G.ns == 4)
    launch_pass_ns<4>(f32, grid, lds, st, t4, L, G.tps, r, mask, nT, u, v, fs, g, part, gate);
  else if (G.ns == 2)
    launch_pass_ns<2>(f32, grid, lds, st, t4, L, G.tps, r, mask, nT, u, v, fs, g, part, gate);
  else
    launch_pass_ns<1>(f32, grid, lds, st, t4, L, G.tps, r, mask, nT, u, v, fs, g, part, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (part) {
    hipLaunchKernelGGL(k_pass_finalize, dim3((unsigned)((L.p + 255) / 256)), dim3(256), 0, st, part, G.split, L.p, L.p_pad, u,
                       v, fs, g, gate);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_topk(const TopkJob& J, int64_t p, int32_t rows, hipStream_t st) {
  // two-pass selection when every row's candidates fit pass 2
  const int64_t chunk2 = 1024 * (int64_t)kLocalEPT;
  const int64_t nb = (p + chunk2 - 1) / chunk2;
  if (J.kmax <= kLocalMaxK && nb * J.kmax <= 1024 * (int64_t)kFinalEPT && nb * J.kmax <= J.cap) {
    hipLaunchKernelGGL(k_topk_local<kLocalEPT>, dim3((unsigned)nb, (unsigned)rows), dim3(1024), 0, st, J, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_final, dim3((unsigned)rows), dim3(1024), 0, st, J, p, (int32_t)nb);
    return hipGetLastError();
  }
  // histogram path (large k or very long rows): about 2048 blocks over all rows, 4096 to 65536
  // entries per block
  int64_t chunk = 4096;
  while (chunk < 65536 && (p + chunk - 1) / chunk * rows > 2048) chunk <<= 1;
  const dim3 grid((unsigned)((p + chunk - 1) / chunk), (unsigned)rows);
  hipLaunchKernelGGL(k_topk_hist, grid, dim3(1024), 0, st, J, p, chunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_topk_collect, grid, dim3(1024), 0, st, J, p, chunk);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* x, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

hipError_t launch_topk_clear_errors(uint32_t* small, int32_t rows, hipStream_t st) {
  hipLaunchKernelGGL(k_topk_clear_errors, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, small, rows);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double val, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, val);
  return hipGetLastError();
}

hipError_t launch_scatter(const int64_t* idx, const double* vals, int32_t k, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, idx, vals, k, out);
  return hipGetLastError();
}

}  // namespace iht
