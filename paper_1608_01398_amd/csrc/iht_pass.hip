// iht_pass.hip -- the gradient pass of the IHT hot path (gfx950).
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
#include <mutex>
#include <set>
#include <type_traits>

#include "iht_internal.h"

namespace iht {
namespace {

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
// The gradient pass.
//
// The block walks its subject range two tiles (64 subjects) at a time. For each pair it builds in
// LDS, for every 4-subject group g (8 per tile) and every packed byte value v, the sums
// T = sum dose * r and M = sum [missing] * r over the group's subjects (the "Four Russians" table);
// each packed byte then costs one table read instead of 4 decodes and multiply-adds. Table of one
// pair: 256 rows of 256 B, row v = [tile A: 8 groups][tile B: 8 groups] x 16 B (FP64 (T, M)); FP32
// rows hold two copies of [A: 8 x 8 B][B: 8 x 8 B]. Two buffers: pair q builds into buffer q % 2;
// buffer 0 is LDS [0, 64 KB), buffer 1 is [64 KB, 128 KB). The lookup address is one v_perm of a
// per-lane offset register and the packed data: byte 0 = slot offset, byte 1 = packed byte value,
// byte 2 = buffer (buffer 1's offset registers carry a 0x01 byte for it), byte 3 = 0.
//
// Conflict-free reads: the LDS serves 16 lanes per cycle for 16-byte reads (32 for 8-byte reads).
// Lane L reads, at step b of a pair, the byte at position b % 8 of its SNP's segment of tile
// (b / 8) ^ ((L / 8) % 2); by the per-SNP rotation of the layout that byte is group (b + L) % 8 of
// that tile. So among 16 lanes served together, lanes 0-7 and 8-15 read different tiles (different
// halves of the row) and different groups within them: 16 distinct bank quads for any data.
constexpr uint32_t kPassBuf1 = 65536;  // LDS offset of table buffer 1
constexpr size_t kPassLdsBytes = 2 * 65536;

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) v2d_t lds_double2;
typedef __attribute__((address_space(3))) v2f_t lds_float2;

template <bool F32>
struct PassTab;
template <>
struct PassTab<false> {
  // slot offset inside a row: tile half * 128 + group * 16
  __device__ static uint32_t slot(int lane, int tile, int grp) { return (uint32_t)(tile * 128 + grp * 16); }
};
template <>
struct PassTab<true> {
  // copy (lanes 16-31 of every 32) * 128 + tile half * 64 + group * 8
  __device__ static uint32_t slot(int lane, int tile, int grp) {
    return (uint32_t)(((lane >> 4) & 1) * 128 + tile * 64 + grp * 8);
  }
};

__device__ __forceinline__ double dose_of(int c) { return c == 3 ? 2.0 : (c == 2 ? 1.0 : 0.0); }
__device__ __forceinline__ double miss_of(int c) { return c == 1 ? 1.0 : 0.0; }

// Builder thread (1024 or 512 per block): group G = tid % 16 of the pair (tile G / 8, group G % 8)
// and byte values v = tid / 16 + STEP m, STEP = threads / 16 (m < 4096 / threads). Codes c0, c1 and
// the low bit of c2 come from tid / 16, the rest from m. Entries sum the group's 4 subjects in order:
// T = ((d0 r0 + d1 r1) + d2 r2) + d3 r3; the part fixed by the thread and the two values of the
// c2 term are formed once, so each entry costs one add for T and one for M, stored immediately.
template <bool F32, int THREADS>
__device__ __forceinline__ void build_pair(uint32_t buf, int G, int vb, const double (&r)[4]) {
  static_assert(THREADS == 512 || THREADS == 1024, "builder mapping");
  constexpr int EPT = 4096 / THREADS;
  constexpr int STEP = THREADS / 16;
  const int c0 = vb & 3, c1 = (vb >> 2) & 3;
  const double T2 = dose_of(c0) * r[0] + dose_of(c1) * r[1];
  const double M2 = miss_of(c0) * r[0] + miss_of(c1) * r[1];
  // the two c2 values reachable from this thread (bit 4 of v is vb bit 4; bit 5 varies with m when
  // STEP = 32, and comes from vb when STEP = 64)
  double T3[2], M3[2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb) {
    const int c2 = ((vb >> 4) & (STEP == 64 ? 3 : 1)) | (STEP == 64 ? 0 : hb << 1);
    T3[hb] = T2 + dose_of(c2) * r[2];
    M3[hb] = M2 + miss_of(c2) * r[2];
  }
  const uint32_t tile = (uint32_t)(G >> 3), grp = (uint32_t)(G & 7);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int v = vb + STEP * m;
    const int hb = STEP == 64 ? 0 : (m & 1);
    const int c3 = v >> 6;  // fixed per m: v = vb + STEP m with vb < STEP
    const double T = c3 >= 2 ? T3[hb] + dose_of(c3) * r[3] : T3[hb];
    const double M = c3 == 1 ? M3[hb] + r[3] : M3[hb];
    const uint32_t row = buf + ((uint32_t)v << 8);
    if constexpr (F32) {
      const v2f_t e = {(float)T, (float)M};
      const uint32_t off = row + tile * 64 + grp * 8;
      *reinterpret_cast<lds_float2*>((size_t)off) = e;
      *reinterpret_cast<lds_float2*>((size_t)(off + 128)) = e;
    } else {
      const v2d_t e = {T, M};
      *reinterpret_cast<lds_double2*>((size_t)(row + tile * 128 + grp * 16)) = e;
    }
#if IHT_PASS_SNP_BARRIER
    __builtin_amdgcn_sched_barrier(0);
#endif
  }
}

// A lookup unit: kUnitLookups lookups of one tile of one SNP. With 8, a unit is the whole tile
// (steps 8 half .. 8 half + 7 of the pair); with 4 it is the byte positions {c, c+4} for two
// consecutive c, so a tile takes two units.
constexpr int kUnitLookups = IHT_PASS_UNIT;
constexpr int kUnitsPerTile = 8 / kUnitLookups;

template <bool F32>
struct Unit {
  using acc_t = typename std::conditional<F32, float, double>::type;
  acc_t t[kUnitLookups], m[kUnitLookups];
};

// Unit `part` of tile `half`: byte positions c + 4h for c in [part * C, part * C + C), h in {0, 1},
// C = kUnitLookups / 2; value index (c - part * C) + C h.
template <bool F32, int BUF>
__device__ __forceinline__ void unit_lookup(const uint32_t (&offs0)[4], const uint32_t (&offs1)[6], uint2 d, int half,
                                            int part, Unit<F32>& U) {
  constexpr int C = kUnitLookups / 2;
#pragma unroll
  for (int cc = 0; cc < C; ++cc) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = part * C + cc;
      const int b = half * 8 + c + 4 * h;  // step; byte c of dword h of the segment
      const uint32_t dw = h ? d.y : d.x;
      // buffer 0: offs0[b / 4] byte b % 4 holds the slot offset; bytes 2-3 of the address are 0.
      // buffer 1: offs1[b / 3] byte b % 3 holds it and its byte 3 is 0x01 -> address byte 2.
      uint32_t addr;
      if constexpr (BUF == 0) {
        const uint32_t sel = (uint32_t)(4 + (b & 3)) | ((uint32_t)c << 8) | (0x0Cu << 16) | (0x0Cu << 24);
        addr = __builtin_amdgcn_perm(offs0[b >> 2], dw, sel);
      } else {
        const uint32_t sel = (uint32_t)(4 + (b % 3)) | ((uint32_t)c << 8) | (7u << 16) | (0x0Cu << 24);
        addr = __builtin_amdgcn_perm(offs1[b / 3], dw, sel);
      }
      if constexpr (F32) {
        const v2f_t e = *reinterpret_cast<const lds_float2*>((size_t)addr);
        U.t[cc + C * h] = e.x;
        U.m[cc + C * h] = e.y;
      } else {
        const v2d_t e = *reinterpret_cast<const lds_double2*>((size_t)addr);
        U.t[cc + C * h] = e.x;
        U.m[cc + C * h] = e.y;
      }
    }
  }
}

// Rotation-invariant tree over byte positions: QT[c] = v[c] + v[c+4], then (QT0 + QT2) + (QT1 + QT3).
// The same pairings of byte positions are the same pairings of groups for every rotation, so the
// tile sum depends only on the column's bytes. q[] collects the QT of a tile across its units.
template <bool F32>
__device__ __forceinline__ void unit_pairs(const Unit<F32>& U, int part, typename Unit<F32>::acc_t (&qt)[4],
                                           typename Unit<F32>::acc_t (&qm)[4]) {
  constexpr int C = kUnitLookups / 2;
#pragma unroll
  for (int cc = 0; cc < C; ++cc) {
    qt[part * C + cc] = U.t[cc] + U.t[cc + C];
    qm[part * C + cc] = U.m[cc] + U.m[cc + C];
  }
}

// All lookups of one pair for the lane's NS SNPs, software-pipelined over the units (kPassPipeDepth
// units of lookups in flight ahead of the one being summed). The two tile sums of a SNP are
// combined as acc += (A + B), which is commutative: identical columns give bitwise identical
// gradients whichever tile a lane reads first.
template <bool F32, int BUF, int NS>
__device__ __forceinline__ void pair_step(const uint32_t (&offs0)[4], const uint32_t (&offs1)[6], const uint2 (&first)[NS],
                                          const uint2 (&second)[NS], double (&accT)[NS], double (&accM)[NS]) {
  using acc_t = typename Unit<F32>::acc_t;
  constexpr int UPS = 2 * kUnitsPerTile;  // units per SNP
  constexpr int NU = NS * UPS;
  constexpr int D = kPassPipeDepth;
  Unit<F32> U[D + 1];
  acc_t qt[4], qm[4];      // pair sums of the tile in progress
  acc_t PT0 = 0, PM0 = 0;  // first tile's sums of the current SNP
  auto issue = [&](int u, Unit<F32>& dst) {
    const int snp = u / UPS, half = (u % UPS) / kUnitsPerTile, part = u % kUnitsPerTile;
    unit_lookup<F32, BUF>(offs0, offs1, half ? second[snp] : first[snp], half, part, dst);
  };
#pragma unroll
  for (int u = 0; u < D && u < NU; ++u) issue(u, U[u]);
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    if (u + D < NU) issue(u + D, U[(u + D) % (D + 1)]);
#if IHT_PASS_SNP_BARRIER
    __builtin_amdgcn_sched_barrier(0);
#endif
    const int snp = u / UPS, half = (u % UPS) / kUnitsPerTile, part = u % kUnitsPerTile;
    unit_pairs<F32>(U[u % (D + 1)], part, qt, qm);
    if (part == kUnitsPerTile - 1) {
      const acc_t PT = (qt[0] + qt[2]) + (qt[1] + qt[3]);
      const acc_t PM = (qm[0] + qm[2]) + (qm[1] + qm[3]);
      if (half) {
        accT[snp] += (double)PT0 + (double)PT;
        accM[snp] += (double)PM0 + (double)PM;
      } else {
        PT0 = PT;
        PM0 = PM;
      }
    }
#if IHT_PASS_SNP_BARRIER
    __builtin_amdgcn_sched_barrier(0);
#endif
  }
}

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

// Centred residual of the subject set: rc[i] = r_i - mean for i in T, 0 elsewhere (up to n_pad),
// mean = sum_T r / |T|, R = sum_T rc (~0) in fs. X_st^T 1_T = 0, so centring leaves the gradient
// unchanged and keeps the table entries small. One workgroup.
__global__ __launch_bounds__(1024) void k_center(const double* __restrict__ r, const double* __restrict__ mask, int64_t n,
                                                 int64_t n_pad, int64_t nT, double* __restrict__ rc, FitState* __restrict__ fs,
                                                 const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[40];
  double s1 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s1 += (mask[i] != 0.0) ? r[i] : 0.0;
  const double mean = block_sum(s1, red) / (double)nT;
  double s2 = 0.0;
  for (int64_t i = threadIdx.x; i < n_pad; i += blockDim.x) {
    const double x = (i < n && mask[i] != 0.0) ? r[i] - mean : 0.0;
    rc[i] = x;
    s2 += x;
  }
  const double R = block_sum(s2, red);
  if (threadIdx.x == 0) {
    fs->mean = mean;
    fs->Rsum = R;
  }
}

template <int NS, bool F32>
__global__ __launch_bounds__(kPassThreads, 1) void k_pass(const uint2* __restrict__ tiled, int64_t p, int64_t p_pad, int32_t ntiles,
                                                  int32_t tps, const double* __restrict__ rc,
                                                  const double* __restrict__ u, const double* __restrict__ v,
                                                  const FitState* __restrict__ fs, double* __restrict__ g,
                                                  double2* __restrict__ partial, int64_t pst, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  // The kernel has no static LDS, so the dynamic allocation starts at LDS address 0: the table
  // buffers are addressed by absolute LDS offsets.

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int t0 = blockIdx.y * tps;  // even: tps is even
  const int t1 = min(ntiles, t0 + tps);

  const int64_t jb = (int64_t)blockIdx.x * (kPassThreads * NS) + tid;
  const uint32_t voff = (uint32_t)(jb * 8);
  // packed bytes of pair 0 in flight first
  uint2 dA[2][NS], dB[2][NS];
  load_tile<NS>(dA[0], tiled, p_pad, voff, t0, t1);
  load_tile<NS>(dB[0], tiled, p_pad, voff, t0 + 1, t1);

  // lane constants: the rotation of its SNPs (j % 8 == tid % 8) and which tile it reads first
  const int rot = tid & 7;
  const int hh = (lane >> 3) & 1;
  // slot offset of step b: tile (b / 8) ^ hh, group (b % 8 + rot) % 8; packed 4 per register for
  // buffer 0, 3 per register plus the 0x01 buffer byte for buffer 1
  uint32_t offs0[4], offs1[6];
#pragma unroll
  for (int k = 0; k < 4; ++k) offs0[k] = 0u;
#pragma unroll
  for (int k = 0; k < 6; ++k) offs1[k] = 0x01000000u;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const uint32_t o = PassTab<F32>::slot(lane, (b >> 3) ^ hh, ((b & 7) + rot) & 7);
    offs0[b >> 2] |= o << (8 * (b & 3));
    offs1[b / 3] |= o << (8 * (b % 3));
  }
  const int G = tid & 15, vb = tid >> 4;

  // centred residuals of builder group G in pair q (zero past the range: all-zero tables)
  auto group_r = [&](int q, double (&rr)[4]) {
    const int t = t0 + 2 * q + (G >> 3);
    const bool live = t < t1;
    const double4 x = *reinterpret_cast<const double4*>(rc + (int64_t)(live ? t : t0) * kTileSubjects + 4 * (G & 7));
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
  double rr[4];
  group_r(0, rr);
  build_pair<F32, kPassThreads>(0u, G, vb, rr);
  group_r(1, rr);
  __syncthreads();

  // Pair q uses register slot q % 2 and table buffer q % 2, both compile-time in the unrolled body.
  // Each step loads pair q+1, builds the table of pair q+1, prefetches the residuals of pair q+2 and
  // consumes pair q. Pairs past the range (at most 1) have all-zero tables and add exact zeros.
  const int npairs = (t1 - t0 + 1) / 2;
  const int trips = (npairs + 1) / 2;
  for (int trip = 0; trip < trips; ++trip) {
#pragma unroll
    for (int uu = 0; uu < 2; ++uu) {
      const int q = trip * 2 + uu;
      const int tn = t0 + 2 * (q + 1);
      load_tile<NS>(dA[uu ^ 1], tiled, p_pad, voff, tn, t1);
      load_tile<NS>(dB[uu ^ 1], tiled, p_pad, voff, tn + 1, t1);
      build_pair<F32, kPassThreads>(uu ? 0u : kPassBuf1, G, vb, rr);
      group_r(q + 2, rr);
      uint2 first[NS], second[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        first[s] = hh ? dB[uu][s] : dA[uu][s];
        second[s] = hh ? dA[uu][s] : dB[uu][s];
      }
      if (uu == 0)
        pair_step<F32, 0, NS>(offs0, offs1, first, second, accT, accM);
      else
        pair_step<F32, 1, NS>(offs0, offs1, first, second, accT, accM);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
    }
  }

#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int64_t j = jb + s * kPassThreads;
    if (j < p) {
      if (partial) {
        partial[(int64_t)blockIdx.y * pst + j] = make_double2(accT[s], accM[s]);
      } else {
        g[j] = v[j] * (accT[s] - u[j] * (fs->Rsum - accM[s]));
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_pass_finalize(const double2* __restrict__ partial, int32_t split, int64_t p,
                                                       int64_t pst, const double* __restrict__ u,
                                                       const double* __restrict__ v, const FitState* __restrict__ fs,
                                                       double* __restrict__ g, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  double D = 0.0, M = 0.0;
  for (int s = 0; s < split; ++s) {
    const double2 e = partial[(int64_t)s * pst + j];
    D += e.x;
    M += e.y;
  }
  g[j] = v[j] * (D - u[j] * (fs->Rsum - M));
}

// ------------------------------------------------------------------------------------------------
// Pass geometry: NS SNPs per lane and `split` subject ranges per SNP block, chosen so one launch
// fills the 256 CUs about once (one 1024-thread workgroup per CU: 128 KB of LDS each).
struct PassGeom {
  int ns;
  int split;
  int tps;
  int64_t groups;
  int64_t stride() const { return groups * kPassThreads * ns; }  // SNPs covered: partial sums per split
};

PassGeom pass_geometry(const Layout& L, int precision) {
  (void)precision;
  const int cand[4] = {8, 4, 2, 1};
  const int ncand = 4;
  PassGeom G{1, 1, (int)((L.ntiles + 1) / 2 * 2), 0};
  G.groups = (L.p + kPassThreads - 1) / kPassThreads;
  for (int ci = 0; ci < ncand; ++ci) {
    const int ns = cand[ci];
    if (ns > kPassMaxNS) continue;
    const int64_t groups = (L.p + (int64_t)kPassThreads * ns - 1) / ((int64_t)kPassThreads * ns);
    if (groups * 2 >= 256 || ns == 1 || (groups >= 64 && L.ntiles >= 8)) {
      int64_t split = std::max<int64_t>(1, 256 / groups);
      split = std::min<int64_t>(split, (L.ntiles + 1) / 2);
      int tps = (int)((L.ntiles + split - 1) / split);
      tps += tps & 1;  // whole tile pairs per block
      split = (L.ntiles + tps - 1) / tps;
      G = PassGeom{ns, (int)split, tps, groups};
      break;
    }
  }
  return G;
}

// hipFuncSetAttribute once per (kernel, device), thread-safe.
std::mutex g_attr_mu;
std::set<std::pair<const void*, int>> g_attr_done;

hipError_t allow_pass_lds(const void* fn) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (g_attr_done.count({fn, dev})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPassLdsBytes);
  if (e == hipSuccess) g_attr_done.insert({fn, dev});
  return e;
}

template <int NS, bool F32>
hipError_t launch_pass_one(dim3 grid, hipStream_t st, const uint2* tiled, const Layout& L, int tps, const double* rc,
                           const double* u, const double* v, const FitState* fs, double* g, double2* partial, int64_t pst,
                           const int32_t* gate) {
  hipError_t e = allow_pass_lds(reinterpret_cast<const void*>(&k_pass<NS, F32>));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pass<NS, F32>), grid, dim3(kPassThreads), kPassLdsBytes, st, tiled, L.p, L.p_pad, (int32_t)L.ntiles,
                     tps, rc, u, v, fs, g, partial, pst, gate);
  return hipGetLastError();
}

template <int NS>
hipError_t launch_pass_ns(bool f32, dim3 grid, hipStream_t st, const uint2* tiled, const Layout& L, int tps, const double* rc,
                          const double* u, const double* v, const FitState* fs, double* g, double2* partial, int64_t pst,
                          const int32_t* gate) {
  return f32 ? launch_pass_one<NS, true>(grid, st, tiled, L, tps, rc, u, v, fs, g, partial, pst, gate)
             : launch_pass_one<NS, false>(grid, st, tiled, L, tps, rc, u, v, fs, g, partial, pst, gate);
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// Launchers

size_t gradient_work_bytes(const Layout& L) {
  size_t b = 0;
  for (int prec = 0; prec < 2; ++prec) {
    const PassGeom G = pass_geometry(L, prec);
    if (G.split > 1) b = std::max(b, (size_t)G.split * (size_t)G.stride() * sizeof(double2));
  }
  return (size_t)L.n_pad * sizeof(double) + b;
}

hipError_t launch_gradient(const uint8_t* tiled, const Layout& L, const double* r, const double* mask,
                           int64_t nT, const double* u, const double* v, FitState* fs, int precision, double* g,
                           double* work, const int32_t* gate, hipStream_t st, const double* rc_ready) {
  const PassGeom G = pass_geometry(L, precision);
  const double* rc = rc_ready ? rc_ready : work;
  double2* part = (G.split > 1) ? reinterpret_cast<double2*>(work + L.n_pad) : nullptr;
  hipError_t e;
  if (!rc_ready) {
    hipLaunchKernelGGL(k_center, dim3(1), dim3(1024), 0, st, r, mask, L.n, L.n_pad, nT, work, fs, gate);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)G.groups, (unsigned)G.split);
  const bool f32 = precision == 1;
  const uint2* t4 = reinterpret_cast<const uint2*>(tiled);
  const int64_t pst = G.stride();
  if (G.ns == 8)
    e = launch_pass_ns<8>(f32, grid, st, t4, L, G.tps, rc, u, v, fs, g, part, pst, gate);
  else if (G.ns == 4)
    e = launch_pass_ns<4>(f32, grid, st, t4, L, G.tps, rc, u, v, fs, g, part, pst, gate);
  else if (G.ns == 2)
    e = launch_pass_ns<2>(f32, grid, st, t4, L, G.tps, rc, u, v, fs, g, part, pst, gate);
  else
    e = launch_pass_ns<1>(f32, grid, st, t4, L, G.tps, rc, u, v, fs, g, part, pst, gate);
  if (e != hipSuccess) return e;
  if (part) {
    hipLaunchKernelGGL(k_pass_finalize, dim3((unsigned)((L.p + 255) / 256)), dim3(256), 0, st, part, G.split, L.p, pst, u,
                       v, fs, g, gate);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace iht
