// rwpt_kernels.hip -- HIP kernels (gfx950) of one explicit step of the
// particle mass-transfer method of arXiv:1811.05474:
//   walk + cell key  -> counting sort into a uniform cell grid (cell-count scan,
//   scatter, canonical in-cell order) -> row sums r_i -> weights + exchange +
//   reaction + audit partials -> per-realisation audit.
//
// Layout: particle-major, positions pos[d * p + k] (packed: one particle is
// one vector load) and masses mass[SP * p + s]
// (SP = 2, 4, 8 species slots, the unused ones zero), kept in cell-sorted order; id[p] maps a sorted slot back to the caller's
// particle index.  Every reduction runs in a fixed order, so results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include <type_traits>

#include "rwpt_kernels.h"
#include "rwpt_layout.h"
#include "rwpt_pairstep.h"

namespace rwpt {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

// Wave-uniform block index -> logical block so that each of the 8 XCDs (which
// receive workgroups round-robin) works on one contiguous range of tiles and
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, q = b >> 3;
  return x * per + (x < rem ? x : rem) + q;
}

// Tile index of the calling wave, as tile_lane_setup derives it (SPLIT > 1:
// one tile per block).
template <int SPLIT = 1>
__device__ __forceinline__ int64_t wave_tile() {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  return SPLIT > 1 ? blk : blk * (kBlock / 64) + wave;
}

// Maximum of v over the 64 lanes of the wave (all active); wave-uniform.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m; m >>= 1) {
    const uint32_t t = __shfl_xor(v, m);
    v = t > v ? t : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

// Between a wave's LDS stores and its loads of what other lanes of the same
// wave stored: the LDS executes one wave's operations in order, so only the
// compiler has to be kept from moving the loads above the stores.
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds of the
// multiply/xor S-box with the key bumped by the golden-ratio and sqrt(3)-1
// Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t a0 = c[0], a2 = c[2];
    const uint32_t hi0 = __umulhi(0xD2511F53u, a0), lo0 = 0xD2511F53u * a0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, a2), lo1 = 0xCD9E8D57u * a2;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
  }
}

// Box-Muller pair from the uniforms (u, v): sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v).
// Binary32 uses the hardware log2 / sqrt / sin / cos (sin and cos take the
// angle in revolutions), accurate to ~1e-6 relative -- far below what a
// random displacement needs; binary64 uses the library functions.
__device__ __forceinline__ void box_muller(float u, float v, float* z0, float* z1) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));  // -2 ln 2 log2 u
  *z0 = r * __builtin_amdgcn_cosf(v);
  *z1 = r * __builtin_amdgcn_sinf(v);
}
__device__ __forceinline__ void box_muller(double u, double v, double* z0, double* z1) {
  const double r = sqrt(-2.0 * log(u));
  double sn, cs;
  sincospi(2.0 * v, &sn, &cs);
  *z0 = r * cs;
  *z1 = r * sn;
}

// Three standard normals for (particle id, step) under the 64-bit seed:
// counter (id, step lo, step hi, 0); uniforms u = w * 2^-32 + 2^-33;
// Box-Muller on (u0, u1) and (u2, u3).
template <typename T, int DIM>
__device__ __forceinline__ void walk_normals(uint32_t pid, uint64_t seed, uint64_t step, T z[3]) {
  uint32_t c[4] = {pid, (uint32_t)step, (uint32_t)(step >> 32), 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const T s32 = (T)2.3283064365386962890625e-10;   // 2^-32
  const T half = (T)1.16415321826934814453125e-10; // 2^-33
  const T u0 = (T)c[0] * s32 + half;
  const T u1 = (T)c[1] * s32 + half;
  box_muller(u0, u1, &z[0], &z[1]);
  z[2] = (T)0;
  if constexpr (DIM > 2) {
    const T u2 = (T)c[2] * s32 + half;
    const T u3 = (T)c[3] * s32 + half;
    T unused;
    box_muller(u2, u3, &z[2], &unused);
  }
}

// Mirror at zero-flux walls until inside the closed box.
template <typename T>
__device__ __forceinline__ T reflect(T x, T lo, T hi) {
  for (int it = 0; it < 64 && (x < lo || x > hi); ++it) x = (x < lo) ? (T)2 * lo - x : (T)2 * hi - x;
  x = x < lo ? lo : x;
  x = x > hi ? hi : x;
  return x;
}

// Squared separation used by the cutoff predicate: dx*dx, then
// fma(dy, dy, .) and fma(dz, dz, .) in the path's precision, dx = x_j - x_i,
// dimension order; every step is correctly rounded and nothing else is
// contracted, so the neighbour sets are reproducible bit for bit.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int DIM>
__device__ __forceinline__ T sep2v(const T xi[DIM], const T xj[DIM]) {
#pragma clang fp contract(off)
  const T d0 = xj[0] - xi[0];
  T s = d0 * d0;
  if constexpr (DIM > 1) {
    const T d1 = xj[1] - xi[1];
    s = fma_t(d1, d1, s);
  }
  if constexpr (DIM > 2) {
    const T d2 = xj[2] - xi[2];
    s = fma_t(d2, d2, s);
  }
  return s;
}

template <typename T, int DIM>
__device__ __forceinline__ T sep2(const T xi[DIM], const T* __restrict__ pos, int64_t j) {
  T xj[DIM];
  load_pos<T, DIM>(pos, j, xj);
  return sep2v<T, DIM>(xi, xj);
}

// Candidates per lane handled per unrolled block (their loads are issued
// together; with one lane per particle they are consecutive and uniform, so
// they merge into wide scalar loads).
constexpr int kUnroll = 4;
// binary32 row partials are added into the binary64 accumulators at least
// every kFlushBlocks * kUnroll candidates per lane
constexpr uint32_t kFlushBlocks = 64;

template <typename T>
__device__ __forceinline__ T rc2_of(const RealParams& P);
template <>
__device__ __forceinline__ float rc2_of<float>(const RealParams& P) { return P.rc2_f; }
template <>
__device__ __forceinline__ double rc2_of<double>(const RealParams& P) { return P.rc2_d; }
template <typename T>
__device__ __forceinline__ T escale_of(const RealParams& P);
template <>
__device__ __forceinline__ float escale_of<float>(const RealParams& P) { return P.escale_f; }
template <>
__device__ __forceinline__ double escale_of<double>(const RealParams& P) { return P.escale_d; }

// ---------------------------------------------------------------------------
// Walk + key
// ---------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_walk_key(
    const T* __restrict__ pos_in, T* __restrict__ pos_out,
    const uint32_t* __restrict__ id, int32_t n, const RealParams* __restrict__ rp,
    const int64_t* __restrict__ real_start, const int32_t* __restrict__ blk_real, int32_t n_real,
    const uint64_t* __restrict__ step_ctr, uint64_t seed, int32_t do_walk,
    uint32_t* __restrict__ cell_count, uint32_t* __restrict__ key_out, uint32_t* __restrict__ slot_out) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  // last realisation whose first particle is <= p, from that of the block's
  // first particle (one block rarely spans more than two realisations)
  int lo = blk_real[blockIdx.x];
  while (lo + 1 < n_real && real_start[lo + 1] <= p) ++lo;
  T x[DIM];
  load_pos<T, DIM>(pos_in, p, x);
  auto walk_and_key = [&](const RealParams& P) -> uint32_t {
    if (do_walk && P.moves) {
      // drift v dt, isotropic amplitude, extra amplitude along v (Eq. 1)
      T z[3];
      walk_normals<T, DIM>(id[p], seed, *step_ctr, z);
      const T amp = (T)P.amp, ampx = (T)P.amp_x;
      T uz = (T)0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) uz += (T)P.udir[k] * z[k];
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const T move = (T)P.drift[k] + amp * z[k] + ampx * uz * (T)P.udir[k];
        x[k] = reflect<T>(x[k] + move, (T)P.lo[k], (T)P.hi[k]);
      }
    }
    int64_t c = 0;
#pragma unroll
    for (int k = DIM - 1; k >= 0; --k) {
      const double u = ((double)x[k] - P.lo[k]) * P.inv_h[k];
      int ck = (int)floor(u);
      ck = ck < 0 ? 0 : ck;
      ck = ck > P.nc[k] - 1 ? P.nc[k] - 1 : ck;
      c = c * P.nc[k] + ck;
    }
    return (uint32_t)(P.cell_off + c);
  };
  // realisations are contiguous, so a wave almost always lies in one: then
  // its parameters are read once through the scalar cache
  const int lo_u = __builtin_amdgcn_readfirstlane(lo);
  const uint32_t key = __ballot(lo != lo_u) == 0 ? walk_and_key(rp[lo_u]) : walk_and_key(rp[lo]);
  store_pos<T, DIM>(pos_out, p, x);
  key_out[p] = key;
  // The input is in cell order from the previous step, so equal new keys
  // mostly sit in runs of consecutive lanes: one atomic per run, the run's
  // lanes take consecutive slots.  (Active lanes are a prefix of the wave.)
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1);
  const unsigned long long starts = __ballot(lane == 0 || prev != key);
  const unsigned long long active = __ballot(1);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
  const int rs = 63 - __clzll(starts & upto);
  const unsigned long long above = starts & ~upto;
  const int re = above ? __ffsll(above) - 1 : 64 - __clzll(active);
  uint32_t base = 0;
  if (lane == rs) base = atomicAdd(&cell_count[key], (uint32_t)(re - rs));
  base = __shfl(base, rs);
  slot_out[p] = base + (uint32_t)(lane - rs);
}

// ---------------------------------------------------------------------------
// Exclusive scan of the cell counts
// ---------------------------------------------------------------------------

// Inclusive scan across the 256 threads of a block; returns the inclusive
// value and the block total.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off);
    if (lane >= off) v += t;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += sh[w];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return v + base;
}

// Coalesced block sums: thread t adds elements t, t + 256, ... of the chunk.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ cnt, int64_t n,
                                                        uint32_t* __restrict__ partials) {
  __shared__ uint32_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + (int64_t)i * kBlock;
    if (k < n) s += cnt[k];
  }
  uint32_t total;
  block_inclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Single block: exclusive scan of the block partials in place; the grand
// total becomes start[n] (the end of the last cell).
__global__ __launch_bounds__(kBlock) void k_scan_top(uint32_t* __restrict__ partials, int32_t nb,
                                                     uint32_t* __restrict__ start, int64_t n) {
  __shared__ uint32_t sh[4];
  const int per = (nb + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += partials[b0 + i];
  uint32_t total;
  const uint32_t incl = block_inclusive_scan(s, sh, &total);
  uint32_t run = incl - s;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const uint32_t v = partials[b0 + i];
      partials[b0 + i] = run;
      run += v;
    }
  if (threadIdx.x == 0) start[n] = total;
}

// LDS index of chunk element k with one pad word per 16, so that thread t
// reading its 16 consecutive elements hits distinct banks.
__device__ __forceinline__ int scan_pad(int k) { return k + (k >> 4); }

// Final pass: coalesced striped loads into LDS, a sequential scan of 16
// consecutive elements per thread, a block scan of the thread sums, then
// coalesced striped stores of the cell starts; the counts are re-zeroed for
// the next step.  DIRECT: partials holds the block sums themselves and every
// block adds up those of the blocks before it (no top-level scan launch; the
// last block writes the grand total start[n]); otherwise partials holds their
// exclusive scan.
template <bool DIRECT>
__global__ __launch_bounds__(kBlock) void k_scan_final(uint32_t* __restrict__ cnt, int64_t n,
                                                       const uint32_t* __restrict__ partials,
                                                       uint32_t* __restrict__ start) {
  __shared__ uint32_t sh[4];
  __shared__ uint32_t buf[kScanChunk + kScanChunk / 16];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t prefix = 0;
  if constexpr (DIRECT) {
    uint32_t s = 0;
    for (int c = t; c < (int)blockIdx.x; c += kBlock) s += partials[c];
    block_inclusive_scan(s, sh, &prefix);
  } else {
    prefix = partials[blockIdx.x];
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int k = t + i * kBlock;
    buf[scan_pad(k)] = (base + k < n) ? cnt[base + k] : 0u;
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = buf[scan_pad(t * kScanItems + i)];
    sum += v[i];
  }
  uint32_t total;
  const uint32_t incl = block_inclusive_scan(sum, sh, &total);
  if constexpr (DIRECT) {
    if (t == 0 && blockIdx.x == gridDim.x - 1) start[n] = prefix + total;
  }
  uint32_t run = prefix + incl - sum;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    buf[scan_pad(t * kScanItems + i)] = run;
    run += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int k = t + i * kBlock;
    if (base + k < n) {
      start[base + k] = buf[scan_pad(k)];
      cnt[base + k] = 0u;  // ready for the next step's counting
    }
  }
}

// ---------------------------------------------------------------------------
// Scatter and canonical in-cell order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_scatter(int32_t n, const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ slot,
                                                    const uint32_t* __restrict__ cell_start,
                                                    const uint32_t* __restrict__ id,
                                                    uint32_t* __restrict__ tmp_src,
                                                    uint32_t* __restrict__ tmp_id,
                                                    uint32_t* __restrict__ tmp_key) {
  // XCD-contiguous ranges: neighbouring particles' gathers and partial-line
  // writes meet in one L2
  const int p = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (p >= n) return;
  const uint32_t k = key[p];
  const uint32_t dst = cell_start[k] + slot[p];
  tmp_src[dst] = (uint32_t)p;
  tmp_id[dst] = id[p];
  tmp_key[dst] = k;
}

// The canonical gather takes kCanonItems particles per thread (block b covers
// kCanonItems * kBlock consecutive sorted slots, item u at threadIdx.x +
// u kBlock), with every item's loads issued before any of them is used, so
// that the items' chains of dependent loads (slot -> cell start -> cell
// members) overlap.  (Two items per thread in the scatter made it slower.)
constexpr int kCanonItems = 2;

// The atomic slot of the scatter depends on arrival order; ranking by the
// (unique) particle id inside each cell makes the sorted order a function of
// the positions alone: (cell, id).
// MOVE: gather the masses into the new order; otherwise record each sorted
// particle's previous slot (src_out) and leave the masses where they are.
template <typename T, int DIM, int SMAX, bool MOVE>
__global__ __launch_bounds__(kBlock) void k_canon(
    int32_t n, const uint32_t* __restrict__ tmp_src, const uint32_t* __restrict__ tmp_id,
    const uint32_t* __restrict__ tmp_key, const uint32_t* __restrict__ cell_start,
    const T* __restrict__ pos_in, T* __restrict__ pos_out, const T* __restrict__ mass_in,
    T* __restrict__ mass_out, uint32_t* __restrict__ id_out, uint32_t* __restrict__ skey,
    uint32_t* __restrict__ src_out) {
  const int64_t e0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kCanonItems * kBlock) + threadIdx.x;
  uint32_t k[kCanonItems], src[kCanonItems], my[kCanonItems], cs[kCanonItems], ce[kCanonItems];
#pragma unroll
  for (int u = 0; u < kCanonItems; ++u) {
    const int64_t e = e0 + u * kBlock;
    const int64_t q = e < n ? e : n - 1;  // a lane past the end repeats the last slot, stores nothing
    k[u] = tmp_key[q];
    src[u] = tmp_src[q];
    my[u] = tmp_id[q];
  }
  // issue the gathers first; the in-cell ranking below overlaps them
  T x[kCanonItems][DIM], m[kCanonItems][SMAX];
#pragma unroll
  for (int u = 0; u < kCanonItems; ++u) {
    load_pos<T, DIM>(pos_in, src[u], x[u]);
    if constexpr (MOVE) load_mass<T, SMAX>(mass_in, src[u], m[u]);  // unused species slots are zero and stay zero
    cs[u] = cell_start[k[u]];
    ce[u] = cell_start[k[u] + 1];
  }
#pragma unroll
  for (int u = 0; u < kCanonItems; ++u) {
    uint32_t rank = 0;
    for (uint32_t f = cs[u]; f < ce[u]; ++f) rank += (tmp_id[f] < my[u]) ? 1u : 0u;
    const int64_t e = e0 + u * kBlock;
    if (e < n) {
      const uint32_t dst = cs[u] + rank;
      store_pos<T, DIM>(pos_out, dst, x[u]);
      if constexpr (MOVE) store_mass<T, SMAX>(mass_out, dst, m[u]);
      else src_out[dst] = src[u];
      id_out[dst] = my[u];
      skey[dst] = k[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Pair kernels
//
// One wave handles a tile of G = 64 / L consecutive sorted particles; lane
// = gl * G + gi pairs particle gi of the tile with every L-th candidate
// (offset gl).  The tile is split into segments of one cell row each; for a
// segment the candidates are, on every neighbour row of the stencil, the
// contiguous sorted range of cells [cx_first - rx, cx_last + rx].  Every
// candidate is still decided by the exact cutoff predicate.
// ---------------------------------------------------------------------------

struct TileLane {
  int gi, gl, n_in, row, cx;
  bool valid;
  int32_t i;
};

template <int LOG2L, typename RowFn>
__device__ __forceinline__ void for_tile_rows(const RealParams& P, const StencilRow* __restrict__ st,
                                              const uint32_t* __restrict__ cell_start,
                                              const TileLane& tl, RowFn&& fn) {
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  int seg = 0;
  while (seg < tl.n_in) {
    const int seg_row = __builtin_amdgcn_readlane(tl.row, seg);
    const unsigned long long m =
        __ballot(tl.gl == 0 && tl.gi > seg && (tl.gi >= tl.n_in || tl.row != seg_row));
    int seg_end = m ? (__ffsll((unsigned long long)m) - 1) : tl.n_in;
    seg_end = seg_end > tl.n_in ? tl.n_in : seg_end;
    const int cxa = __builtin_amdgcn_readlane(tl.cx, seg);
    const int cxb = __builtin_amdgcn_readlane(tl.cx, seg_end - 1);
    const bool act = tl.valid && tl.gi >= seg && tl.gi < seg_end;
    const int cy = seg_row % nc1, cz = seg_row / nc1;
    for (int r = 0; r < P.n_stencil; ++r) {
      const StencilRow sr = st[P.stencil_off + r];
      const int ny = cy + sr.dy, nz = cz + sr.dz;
      if (ny < 0 || ny >= nc1 || nz < 0 || nz >= nc2) continue;
      const int xa = cxa - sr.rx < 0 ? 0 : cxa - sr.rx;
      const int xb = cxb + sr.rx > nc0 - 1 ? nc0 - 1 : cxb + sr.rx;
      const int64_t cb = P.cell_off + ((int64_t)nz * nc1 + ny) * nc0;
      const uint32_t jb = cell_start[cb + xa];
      const uint32_t je = cell_start[cb + xb + 1];
      fn(jb, je, act);
    }
    seg = seg_end;
  }
}

// Load the tile header and this lane's particle.
// SPLIT > 1: the SPLIT = kBlock / 64 waves of a block share one tile (each
// takes every SPLIT-th chunk of its candidates); otherwise one tile per wave.
template <int LOG2L, int SPLIT = 1>
__device__ __forceinline__ bool tile_lane_setup(const Tile* __restrict__ tiles, int32_t ntiles,
                                                TileLane& tl, Tile& tile) {
  static_assert(SPLIT == 1 || SPLIT == kBlock / 64, "a split tile takes the waves of one block");
  constexpr int G = 64 >> LOG2L;
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave; say so, so that everything
  // derived from the tile is kept in scalar registers and loaded through the
  // scalar cache
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int t = SPLIT > 1 ? blk : blk * (kBlock / 64) + wave;
  if (t >= ntiles) return false;
  tile = tiles[t];
  tl.gi = lane & (G - 1);
  tl.gl = lane >> (6 - LOG2L);
  tl.n_in = tile.end - tile.begin;
  tl.i = tile.begin + tl.gi;
  tl.valid = tl.gi < tl.n_in;
  return true;
}

template <typename T, int DIM>
__device__ __forceinline__ void lane_cell(const RealParams& P, const uint32_t* __restrict__ skey,
                                          int32_t ii, TileLane& tl) {
  const uint32_t lk = skey[ii] - (uint32_t)P.cell_off;
  tl.cx = (int)(lk % (uint32_t)P.nc[0]);
  tl.row = (int)(lk / (uint32_t)P.nc[0]);
}

// Exchange of a double with lane ^ M: a DPP quad permutation for M = 1, 2
// (no LDS traffic), a cross-lane permute otherwise.
template <int M>
__device__ __forceinline__ double xor_shfl(double v) {
  if constexpr (M == 1 || M == 2) {
    constexpr int ctrl = M == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, ctrl, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), ctrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
  } else {
    return __shfl_xor(v, M);
  }
}

// Sum of NV values over each aligned group of G lanes by recursive halving (a
// reduce-scatter): at step M every lane keeps one half of its values, adds the
// partner's (lane ^ M) copy of that half, and hands over the other half, so
// the number of values exchanged halves at every step; once one value is
// left, the remaining steps add it up plainly.  On return v[0 .. NK) holds the
// group totals of values idx .. idx + NK - 1, and lanes that differ only in
// the bits above the first NB (the halving steps) hold the same totals.  An
// upper half shorter than the lower one is padded with zeros; `real` counts
// the lane's values that are not padding (only those may be written out).
constexpr int halved_count(int n, int g) {
  for (int m = 1; m < g && n > 1; m <<= 1) n = (n + 1) / 2;
  return n;
}
constexpr int halving_bits(int n, int g) {
  int b = 0;
  for (int m = 1; m < g && n > 1; m <<= 1) {
    n = (n + 1) / 2;
    ++b;
  }
  return b;
}

template <int M, int G, int N, int NV>
__device__ __forceinline__ void halve_sum(double (&v)[NV], int& idx, int& real, int lane) {
  if constexpr (M < G) {
    if constexpr (N > 1) {
      constexpr int H = (N + 1) / 2;
      const bool up = (lane & M) != 0;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        double hi = 0.0;
        if (k + H < N) hi = v[k + H];
        const double keep = up ? hi : v[k];
        const double send = up ? v[k] : hi;
        v[k] = keep + xor_shfl<M>(send);
      }
      idx += up ? H : 0;
      real = up ? (real > H ? real - H : 0) : (real < H ? real : H);
      halve_sum<M * 2, G, H, NV>(v, idx, real, lane);
    } else {
      v[0] += xor_shfl<M>(v[0]);
      halve_sum<M * 2, G, 1, NV>(v, idx, real, lane);
    }
  }
}

// After the lane reductions: new masses (Eq. 6), reaction, and the tile's
// audit partials.  `writer` lanes (one per particle) hold acc / racc; lanes
// 0..G-1 are the writers' first copies, so the audit is reduced over them.
template <typename T, int SMAX, int G>
__device__ __forceinline__ void exchange_epilogue(const RealParams& P, bool sym, const double acc[SMAX],
                                                  double racc, const T Mi[SMAX], bool writer, int32_t i,
                                                  T* __restrict__ mout, int S, int react_a,
                                                  int react_b, double* __restrict__ audit_part, int64_t t) {
  double tot[SMAX + 1];
#pragma unroll
  for (int s = 0; s <= SMAX; ++s) tot[s] = 0.0;
  if (writer) {
    double Mn[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      double dm = 0.0;
      if (P.active) dm = sym ? 0.25 * acc[s] : 0.5 * acc[s] / racc;
      Mn[s] = (double)Mi[s] + dm;
    }
    // the reacting pair by its slot indices (uniform, < S <= SMAX: indexed
    // register moves, not a select over every slot)
    if (react_a >= 0) {
      const double A = Mn[react_a], B = Mn[react_b];
      double m = A < B ? A : B;
      m = m > 0.0 ? m : 0.0;
      Mn[react_a] = A - m;
      Mn[react_b] = B - m;
    }
    T out[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      out[s] = s < S ? (T)Mn[s] : (T)0;  // unused species slots stay zero
      tot[s] = (double)out[s];
    }
    store_mass<T, SMAX>(mout, i, out);
    tot[SMAX] = react_a >= 0 ? tot[react_a] - tot[react_b] : 0.0;
  }
  // totals over lanes 0..G-1 (the other lanes hold zeros and are reduced
  // among themselves); value SMAX is sum(A - B)
  constexpr int NV = SMAX + 1, NK = halved_count(NV, G), NB = halving_bits(NV, G);
  const int lane = threadIdx.x & 63;
  int idx = 0, real = NV;
  halve_sum<1, G, NV, NV>(tot, idx, real, lane);
  if (lane < (1 << NB)) {
    double* part = audit_part + t * (S + 1);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int vi = idx + k;
      if (k < real) {
        if (vi < S) part[vi] = tot[k];
        else if (vi == SMAX) part[S] = tot[k];
      }
    }
  }
}

// Row sums r_i = sum_{j in N(i)} w_ij (self included) and q_i = 1 / r_i:
// the normalisation of the co-location weights.
template <typename T, int DIM, int LOG2L>
__global__ __launch_bounds__(kBlock) void k_rowsum(
    const T* __restrict__ pos, const uint32_t* __restrict__ skey,
    const uint32_t* __restrict__ cell_start, const Tile* __restrict__ tiles, const int32_t ntiles,
    const RealParams* __restrict__ rp, const StencilRow* __restrict__ st, double* __restrict__ r_out,
    T* __restrict__ q_out) {
  constexpr int L = 1 << LOG2L;
  constexpr int G = 64 >> LOG2L;
  WeightFn<T> wfn;  // before any return: the binary64 form has a block barrier
  wfn.setup();
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<LOG2L>(tiles, ntiles, tl, tile)) return;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  lane_cell<T, DIM>(P, skey, ii, tl);
  const T rc2 = rc2_of<T>(P), esc = escale_of<T>(P);
  double acc = 0.0;
  if (P.active) {
    for_tile_rows<LOG2L>(P, st, cell_start, tl, [&](uint32_t jb, uint32_t je, bool act) {
      T accr = (T)0;
      const uint32_t len = je - jb, nblk = len / (L * kUnroll);
      uint32_t j = jb + tl.gl;
      for (uint32_t b = 0; b < nblk;) {
        // at most kFlushBlocks blocks per binary32 partial, then into binary64
        const uint32_t bend = nblk - b > kFlushBlocks ? b + kFlushBlocks : nblk;
        for (; b < bend; ++b, j += L * kUnroll) {
          T xj[kUnroll][DIM];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
            load_pos<T, DIM>(pos, j + u * L, xj[u]);
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const T s2 = sep2v<T, DIM>(xi, xj[u]);
            const T w = wfn(s2, esc);
            accr += (act && s2 <= rc2) ? w : (T)0;
          }
        }
        acc += (double)accr;
        accr = (T)0;
      }
      for (; j < je; j += L) {
        const T s2 = sep2<T, DIM>(xi, pos, j);
        const T w = wfn(s2, esc);
        accr += (act && s2 <= rc2) ? w : (T)0;
      }
      acc += (double)accr;
    });
  } else {
    acc = 1.0;  // only the self weight
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
  if (tl.gl == 0 && tl.valid) {
    if (!P.active) acc = 1.0;
    if (r_out) r_out[tl.i] = acc;
    q_out[tl.i] = (T)(1.0 / acc);
  }
}

// Weights + exchange (Eq. 4) + explicit update (Eq. 6) + reaction + audit
// partials.  Symmetric normalisation: dM_i = 1/4 sum_j w_ij (q_i + q_j)(M_j - M_i);
// row normalisation: dM_i = 1/2 (sum_j w_ij (M_j - M_i)) / r_i.
template <typename T, int DIM, int SMAX, int LOG2L>
__global__ __launch_bounds__(kBlock) void k_exchange(
    const T* __restrict__ pos, const T* __restrict__ min_, T* __restrict__ mout,
    const T* __restrict__ q, const uint32_t* __restrict__ skey, const uint32_t* __restrict__ cell_start,
    const Tile* __restrict__ tiles, const int32_t ntiles, const RealParams* __restrict__ rp,
    const StencilRow* __restrict__ st, const int32_t S, const int32_t react_a, const int32_t react_b,
    const int32_t norm, double* __restrict__ audit_part) {
  constexpr int L = 1 << LOG2L;
  constexpr int G = 64 >> LOG2L;
  WeightFn<T> wfn;  // before any return: the binary64 form has a block barrier
  wfn.setup();
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<LOG2L>(tiles, ntiles, tl, tile)) return;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  T Mi[SMAX];
  load_mass<T, SMAX>(min_, ii, Mi);
  lane_cell<T, DIM>(P, skey, ii, tl);
  const T rc2 = rc2_of<T>(P), esc = escale_of<T>(P);
  double acc[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) acc[s] = 0.0;
  double racc = 0.0;
  const bool sym = (norm == 0);
  if (P.active) {
    if (sym) {
      const T qi = q[ii];
      for_tile_rows<LOG2L>(P, st, cell_start, tl, [&](uint32_t jb, uint32_t je, bool act) {
        T accr[SMAX];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) accr[s] = (T)0;
        const uint32_t len = je - jb, nblk = len / (L * kUnroll);
        uint32_t j = jb + tl.gl;
        // species slots S..SMAX-1 exist and hold zeros, so no guard is needed
        auto eval = [&](const T xj[DIM], T qj, const T mj[SMAX]) {
          const T s2 = sep2v<T, DIM>(xi, xj);
          T w = wfn(s2, esc);
          w = (act && s2 <= rc2) ? w : (T)0;
          const T p = w * (qi + qj);  // 2 * symmetric P_ij
#pragma unroll
          for (int s = 0; s < SMAX; ++s) accr[s] += p * (mj[s] - Mi[s]);
        };
        for (uint32_t b = 0; b < nblk;) {
          const uint32_t bend = nblk - b > kFlushBlocks ? b + kFlushBlocks : nblk;
          for (; b < bend; ++b, j += L * kUnroll) {
            T xj[kUnroll][DIM], qj[kUnroll], mj[kUnroll][SMAX];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
              load_pos<T, DIM>(pos, j + u * L, xj[u]);
              qj[u] = q[j + u * L];
              load_mass<T, SMAX>(min_, j + u * L, mj[u]);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) eval(xj[u], qj[u], mj[u]);
          }
#pragma unroll
          for (int s = 0; s < SMAX; ++s) {
            acc[s] += (double)accr[s];
            accr[s] = (T)0;
          }
        }
        for (; j < je; j += L) {
          T xj[DIM], mj[SMAX];
          load_pos<T, DIM>(pos, j, xj);
          load_mass<T, SMAX>(min_, j, mj);
          eval(xj, q[j], mj);
        }
#pragma unroll
        for (int s = 0; s < SMAX; ++s) acc[s] += (double)accr[s];
      });
    } else {
      for_tile_rows<LOG2L>(P, st, cell_start, tl, [&](uint32_t jb, uint32_t je, bool act) {
        T accr[SMAX];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) accr[s] = (T)0;
        T rr = (T)0;
        const uint32_t len = je - jb, nblk = len / (L * kUnroll);
        uint32_t j = jb + tl.gl;
        auto eval = [&](const T xj[DIM], const T mj[SMAX]) {
          const T s2 = sep2v<T, DIM>(xi, xj);
          T w = wfn(s2, esc);
          w = (act && s2 <= rc2) ? w : (T)0;
          rr += w;
#pragma unroll
          for (int s = 0; s < SMAX; ++s) accr[s] += w * (mj[s] - Mi[s]);
        };
        for (uint32_t b = 0; b < nblk;) {
          const uint32_t bend = nblk - b > kFlushBlocks ? b + kFlushBlocks : nblk;
          for (; b < bend; ++b, j += L * kUnroll) {
            T xj[kUnroll][DIM], mj[kUnroll][SMAX];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
              load_pos<T, DIM>(pos, j + u * L, xj[u]);
              load_mass<T, SMAX>(min_, j + u * L, mj[u]);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) eval(xj[u], mj[u]);
          }
#pragma unroll
          for (int s = 0; s < SMAX; ++s) {
            acc[s] += (double)accr[s];
            accr[s] = (T)0;
          }
          racc += (double)rr;
          rr = (T)0;
        }
        for (; j < je; j += L) {
          T xj[DIM], mj[SMAX];
          load_pos<T, DIM>(pos, j, xj);
          load_mass<T, SMAX>(min_, j, mj);
          eval(xj, mj);
        }
#pragma unroll
        for (int s = 0; s < SMAX; ++s) acc[s] += (double)accr[s];
        racc += (double)rr;
      });
    }
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
#pragma unroll
    for (int s = 0; s < SMAX; ++s) acc[s] += __shfl_xor(acc[s], off);
    racc += __shfl_xor(racc, off);
  }
  exchange_epilogue<T, SMAX, G>(P, sym, acc, racc, Mi, tl.gl == 0 && tl.valid, tl.i, mout, S, react_a,
                                react_b, audit_part, wave_tile());
}

// ---------------------------------------------------------------------------
// Pair kernels, 4 lanes per particle with DPP row broadcast (binary32).
//
// A wave holds 16 particles (gi = lane & 15) in each of its four 16-lane rows
// (gl = lane >> 4).  The tile's candidate rows are streamed as one virtual
// list: every lane loads one candidate of a chunk of 64 (coalesced, one load
// per array), then in 16 steps row gl evaluates candidate 16 gl + k, which
// `row_share:k` broadcasts to the whole row straight into the consuming VALU
// instruction.  Each particle sees all 64 candidates across its four lanes.
// ---------------------------------------------------------------------------

// Wave-uniform cursor over the non-empty stencil rows of one segment.
struct RowCursor {
  int r;            // next stencil entry to examine
  uint32_t jb, je;  // current row's sorted candidate range
  uint32_t p;       // virtual index of jb
  bool valid;
};

__device__ __forceinline__ void cursor_advance(RowCursor& c, const RealParams& P, const StencilRow* __restrict__ st,
                                               const uint32_t* __restrict__ cell_start, int cy, int cz, int cxa,
                                               int cxb) {
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  c.valid = false;
  while (c.r < P.n_stencil) {
    const StencilRow sr = st[P.stencil_off + c.r];
    ++c.r;
    const int ny = cy + sr.dy, nz = cz + sr.dz;
    if (ny < 0 || ny >= nc1 || nz < 0 || nz >= nc2) continue;
    const int xa = cxa - sr.rx < 0 ? 0 : cxa - sr.rx;
    const int xb = cxb + sr.rx > nc0 - 1 ? nc0 - 1 : cxb + sr.rx;
    const int64_t cb = P.cell_off + ((int64_t)nz * nc1 + ny) * nc0;
    const uint32_t jb = cell_start[cb + xa], je = cell_start[cb + xb + 1];
    if (je > jb) {
      c.jb = jb;
      c.je = je;
      c.valid = true;
      return;
    }
  }
}

// Lane `lane` of the chunk starting at virtual index vbase: its candidate j
// (or jdummy when the chunk runs past the segment's last row), advancing the
// cursor over every row that ends inside the chunk.
__device__ __forceinline__ void chunk_pick(RowCursor& c, const RealParams& P, const StencilRow* __restrict__ st,
                                           const uint32_t* __restrict__ cell_start, int cy, int cz, int cxa,
                                           int cxb, uint32_t vbase, int32_t jdummy, int32_t& j, bool& has) {
  const uint32_t v = vbase + (uint32_t)(threadIdx.x & 63);
  j = jdummy;
  has = false;
  while (c.valid) {
    const uint32_t len = c.je - c.jb;
    if (v >= c.p && v < c.p + len) {
      j = (int32_t)(c.jb + (v - c.p));
      has = true;
    }
    if (c.p + len <= vbase + 64) {
      c.p += len;
      cursor_advance(c, P, st, cell_start, cy, cz, cxa, cxb);
    } else {
      break;
    }
  }
}

// A segment's last chunk when it holds n <= 32 candidates: lane (g, K) of
// row g takes candidate g * per + K for K < per (per = 4 for n <= 16, else 8),
// so that the chunk is evaluated in per broadcast steps instead of 16.  The
// picked (j, has) of candidate c sits in lane c; every lane takes part in the
// permutes.  Returns the chunk's step count.
__device__ __forceinline__ int chunk_compact(const RowCursor& c, uint32_t vbase, int32_t& j, bool& has) {
  if (c.valid) return 16;
  const uint32_t n = __builtin_amdgcn_readfirstlane(c.p - vbase);
  if (n > 32u) return 16;
  const int per = n > 16u ? 8 : 4;
  const int lane = threadIdx.x & 63, g = lane >> 4, k = lane & 15;
  const int src = g * per + k;  // < 64 for every lane
  const int32_t js = __shfl(j, src);
  const bool hs = __shfl(has ? 1 : 0, src) != 0;
  j = js;
  has = hs && k < per;
  return per;
}

// compute(data, act, nk) with the step count nk as a compile-time constant.
template <typename ComputeFn, typename Data>
__device__ __forceinline__ void compute_steps(ComputeFn&& compute, const Data& d, bool act, int nk) {
  if (nk == 16) compute(d, act, std::integral_constant<int, 16>{});
  else if (nk == 8) compute(d, act, std::integral_constant<int, 8>{});
  else compute(d, act, std::integral_constant<int, 4>{});
}

// Runs compute(load(j, has), act, nk) for every chunk of 64 virtual
// candidates of every segment of the tile (NPARTS > 1: only chunks part, part
// + NPARTS, ...; the cursor still walks the others, without loads); `act`
// marks the lanes whose particle is in the segment, nk the chunk's broadcast
// steps (16, or 8 or 4 for a short last chunk of a whole-tile launch; the
// split form keeps 16, where the compaction measured slower).  Software-pipelined: the
// candidates of the next chunk are picked and their loads issued before the
// current chunk is computed, so the load latency overlaps the chunk's
// arithmetic.
template <int NPARTS, typename LoadFn, typename ComputeFn>
__device__ __forceinline__ void for_tile_chunks(const RealParams& P, const StencilRow* __restrict__ st,
                                                const uint32_t* __restrict__ cell_start, const TileLane& tl,
                                                int32_t jdummy, int part, LoadFn&& load, ComputeFn&& compute) {
  const int nc1 = P.nc[1];
  int seg = 0;
  while (seg < tl.n_in) {
    const int seg_row = __builtin_amdgcn_readlane(tl.row, seg);
    const unsigned long long m =
        __ballot(tl.gl == 0 && tl.gi > seg && (tl.gi >= tl.n_in || tl.row != seg_row));
    int seg_end = m ? (__ffsll((unsigned long long)m) - 1) : tl.n_in;
    seg_end = seg_end > tl.n_in ? tl.n_in : seg_end;
    const int cxa = __builtin_amdgcn_readlane(tl.cx, seg);
    const int cxb = __builtin_amdgcn_readlane(tl.cx, seg_end - 1);
    const bool act = tl.valid && tl.gi >= seg && tl.gi < seg_end;
    const int cy = seg_row % nc1, cz = seg_row / nc1;
    RowCursor c;
    c.r = 0;
    c.p = 0;
    cursor_advance(c, P, st, cell_start, cy, cz, cxa, cxb);
    // after picking the chunk at vbase, c.valid says whether a chunk follows
    uint32_t vbase = 0;
    int32_t j;
    bool has;
    if constexpr (NPARTS > 1) {
      for (int k = 0; k < part && c.valid; ++k) {  // chunks before this part's first
        chunk_pick(c, P, st, cell_start, cy, cz, cxa, cxb, vbase, jdummy, j, has);
        vbase += 64;
      }
    }
    if (c.valid) {
      chunk_pick(c, P, st, cell_start, cy, cz, cxa, cxb, vbase, jdummy, j, has);
      int nk = NPARTS == 1 ? chunk_compact(c, vbase, j, has) : 16;
      auto cur = load(j, has);
      while (true) {
        if constexpr (NPARTS > 1) {
          for (int k = 1; k < NPARTS && c.valid; ++k) {  // the other parts' chunks
            vbase += 64;
            chunk_pick(c, P, st, cell_start, cy, cz, cxa, cxb, vbase, jdummy, j, has);
          }
        }
        const bool next = c.valid;
        decltype(cur) nxt = cur;
        int nk_next = 16;
        if (next) {
          vbase += 64;
          chunk_pick(c, P, st, cell_start, cy, cz, cxa, cxb, vbase, jdummy, j, has);
          if constexpr (NPARTS == 1) nk_next = chunk_compact(c, vbase, j, has);
          nxt = load(j, has);
        }
        if constexpr (NPARTS == 1) compute_steps(compute, cur, act, nk);
        else compute(cur, act, std::integral_constant<int, 16>{});
        if (!next) break;
        cur = nxt;
        nk = nk_next;
      }
    }
    seg = seg_end;
  }
}

template <int DIM, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_rowsum_dpp(
    const float* __restrict__ pos, const uint32_t* __restrict__ skey,
    const uint32_t* __restrict__ cell_start, const Tile* __restrict__ tiles, const int32_t ntiles,
    const RealParams* __restrict__ rp, const StencilRow* __restrict__ st, double* __restrict__ r_out,
    float* __restrict__ q_out) {
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<2, SPLIT>(tiles, ntiles, tl, tile)) return;  // block-uniform when SPLIT > 1
  const int part = SPLIT > 1 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  float xi[DIM];
  load_pos<float, DIM>(pos, ii, xi);
  lane_cell<float, DIM>(P, skey, ii, tl);
  const float rc2 = P.rc2_f, esc = P.escale_f;
  double acc = 0.0;
  if (P.active) {
    struct Cand {
      float x[DIM];
      bool has;
    };
    for_tile_chunks<SPLIT>(
        P, st, cell_start, tl, tile.begin, part,
        [&](int32_t j, bool has) {
          Cand d;
          load_pos<float, DIM>(pos, j, d.x);
          d.has = has;
          return d;
        },
        [&](const Cand& d, bool act, auto nkc) {
          float xj[DIM];
#pragma unroll
          for (int k = 0; k < DIM; ++k) xj[k] = d.x[k];
          if (!d.has) xj[0] = 3.0e38f;  // s^2 overflows to +inf: outside the cutoff, weight 0
          acc += (double)rowsum_chunk<DIM, decltype(nkc)::value>(xj, xi, rc2, esc, act);
        });
  } else {
    acc = 1.0;
  }
  if constexpr (SPLIT > 1) {
    // the parts' partial sums, added in part order by the first wave
    __shared__ double sh_part[SPLIT - 1][64];
    const int lane = threadIdx.x & 63;
    if (part > 0) sh_part[part - 1][lane] = acc;
    __syncthreads();
    if (part > 0) return;
#pragma unroll
    for (int w = 0; w < SPLIT - 1; ++w) acc += sh_part[w][lane];
  }
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (tl.gl == 0 && tl.valid) {
    if (!P.active) acc = 1.0;
    if (r_out) r_out[tl.i] = acc;
    q_out[tl.i] = (float)(1.0 / acc);
  }
}

template <int DIM, int SMAX, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_exchange_dpp(
    const float* __restrict__ pos, const float* __restrict__ min_, float* __restrict__ mout,
    const float* __restrict__ q, const uint32_t* __restrict__ skey, const uint32_t* __restrict__ cell_start,
    const Tile* __restrict__ tiles, const int32_t ntiles, const RealParams* __restrict__ rp,
    const StencilRow* __restrict__ st, const int32_t S, const int32_t react_a, const int32_t react_b,
    const int32_t norm, double* __restrict__ audit_part) {
  constexpr int G = 16;
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<2, SPLIT>(tiles, ntiles, tl, tile)) return;  // block-uniform when SPLIT > 1
  const int part = SPLIT > 1 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  float xi[DIM];
  load_pos<float, DIM>(pos, ii, xi);
  float Mi[SMAX];
  load_mass<float, SMAX>(min_, ii, Mi);
  lane_cell<float, DIM>(P, skey, ii, tl);
  const float rc2 = P.rc2_f, esc = P.escale_f;
  double acc[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) acc[s] = 0.0;
  double racc = 0.0;
  const bool sym = (norm == 0);
  const float qi = q[ii];
  if (P.active) {
    struct Cand {
      float x[DIM], m[SMAX], q;
      bool has;
    };
    for_tile_chunks<SPLIT>(
        P, st, cell_start, tl, tile.begin, part,
        [&](int32_t j, bool has) {
          Cand d;
          load_pos<float, DIM>(pos, j, d.x);
          d.q = q[j];
          // species slots S..SMAX-1 exist and hold zeros, so no guard is needed
          load_mass<float, SMAX>(min_, j, d.m);
          d.has = has;
          return d;
        },
        [&](const Cand& d, bool act, auto nkc) {
          constexpr int NK = decltype(nkc)::value;
          float xj[DIM], mj[SMAX];
#pragma unroll
          for (int k = 0; k < DIM; ++k) xj[k] = d.x[k];
#pragma unroll
          for (int s = 0; s < SMAX; ++s) mj[s] = d.m[s];
          if (!d.has) xj[0] = 3.0e38f;  // outside the cutoff, weight 0
          float accr[SMAX];
#pragma unroll
          for (int s = 0; s < SMAX; ++s) accr[s] = 0.0f;
          float rr = 0.0f;
          if (sym) {
            exchange_chunk_sym<DIM, SMAX, NK>(xj, xi, d.q, qi, mj, Mi, rc2, esc, act, accr);
          } else {
            exchange_chunk_row<DIM, SMAX, NK>(xj, xi, mj, Mi, rc2, esc, act, rr, accr);
          }
#pragma unroll
          for (int s = 0; s < SMAX; ++s) acc[s] += (double)accr[s];
          if (!sym) racc += (double)rr;  // r_i: only the row normalisation divides by it
        });
  }
  if constexpr (SPLIT > 1) {
    // the parts' partial sums, added in part order by the first wave
    __shared__ double sh_part[SPLIT - 1][SMAX + 1][64];
    const int lane = threadIdx.x & 63;
    if (part > 0) {
#pragma unroll
      for (int s = 0; s < SMAX; ++s) sh_part[part - 1][s][lane] = acc[s];
      sh_part[part - 1][SMAX][lane] = racc;
    }
    __syncthreads();
    if (part > 0) return;
#pragma unroll
    for (int w = 0; w < SPLIT - 1; ++w) {
#pragma unroll
      for (int s = 0; s < SMAX; ++s) acc[s] += sh_part[w][s][lane];
      racc += sh_part[w][SMAX][lane];
    }
  }
#pragma unroll
  for (int off = 16; off < 64; off <<= 1) {
#pragma unroll
    for (int s = 0; s < SMAX; ++s) acc[s] += __shfl_xor(acc[s], off);
    if (!sym) racc += __shfl_xor(racc, off);
  }
  exchange_epilogue<float, SMAX, G>(P, sym, acc, racc, Mi, tl.gl == 0 && tl.valid, tl.i, mout, S,
                                    react_a, react_b, audit_part, wave_tile<SPLIT>());
}

// ---------------------------------------------------------------------------
// Pair kernels with private candidate lists: one lane per particle, for
// sparse neighbourhoods, where the candidate union of a shared tile would be
// mostly misses.  The row-sum pass takes each particle's own cutoff box and
// keeps its neighbours in a per-wave cache; the exchange reads the cache, and
// lanes that overflowed it walk the stencil rows [cx - rx, cx + rx] around
// their cell (for_own_rows).
// ---------------------------------------------------------------------------

template <typename T, int DIM, typename RowFn>
__device__ __forceinline__ void for_own_rows(const RealParams& P, const StencilRow* __restrict__ st,
                                             const uint32_t* __restrict__ cell_start, uint32_t lk, RowFn&& fn) {
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  const int cx = (int)(lk % (uint32_t)nc0);
  const int rest = (int)(lk / (uint32_t)nc0);
  const int cy = rest % nc1, cz = rest / nc1;
  for (int r = 0; r < P.n_stencil; ++r) {
    const StencilRow sr = st[P.stencil_off + r];
    const int ny = cy + sr.dy, nz = cz + sr.dz;
    if (ny < 0 || ny >= nc1 || nz < 0 || nz >= nc2) continue;
    const int xa = cx - sr.rx < 0 ? 0 : cx - sr.rx;
    const int xb = cx + sr.rx > nc0 - 1 ? nc0 - 1 : cx + sr.rx;
    const int64_t cb = P.cell_off + ((int64_t)nz * nc1 + ny) * nc0;
    fn(cell_start[cb + xa], cell_start[cb + xb + 1]);
  }
}


// Row-sum pass of the one-lane-per-particle kernels.  Each lane takes the
// cells its own cutoff box [x - r, x + r]^d overlaps (r the geometric cutoff,
// cells by the same monotone map as the cell keys, so no neighbour is
// missed): per axis a cell range, hence (y, z) rows of one contiguous x-range
// each.  Rows are taken kRowBatch at a time: all their cell ranges are loaded
// first, then the concatenated candidate list is walked kCandBatch candidates
// per iteration with all their loads in flight.  Candidate t of the
// concatenation is j = t + delta[q] for the last row q whose first flat index
// off[q] is <= t.
template <int DIM>
struct PrivBatch {
  // two rows at a time in 2-D and 3-D: every iteration waits for the lane with
  // the longest concatenation, and two shorter ones waste fewer slots than one
  // of all four rows (8e6 particles in 3-D, steps of 0.655 against 0.660 ms
  // with four rows; 0.68-0.72 ms with one row at a time)
  static constexpr int kRowBatch = DIM == 1 ? 1 : 2;
  // six keeps eight waves per SIMD in the binary32 3-D row sum; measured
  // against 2, 3, 4, 8 and 12 at 8e6 particles (225.7 us against 315, 286,
  // 267, 230 and 259)
  static constexpr int kCandBatch = 6;
};

// Cell coordinate of coordinate value v along axis k (as the cell keys map it).
// Clamped in floating point first, so that an infinite cutoff (v = +-inf)
// converts safely.
__device__ __forceinline__ int cell_of(const RealParams& P, int k, double v) {
  double u = floor((v - P.lo[k]) * P.inv_h[k]);
  u = u < 0.0 ? 0.0 : u;
  u = u > (double)(P.nc[k] - 1) ? (double)(P.nc[k] - 1) : u;
  return (int)u;
}

// Candidate walk of the one-lane-per-particle kernels: the (y, z) rows of
// cells that the lane's own cutoff box overlaps, each one contiguous sorted
// range, taken kRowBatch rows at a time; their concatenation is walked
// kCandBatch candidates per call of batch(jv, s2, ok) with all the batch's
// position loads issued together.  jv: sorted indices; s2: squared
// separations (sep2v, the cutoff predicate's arithmetic); ok: whether the
// entry is a candidate (the tail of the last batch repeats particle ii).
template <typename T, int DIM, typename BatchFn>
__device__ __forceinline__ void priv_walk(const RealParams& P, const uint32_t* __restrict__ cell_start,
                                          const T* __restrict__ pos, const T (&xi)[DIM], int32_t ii,
                                          BatchFn&& batch) {
  constexpr int RB = PrivBatch<DIM>::kRowBatch, CB = PrivBatch<DIM>::kCandBatch;
  const double rg = P.rc_geo;
  int ca[3] = {0, 0, 0}, cb_[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    ca[k] = cell_of(P, k, (double)xi[k] - rg);
    cb_[k] = cell_of(P, k, (double)xi[k] + rg);
  }
  const int nyr = cb_[1] - ca[1] + 1;
  const int nrows = nyr * (cb_[2] - ca[2] + 1);
  const uint32_t nc0 = (uint32_t)P.nc[0], nc1 = (uint32_t)P.nc[1];
  const uint32_t coff = (uint32_t)P.cell_off;
  // rows in turn from the particle's own (y, z) row, so that the lanes of a
  // wave (mostly one cell row) gather from the same rows at the same time
  const int cy = DIM > 1 ? cell_of(P, 1, (double)xi[1]) : 0, cz = DIM > 2 ? cell_of(P, 2, (double)xi[2]) : 0;
  int yy = cy, zz = cz;
  for (int r0 = 0; r0 < nrows; r0 += RB) {
    uint32_t off[RB];
    int32_t delta[RB];
    uint32_t total = 0;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const bool in = r0 + q < nrows;
      const uint32_t base = coff + ((uint32_t)zz * nc1 + (uint32_t)yy) * nc0;
      const uint32_t jb = cell_start[base + (uint32_t)ca[0]];
      const uint32_t je = cell_start[base + (uint32_t)cb_[0] + 1u];
      off[q] = total;
      delta[q] = (int32_t)jb - (int32_t)total;
      total += in ? je - jb : 0u;
      // next row: y fastest, each axis cycling from the own cell; past the
      // last row (yy, zz) keeps cycling over valid cells
      const int yn = yy == cb_[1] ? ca[1] : yy + 1;
      zz = yn == cy ? (zz == cb_[2] ? ca[2] : zz + 1) : zz;
      yy = yn;
    }
    for (uint32_t t0 = 0; t0 < total; t0 += CB) {
      uint32_t jv[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const uint32_t t = t0 + u;
        int32_t d = delta[0];
#pragma unroll
        for (int q = 1; q < RB; ++q) d = t >= off[q] ? delta[q] : d;
        jv[u] = t < total ? (uint32_t)((int32_t)t + d) : (uint32_t)ii;
      }
      T xj[CB][DIM];
#pragma unroll
      for (int u = 0; u < CB; ++u) load_pos<T, DIM>(pos, jv[u], xj[u]);
      T s2[CB];
      bool ok[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        s2[u] = sep2v<T, DIM>(xi, xj[u]);
        ok[u] = t0 + u < total;
      }
      batch(jv, s2, ok);
    }
  }
}

// (eight waves per SIMD: the binary32 form then fits 64 VGPRs without spills)
template <typename T, int DIM, bool IND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_rowsum_priv(
    const T* __restrict__ pos, const uint32_t* __restrict__ cell_start, const Tile* __restrict__ tiles,
    const int32_t ntiles, const RealParams* __restrict__ rp, double* __restrict__ r_out,
    T* __restrict__ q_out, uint16_t* __restrict__ nb_meta, uint32_t* __restrict__ nb_idx,
    T* __restrict__ nb_w, uint32_t* __restrict__ nb_src, const uint32_t* __restrict__ src_of) {
  constexpr int CB = PrivBatch<DIM>::kCandBatch;
  WeightFn<T> wfn;  // before any return: the binary64 form has a block barrier
  wfn.setup();
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(tiles, ntiles, tl, tile)) return;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  const T rc2 = rc2_of<T>(P), esc = escale_of<T>(P);
  double acc = 1.0;  // only the self weight when the transfer is off
  // the lane's cached neighbours, slot-major per wave: [slot][lane]
  __shared__ uint32_t sh_j[kBlock / 64][kCacheLane * 64];
  __shared__ T sh_w[kBlock / 64][kCacheLane * 64];
  const int lane = threadIdx.x & 63;
  uint32_t* const lj = &sh_j[threadIdx.x >> 6][lane];
  T* const lw = &sh_w[threadIdx.x >> 6][lane];
  uint32_t cnt = 0;
  if (P.active && tl.valid) {
    acc = 0.0;
    priv_walk<T, DIM>(P, cell_start, pos, xi, ii, [&](const uint32_t (&jv)[CB], const T (&s2)[CB],
                                                      const bool (&ok)[CB]) {
      T a = (T)0;
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const T w = wfn(s2[u], esc);
        const bool hit = ok[u] && s2[u] <= rc2;
        a += hit ? w : (T)0;
        if (hit && jv[u] != (uint32_t)ii && cnt <= (uint32_t)kCacheLane) {
          if (cnt < (uint32_t)kCacheLane) {
            lj[cnt * 64] = jv[u];
            lw[cnt * 64] = w;
          }
          ++cnt;
        }
      }
      acc += (double)a;
    });
  }
  // wave-exclusive prefix of the kept counts (each at most kCacheLane < 16)
  const uint32_t keep = cnt <= (uint32_t)kCacheLane ? cnt : 0u;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t off = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) off += (uint32_t)__popcll(__ballot((keep >> b) & 1u) & below) << b;
  // Lanes whose entries would pass the end of the wave's region come after
  // every lane that keeps its entries (the offsets only grow), so the kept
  // entries are [0, nent) of the region.
  const bool miss = cnt > (uint32_t)kCacheLane || off + keep > (uint32_t)kCacheWave;
  const uint32_t nent = wave_max_u32(miss ? 0u : off + keep);
  // The wave writes its entries flat, entry e by lane e mod 64: coalesced
  // stores and one gather of the previous slots per 64 entries, instead of
  // each lane storing its own up to kCacheLane entries.  The entry's owner
  // is the last lane whose offset is <= e (a lane with no entries shares its
  // offset with the next lane).
  wave_lds_fence();
  const int64_t wbase = wave_tile() * kCacheWave;
  for (uint32_t r0 = 0; r0 < nent; r0 += 64) {
    const uint32_t e = r0 + (uint32_t)lane;
    int o = 0;
#pragma unroll
    for (int b = 32; b; b >>= 1) o = __shfl(off, o + b) <= e ? o + b : o;
    // every lane takes part in the permutes (one from a disabled lane reads zero)
    const uint32_t off_o = __shfl(off, o);
    const bool have = e < nent;
    const uint32_t k = have ? e - off_o : 0u;
    const uint32_t j = sh_j[threadIdx.x >> 6][k * 64 + (have ? o : lane)];
    const T w = sh_w[threadIdx.x >> 6][k * 64 + (have ? o : lane)];
    uint32_t s = 0;
    if constexpr (IND) s = src_of[have ? j : 0u];
    if (have) {
      nb_idx[wbase + e] = j;
      nb_w[wbase + e] = w;
      if constexpr (IND) nb_src[wbase + e] = s;
    }
  }
  if (!tl.valid) return;
  if (r_out) r_out[ii] = acc;
  q_out[ii] = (T)(1.0 / acc);
  nb_meta[ii] = miss ? (uint16_t)kCacheMiss : (uint16_t)(keep ? ((off << 4) | keep) : 0u);
}

// Exchange with the row-sum pass's neighbour cache.  The wave reads its
// cached entries flat, entry e by lane e mod 64 (coalesced loads, one gather
// of the neighbours' q and masses per 64 entries), stages them in LDS, and
// each lane then adds its own entries in their order: no positions, no
// search.  A lane marked as a miss walks its stencil rows as the row-sum pass
// did.  r_i for the row normalisation comes from the row-sum pass.
template <typename T, int DIM, int SMAX, bool IND>
__global__ __launch_bounds__(kBlock) void k_exchange_priv(
    const T* __restrict__ pos, const T* __restrict__ min_, T* __restrict__ mout,
    const T* __restrict__ q, const double* __restrict__ r_in, const uint32_t* __restrict__ skey,
    const uint32_t* __restrict__ cell_start, const Tile* __restrict__ tiles, const int32_t ntiles,
    const RealParams* __restrict__ rp, const StencilRow* __restrict__ st, const int32_t S,
    const int32_t react_a, const int32_t react_b, const int32_t norm, double* __restrict__ audit_part,
    const uint16_t* __restrict__ nb_meta, const uint32_t* __restrict__ nb_idx, const T* __restrict__ nb_w,
    const uint32_t* __restrict__ nb_src, const uint32_t* __restrict__ src_of) {
  WeightFn<T> wfn;  // before any return: the binary64 form has a block barrier
  wfn.setup();
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(tiles, ntiles, tl, tile)) return;
  const RealParams& P = rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T Mi[SMAX];
  load_mass<T, SMAX>(min_, IND ? src_of[ii] : (uint32_t)ii, Mi);
  double acc[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) acc[s] = 0.0;
  double racc = 0.0;
  const bool sym = (norm == 0);
  const bool mine = P.active && tl.valid;
  const T qi = mine ? q[ii] : (T)0;
  const uint32_t meta = mine ? (uint32_t)nb_meta[ii] : kCacheMiss;
  const bool cached = mine && (meta & 15u) != kCacheMiss;
  const uint32_t c = cached ? meta & 15u : 0u, off = meta >> 4;
  // the kept entries of the wave are [0, nent) of its region
  const uint32_t nent = wave_max_u32(cached ? off + c : 0u);
  const uint32_t cmax = wave_max_u32(c);
  // at most kCacheLane terms per lane, summed in the path's precision, then widened
  T accc[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) accc[s] = (T)0;
  __shared__ T st_m[kBlock / 64][64 * SMAX];  // staged masses of the round's entries
  __shared__ T st_wq[kBlock / 64][64 * 2];    // staged (w_ij, q_j)
  T* const sm = st_m[threadIdx.x >> 6];
  T* const swq = st_wq[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  const int64_t wbase = wave_tile() * kCacheWave;
  for (uint32_t r0 = 0; r0 < nent; r0 += 64) {
    const uint32_t e = r0 + (uint32_t)lane;
    const int64_t ge = wbase + (e < nent ? e : 0u);  // entry 0 exists when nent > 0
    const uint32_t j = nb_idx[ge];
    const uint32_t sj = IND ? nb_src[ge] : j;
    typename VecOf<T, 2>::type wq;
    wq.x = nb_w[ge];
    wq.y = q[j];
    T Mj[SMAX];
    load_mass<T, SMAX>(min_, sj, Mj);
    wave_lds_fence();  // the previous round's LDS loads stay before these stores
    store_mass<T, SMAX>(sm, lane, Mj);
    *(typename VecOf<T, 2>::type*)(swq + 2 * lane) = wq;
    wave_lds_fence();
    for (uint32_t k = 0; k < cmax; ++k) {
      const uint32_t ek = off + k - r0;  // the entry's lane in this round
      if (k < c && off + k >= r0 && ek < 64u) {
        T mj[SMAX];
        load_mass<T, SMAX>(sm, ek, mj);
        const typename VecOf<T, 2>::type v = *(const typename VecOf<T, 2>::type*)(swq + 2 * ek);
        const T p = sym ? v.x * (qi + v.y) : v.x;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) accc[s] += p * (mj[s] - Mi[s]);
      }
    }
  }
  if (cached) {
    racc = sym ? 1.0 : r_in[ii];  // only the row normalisation divides by r_i
#pragma unroll
    for (int s = 0; s < SMAX; ++s) acc[s] = (double)accc[s];
  } else if (mine) {
    T xi[DIM];
    load_pos<T, DIM>(pos, ii, xi);
    const T rc2 = rc2_of<T>(P), esc = escale_of<T>(P);
    // each term is added in binary64 as it is found (the terms are few; no
    // binary32 partials beside the binary64 sums)
    for_own_rows<T, DIM>(P, st, cell_start, skey[ii] - (uint32_t)P.cell_off, [&](uint32_t jb, uint32_t je) {
      for (uint32_t j = jb; j < je; ++j) {
        const T s2 = sep2<T, DIM>(xi, pos, j);
        if (!(s2 <= rc2)) continue;  // sparse: most candidates miss, skip their loads
        const T w = wfn(s2, esc);
        // species slots S..SMAX-1 exist and hold zeros
        const T p = sym ? w * (qi + q[j]) : w;
        racc += (double)w;
        T mj[SMAX];
        load_mass<T, SMAX>(min_, IND ? src_of[j] : j, mj);
#pragma unroll
        for (int s = 0; s < SMAX; ++s) acc[s] += (double)(p * (mj[s] - Mi[s]));
      }
    });
  }
  exchange_epilogue<T, SMAX, 64>(P, sym, acc, racc, Mi, tl.valid, tl.i, mout, S, react_a, react_b,
                                 audit_part, wave_tile());
}

// Counts ordered pairs j != i within the cutoff and candidate evaluations.
template <typename T, int DIM, int LOG2L>
__global__ __launch_bounds__(kBlock) void k_count(PairArgs a) {
  constexpr int L = 1 << LOG2L;
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<LOG2L>(a.tiles, a.ntiles, tl, tile)) return;
  const RealParams& P = a.rp[tile.real];
  const T* __restrict__ pos = (const T*)a.pos;
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  const uint32_t lk = a.skey[ii] - (uint32_t)P.cell_off;
  tl.cx = (int)(lk % (uint32_t)P.nc[0]);
  tl.row = (int)(lk / (uint32_t)P.nc[0]);
  const T rc2 = rc2_of<T>(P);
  unsigned long long pairs = 0, evals = 0;
  if (P.active) {
    for_tile_rows<LOG2L>(P, a.st, a.cell_start, tl, [&](uint32_t jb, uint32_t je, bool act) {
      const uint32_t len = je - jb, nfull = len >> LOG2L, rem = len & (L - 1);
      uint32_t j = jb + tl.gl;
      auto body = [&](uint32_t jj) {
        const T s2 = sep2<T, DIM>(xi, pos, jj);
        if (act) {
          ++evals;
          if (s2 <= rc2 && jj != (uint32_t)tl.i) ++pairs;
        }
      };
      for (uint32_t c = 0; c < nfull; ++c, j += L) body(j);
      if (rem && (uint32_t)tl.gl < rem) body(j);
    });
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    pairs += __shfl_xor(pairs, off);
    evals += __shfl_xor(evals, off);
  }
  if ((threadIdx.x & 63) == 0) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    a.counts[2 * t] = pairs;
    a.counts[2 * t + 1] = evals;
  }
}

// The same counts for the private-list kernels: every particle's candidates
// are those of the row-sum pass's own walk (priv_walk).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_count_priv(PairArgs a) {
  constexpr int CB = PrivBatch<DIM>::kCandBatch;
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(a.tiles, a.ntiles, tl, tile)) return;
  const RealParams& P = a.rp[tile.real];
  const T* __restrict__ pos = (const T*)a.pos;
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  const T rc2 = rc2_of<T>(P);
  unsigned long long pairs = 0, evals = 0;
  if (P.active && tl.valid) {
    priv_walk<T, DIM>(P, a.cell_start, pos, xi, ii, [&](const uint32_t (&jv)[CB], const T (&s2)[CB],
                                                        const bool (&ok)[CB]) {
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        evals += ok[u] ? 1u : 0u;
        pairs += (ok[u] && s2[u] <= rc2 && jv[u] != (uint32_t)ii) ? 1u : 0u;
      }
    });
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    pairs += __shfl_xor(pairs, off);
    evals += __shfl_xor(evals, off);
  }
  if ((threadIdx.x & 63) == 0) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    a.counts[2 * t] = pairs;
    a.counts[2 * t + 1] = evals;
  }
}

// Neighbour pairs of the one-lane-per-particle tiling, through the row-sum
// pass's own candidate walk and predicate: FILL = false counts per particle
// (j = i included), FILL = true writes (i, j) sorted-slot pairs at
// rowptr[i] + cursor.
template <typename T, int DIM, bool FILL>
__global__ __launch_bounds__(kBlock) void k_nbr_priv(PairArgs a) {
  constexpr int CB = PrivBatch<DIM>::kCandBatch;
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(a.tiles, a.ntiles, tl, tile)) return;
  if (!tl.valid) return;
  const RealParams& P = a.rp[tile.real];
  const T* __restrict__ pos = (const T*)a.pos;
  const int32_t ii = tl.i;
  auto record = [&](uint32_t j) {
    const uint32_t at = atomicAdd(&a.nbr_cursor[ii], 1u);
    if (FILL) {
      const unsigned long long o = a.nbr_rowptr[ii] + at;
      a.nbr_pairs[2 * o] = (uint32_t)ii;
      a.nbr_pairs[2 * o + 1] = j;
    }
  };
  if (!P.active) {
    record((uint32_t)ii);
    return;
  }
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  const T rc2 = rc2_of<T>(P);
  priv_walk<T, DIM>(P, a.cell_start, pos, xi, ii, [&](const uint32_t (&jv)[CB], const T (&s2)[CB],
                                                      const bool (&ok)[CB]) {
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if (ok[u] && s2[u] <= rc2) record(jv[u]);
  });
}

// Neighbour pairs and counts of the row-broadcast tiling (binary32, four lanes
// per particle), through the chunk enumeration (for_tile_chunks, whole or
// split tiles as the pair kernels are launched) and the per-candidate
// predicate of row_weight.  MODE 0: per-particle counts (j = i included);
// MODE 1: (i, j) pairs at rowptr[i] + cursor; MODE 2: per tile, the ordered
// pairs j != i and the candidate evaluations the pair kernels perform (every
// step of every chunk for every particle of the segment).
template <int DIM, int SPLIT, int MODE>
__global__ __launch_bounds__(kBlock) void k_nbr_dpp(PairArgs a) {
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<2, SPLIT>(a.tiles, a.ntiles, tl, tile)) return;  // block-uniform when SPLIT > 1
  const int part = SPLIT > 1 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const RealParams& P = a.rp[tile.real];
  const float* __restrict__ pos = (const float*)a.pos;
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  float xi[DIM];
  load_pos<float, DIM>(pos, ii, xi);
  lane_cell<float, DIM>(P, a.skey, ii, tl);
  const float rc2 = P.rc2_f;
  unsigned long long pairs = 0, evals = 0;
  auto record = [&](uint32_t j) {
    const uint32_t at = atomicAdd(&a.nbr_cursor[tl.i], 1u);
    if (MODE == 1) {
      const unsigned long long o = a.nbr_rowptr[tl.i] + at;
      a.nbr_pairs[2 * o] = (uint32_t)tl.i;
      a.nbr_pairs[2 * o + 1] = j;
    }
  };
  if (P.active) {
    struct Cand {
      float x[DIM];
      int32_t j;
      bool has;
    };
    for_tile_chunks<SPLIT>(
        P, a.st, a.cell_start, tl, tile.begin, part,
        [&](int32_t j, bool has) {
          Cand d;
          load_pos<float, DIM>(pos, j, d.x);
          d.j = j;
          d.has = has;
          return d;
        },
        [&](const Cand& d, bool act, auto nkc) {
          float xj[DIM];
#pragma unroll
          for (int k = 0; k < DIM; ++k) xj[k] = d.x[k];
          if (!d.has) xj[0] = 3.0e38f;
          const float jf = __builtin_bit_cast(float, d.j);
          const float hf = d.has ? 1.0f : 0.0f;
          Steps<0, decltype(nkc)::value>::run([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            // s^2 of the broadcast candidate exactly as row_weight forms it
            const float d0 = rshare<K>(xj[0]) - xi[0];
            float s2 = d0 * d0;
            if constexpr (DIM > 1) {
              const float d1 = rshare<K>(xj[1]) - xi[1];
              s2 = __builtin_fmaf(d1, d1, s2);
            }
            if constexpr (DIM > 2) {
              const float d2 = rshare<K>(xj[2]) - xi[2];
              s2 = __builtin_fmaf(d2, d2, s2);
            }
            // every broadcast is read with all lanes enabled (a DPP read from
            // a disabled lane does not deliver its value), then combined
            const uint32_t jk = (uint32_t)__builtin_bit_cast(int32_t, rshare<K>(jf));
            const float hk = rshare<K>(hf);
            const bool hit = act & (hk != 0.0f) & (s2 <= rc2);
            if constexpr (MODE == 2) {
              evals += act ? 1u : 0u;
              pairs += (hit && jk != (uint32_t)tl.i) ? 1u : 0u;
            } else {
              if (hit) record(jk);
            }
          });
        });
  } else if (MODE != 2 && tl.valid && tl.gl == 0 && part == 0) {
    record((uint32_t)tl.i);  // only the self pair
  }
  if constexpr (MODE == 2) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      pairs += __shfl_xor(pairs, off);
      evals += __shfl_xor(evals, off);
    }
    const int lane = threadIdx.x & 63;
    if constexpr (SPLIT > 1) {
      __shared__ unsigned long long shc[SPLIT][2];
      if (lane == 0) {
        shc[part][0] = pairs;
        shc[part][1] = evals;
      }
      __syncthreads();
      if (part == 0 && lane == 0) {
        unsigned long long p = 0, e = 0;
#pragma unroll
        for (int w = 0; w < SPLIT; ++w) {
          p += shc[w][0];
          e += shc[w][1];
        }
        const int64_t t = wave_tile<SPLIT>();
        a.counts[2 * t] = p;
        a.counts[2 * t + 1] = e;
      }
    } else if (lane == 0) {
      const int64_t t = wave_tile();
      a.counts[2 * t] = pairs;
      a.counts[2 * t + 1] = evals;
    }
  }
}

// Neighbour export: FILL = false counts per particle (j = i included), FILL =
// true writes (i, j) sorted-slot pairs at rowptr[i] + cursor.
template <typename T, int DIM, int LOG2L, bool FILL>
__global__ __launch_bounds__(kBlock) void k_nbr(PairArgs a) {
  constexpr int L = 1 << LOG2L;
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<LOG2L>(a.tiles, a.ntiles, tl, tile)) return;
  const RealParams& P = a.rp[tile.real];
  const T* __restrict__ pos = (const T*)a.pos;
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  T xi[DIM];
  load_pos<T, DIM>(pos, ii, xi);
  const uint32_t lk = a.skey[ii] - (uint32_t)P.cell_off;
  tl.cx = (int)(lk % (uint32_t)P.nc[0]);
  tl.row = (int)(lk / (uint32_t)P.nc[0]);
  const T rc2 = rc2_of<T>(P);
  if (!P.active) {
    if (tl.valid && tl.gl == 0) {
      if (FILL) {
        const uint32_t at = atomicAdd(&a.nbr_cursor[tl.i], 1u);
        const unsigned long long o = a.nbr_rowptr[tl.i] + at;
        a.nbr_pairs[2 * o] = (uint32_t)tl.i;
        a.nbr_pairs[2 * o + 1] = (uint32_t)tl.i;
      } else {
        atomicAdd(&a.nbr_cursor[tl.i], 1u);
      }
    }
    return;
  }
  for_tile_rows<LOG2L>(P, a.st, a.cell_start, tl, [&](uint32_t jb, uint32_t je, bool act) {
    const uint32_t len = je - jb, nfull = len >> LOG2L, rem = len & (L - 1);
    uint32_t j = jb + tl.gl;
    auto body = [&](uint32_t jj) {
      const T s2 = sep2<T, DIM>(xi, pos, jj);
      if (act && s2 <= rc2) {
        const uint32_t at = atomicAdd(&a.nbr_cursor[tl.i], 1u);
        if (FILL) {
          const unsigned long long o = a.nbr_rowptr[tl.i] + at;
          a.nbr_pairs[2 * o] = (uint32_t)tl.i;
          a.nbr_pairs[2 * o + 1] = jj;
        }
      }
    };
    for (uint32_t c = 0; c < nfull; ++c, j += L) body(j);
    if (rem && (uint32_t)tl.gl < rem) body(j);
  });
}

// ---------------------------------------------------------------------------
// Audit
// ---------------------------------------------------------------------------

constexpr int kAuditValues = 9;  // S + 1 audit values for at most eight species

// Fixed-order sum over the block of acc[0 .. S1): recursive halving inside
// each wave, then the waves added in wave order through LDS.  Thread v < S1
// gets the total of value v; the others get 0.  Every thread must call it.
template <int NV>
__device__ __forceinline__ double block_sum_fixed(double (&acc)[NV], double (*sh)[NV], int S1) {
  constexpr int NK = halved_count(NV, 64);
  constexpr int NB = halving_bits(NV, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int idx = 0, real = NV;
  halve_sum<1, 64, NV, NV>(acc, idx, real, lane);
#pragma unroll
  for (int k = 0; k < NK; ++k)
    if (k < real && lane < (1 << NB)) sh[wave][idx + k] = acc[k];
  __syncthreads();
  double c = 0.0;
  if ((int)threadIdx.x < S1) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) c += sh[w][threadIdx.x];
  }
  __syncthreads();  // sh may be reused on return
  return c;
}

// Audit in one launch: every block sums one chunk of at most kAuditChunk
// consecutive tiles of one realisation (each thread loads all of its
// kAuditChunk / kBlock tiles at once) in a fixed order.  A realisation of one
// chunk is finished by that block.  Otherwise each chunk block publishes its
// sums, and the block that completes the realisation's last chunk (counter
// done[r]) adds the realisation's chunk sums in chunk order with one wave
// (lanes over chunks, then recursive halving), so realisations are finalised
// in parallel and the result does not depend on which block finishes last.
// Block 0 advances the step counter, which no block of this launch reads.
// The counters are returned to zero for the next launch (no memset node, so
// the launch can be captured).
__global__ __launch_bounds__(kBlock) void k_audit(const double* __restrict__ part, int32_t S1,
                                                  const AuditChunk* __restrict__ chunks,
                                                  double* __restrict__ chunk_part,
                                                  const int32_t* __restrict__ chunk_start,
                                                  double* __restrict__ out, uint32_t* __restrict__ done,
                                                  uint64_t* __restrict__ step_ctr, int32_t bump) {
  constexpr int NV = kAuditValues;
  __shared__ double sh[kBlock / 64][NV];
  __shared__ int last;
  const AuditChunk ch = chunks[blockIdx.x];
  // every load of the thread's tiles first, then the sums in tile order
  constexpr int U = kAuditChunk / kBlock;
  double val[U][NV];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = ch.begin + (int)threadIdx.x + u * kBlock;
    const double* pt = part + (int64_t)t * S1;
#pragma unroll
    for (int v = 0; v < NV; ++v) val[u][v] = (t < ch.end && v < S1) ? pt[v] : 0.0;
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += val[u][v];
  const double c = block_sum_fixed<NV>(acc, sh, S1);
  if (bump && blockIdx.x == 0 && threadIdx.x == 0) *step_ctr = *step_ctr + 1;
  const int r = ch.real;
  if (ch.n_in_real == 1) {
    if ((int)threadIdx.x < S1) out[(int64_t)r * S1 + threadIdx.x] = c;
    return;
  }
  if (threadIdx.x < 64) {
    // the writers (S1 <= 9 threads) are all in wave 0, which alone needs the
    // device-scope fence before thread 0 signals completion
    if ((int)threadIdx.x < S1) chunk_part[(int64_t)blockIdx.x * S1 + threadIdx.x] = c;
    __threadfence();
  }
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&done[r], 1u) == (uint32_t)(ch.n_in_real - 1);
  __syncthreads();
  if (last && threadIdx.x < 64) {
    __threadfence();
    const int lane = threadIdx.x;
    const int c0 = chunk_start[r], c1 = chunk_start[r + 1];
    double a[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v] = 0.0;
    for (int k = c0 + lane; k < c1; k += 64) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (v < S1)
          a[v] += __hip_atomic_load(&chunk_part[(int64_t)k * S1 + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    constexpr int NK = halved_count(NV, 64);
    constexpr int NB = halving_bits(NV, 64);
    int ri = 0, rr = NV;
    halve_sum<1, 64, NV, NV>(a, ri, rr, lane);
#pragma unroll
    for (int k = 0; k < NK; ++k)
      if (k < rr && lane < (1 << NB) && ri + k < S1) out[(int64_t)r * S1 + ri + k] = a[k];
    if (lane == 0) done[r] = 0u;
  }
}

// ---------------------------------------------------------------------------
// Half-stencil tiling (binary32): each unordered pair evaluated once.
//
// A work item (one wave) is a segment of seg_w cells of one cell row.  It
// takes the segment's particles in tiles of 16 (one per lane of each 16-lane
// DPP row) and, for each tile, only the forward half of the candidates: the
// later particles of its own row within reach, and the forward stencil rows
// (dz > 0, or dz = 0 and dy > 0).  Pairs inside a tile are evaluated from
// both ends (one-sided).  For the other pairs a row's 16 lanes hold the tile's
// particles and 16 candidates; at step K lane k pairs its particle with the
// candidate K lanes away (DPP row_ror:K, folded into the subtraction), and
// the candidate's accumulator travels with it (row_ror:1 folded into the
// accumulation), so after 16 steps each lane holds, for the candidate it
// loaded, the sum over the tile's particles.  The particle's own sums stay in
// its lane.  The candidate sums are added into slot planes indexed by
// (direction, segment index mod npar): with seg_w >= 2 * the widest reach /
// (npar - 1), at most npar consecutive segments of a row reach any target
// cell, so every slot is written by one wave only, which clears its slots
// first and then accumulates in program order.  A finalizer adds a particle's own sum
// and its slots in a fixed order.  No floating-point atomics: the result is
// bitwise reproducible.
// ---------------------------------------------------------------------------

// Value of the lane K places along this lane's 16-lane row (row_ror:K).
template <int K>
__device__ __forceinline__ float rror(float v) {
  if constexpr (K == 0) {
    return v;
  } else {
    // every source lane of a row rotation exists; bound_ctrl lets the
    // compiler fold the read into the consuming instruction
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + K, 0xf,
                                                                 0xf, true));
  }
}

__device__ __forceinline__ bool forward_row(const StencilRow& sr) { return sr.dz > 0 || (sr.dz == 0 && sr.dy > 0); }

__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Wave-uniform cursor over the forward candidate ranges of one tile: the own
// row first (direction 0: particles after the tile up to the reach), then the
// forward stencil rows in stencil order (directions 1, 2, ... counted whether
// or not the target row exists, as the finalizers count them).
// Forward rows whose candidate ranges a tile loads ahead, with its particles
// (the others are looked up when the cursor reaches them).
constexpr int kHalfPreRows = 2;

struct HalfCursor {
  uint32_t own_je;                                  // end of the own row's range
  uint32_t fjb[kHalfPreRows], fje[kHalfPreRows];    // the first forward rows' ranges
  int k;            // next forward row (-1: the own row is next)
  int f;            // stencil entry to scan from for forward rows past the first kHalfPreRows
  int dix;          // direction of the current range
  uint32_t jb, je;  // current range of sorted indices
  uint32_t p;       // virtual index of jb
  bool valid;
};

// Moves the cursor to the next non-empty range: the own row's later
// particles, then the forward rows in stencil order (direction 1 + their
// index among the forward rows, counted whether or not the row exists); the
// first NPRE forward rows come from the ranges loaded with the tile.
template <int NPRE>
__device__ __forceinline__ void half_advance(HalfCursor& c, const RealParams& P, const StencilRow* __restrict__ st,
                                             const uint32_t* __restrict__ cell_start, int y, int z, int64_t rowbase,
                                             int cxa, int cxb, uint32_t t1) {
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  c.valid = false;
  if (c.k < 0) {
    c.k = 0;
    if (c.own_je > t1) {
      c.jb = t1;
      c.je = c.own_je;
      c.dix = 0;
      c.valid = true;
      return;
    }
  }
  while (c.k < P.n_fwd) {
    const int k = c.k++;
    uint32_t jb = 0u, je = 0u;
    if (k < NPRE) {
#pragma unroll
      for (int u = 0; u < NPRE; ++u)
        if (u == k) {
          jb = c.fjb[u];
          je = c.fje[u];
        }
    } else {
      StencilRow sr = st[P.stencil_off + c.f++];
      while (!forward_row(sr)) sr = st[P.stencil_off + c.f++];  // a k-th forward row exists: k < n_fwd
      const int ty = y + sr.dy, tz = z + sr.dz;
      if (ty >= 0 && ty < nc1 && tz >= 0 && tz < nc2) {
        const int64_t cb = P.cell_off + ((int64_t)tz * nc1 + ty) * nc0;
        const int xa = cxa - sr.rx < 0 ? 0 : cxa - sr.rx;
        const int xb = cxb + sr.rx > nc0 - 1 ? nc0 - 1 : cxb + sr.rx;
        jb = cell_start[cb + xa];
        je = cell_start[cb + xb + 1];
      }
    }
    if (je > jb) {
      c.jb = jb;
      c.je = je;
      c.dix = k + 1;
      c.valid = true;
      return;
    }
  }
}

// Lane's candidate of the chunk at virtual index vbase (jdummy, has = false
// past the last range) and its direction; advances over ranges ending in the
// chunk.
template <int NPRE>
__device__ __forceinline__ void half_pick(HalfCursor& c, const RealParams& P, const StencilRow* __restrict__ st,
                                          const uint32_t* __restrict__ cell_start, int y, int z, int64_t rowbase,
                                          int cxa, int cxb, uint32_t t1, uint32_t vbase, int32_t jdummy, int32_t& j,
                                          bool& has, int& dix) {
  const uint32_t v = vbase + (uint32_t)(threadIdx.x & 63);
  j = jdummy;
  has = false;
  dix = 0;
  while (c.valid) {
    const uint32_t len = c.je - c.jb;
    if (v >= c.p && v < c.p + len) {
      j = (int32_t)(c.jb + (v - c.p));
      has = true;
      dix = c.dix;
    }
    if (c.p + len <= vbase + 64) {
      c.p += len;
      half_advance<NPRE>(c, P, st, cell_start, y, z, rowbase, cxa, cxb, t1);
    } else {
      break;
    }
  }
}

// Dispatch position (a realisation, in the order of item_start) of work item
// w: binary search over the first items.
__device__ __forceinline__ int half_real(const int64_t* __restrict__ item_start, int n_real, int64_t w) {
  int lo = 0, hi = n_real - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (item_start[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One pass of the half-stencil tiling.  EXCH = false: row sums (V = 1, the
// weight w_ij to both ends); EXCH = true: the exchange (V = SMAX species
// values: t = w_ij (q_i + q_j)(M_j - M_i) for the symmetric normalisation or
// w_ij (M_j - M_i) for the row normalisation, +t to i and -t to j).
template <int DIM, int SMAX, bool EXCH, bool SYM>
__global__ __launch_bounds__(kBlock) void k_half_pairs(PairArgs a) {
  constexpr int V = EXCH ? SMAX : 1;
  const int lane = threadIdx.x & 63;
  const int gi = lane & 15, gl = lane >> 4;
  // Items are numbered in dispatch order (realisations by decreasing cost per
  // item).  Blocks are handed to the eight XCDs in turn, so in every round of
  // 8 kHalfGroup launch-order blocks the XCDs each take kHalfGroup
  // consecutive blocks (4 kHalfGroup neighbouring items, which share their
  // halo rows in that XCD's L2): every XCD gets a like share of the costly
  // items and runs its items from the longest.  The last, partial round keeps
  // the launch order.
  const int64_t b = blockIdx.x;
  constexpr int64_t kRound = 8 * kHalfGroup;
  int64_t lb = b;
  if (b < ((int64_t)gridDim.x / kRound) * kRound) {
    const int64_t rr = b % kRound;
    lb = (b - rr) + (rr % 8) * kHalfGroup + rr / 8;
  }
  const int64_t w = lb * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= a.half_nitems) return;
  const int k = __builtin_amdgcn_readfirstlane(half_real(a.half_item_start, a.n_real, w));
  const int r = a.half_item_real[k];
  // a local copy: the slot stores below could alias the parameter array for
  // the compiler, which would then reload its fields after every store
  const RealParams P = a.rp[r];
  if (!P.active || P.nseg <= 0) return;
  const float* __restrict__ pos = (const float*)a.pos;
  const float* __restrict__ min_ = (const float*)a.mass_in;
  const float* __restrict__ q = (const float*)a.q_in;
  float* __restrict__ slots = a.half_slots;
  const int64_t cap = a.half_cap;
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  const int W = P.seg_w;
  const int64_t li = w - a.half_item_start[k];
  const int row = (int)(li / P.nseg), sg = (int)(li % P.nseg);
  const int y = row % nc1, z = row / nc1;
  const int64_t rowbase = P.cell_off + (int64_t)row * nc0;
  const int c0 = sg * W, c1 = ((sg + 1) * W < nc0 ? (sg + 1) * W : nc0) - 1;
  const int npar = P.npar, par = sg % npar;
  const uint32_t* __restrict__ cs = a.cell_start;

  // clear this item's slots: one window per direction, on the target row
  auto clear = [&](int dix, int64_t cb, int xa, int xb) {
    const uint32_t wb = cs[cb + xa], we = cs[cb + xb + 1];
    float* __restrict__ plane = slots + (int64_t)(npar * dix + par) * cap * V;
    for (uint32_t j = wb + lane; j < we; j += 64) {
#pragma unroll
      for (int v = 0; v < V; ++v) plane[(int64_t)j * V + v] = 0.0f;
    }
  };
  clear(0, rowbase, c0, c1 + P.rx_own > nc0 - 1 ? nc0 - 1 : c1 + P.rx_own);
  {
    int nf = 0;
    for (int f = 0; f < P.n_stencil; ++f) {
      const StencilRow sr = a.st[P.stencil_off + f];
      if (!forward_row(sr)) continue;
      ++nf;
      const int ty = y + sr.dy, tz = z + sr.dz;
      if (ty < 0 || ty >= nc1 || tz < 0 || tz >= nc2) continue;
      clear(nf, P.cell_off + ((int64_t)tz * nc1 + ty) * nc0, c0 - sr.rx < 0 ? 0 : c0 - sr.rx,
            c1 + sr.rx > nc0 - 1 ? nc0 - 1 : c1 + sr.rx);
    }
  }

  // the first NPRE forward rows (target row's first cell relative to the
  // realisation's, reach; cb < 0: outside the grid) and the stencil entry
  // after them, whose ranges are loaded with each tile (the exchange pass,
  // short of registers, takes one row ahead and looks the others up as it
  // goes).
  constexpr int NPRE = EXCH ? 1 : kHalfPreRows;
  int32_t pre_cb[kHalfPreRows];
  int pre_rx[kHalfPreRows];
  int f_pre = 0;
  {
    int nf = 0;
    for (int f = 0; f < P.n_stencil && nf < NPRE; ++f) {
      const StencilRow sr = a.st[P.stencil_off + f];
      if (!forward_row(sr)) continue;
      const int ty = y + sr.dy, tz = z + sr.dz;
      const bool in = ty >= 0 && ty < nc1 && tz >= 0 && tz < nc2;
#pragma unroll
      for (int u = 0; u < NPRE; ++u)
        if (u == nf) {
          pre_cb[u] = in ? (tz * nc1 + ty) * nc0 : -1;
          pre_rx[u] = sr.rx;
        }
      ++nf;
      f_pre = f + 1;
    }
  }
  const uint32_t pb = cs[rowbase + c0], pe = cs[rowbase + c1 + 1];
  const float rc2 = P.rc2_f, esc = P.escale_f;
  // a tile's particles, its cells along x and the end of its own-row range,
  // loaded one tile ahead so that their latency overlaps the previous tile
  struct TileIn {
    float x[DIM], m[SMAX], q;
    int cxa, cxb;
    uint32_t own_je, fjb[kHalfPreRows], fje[kHalfPreRows];
  };
  auto tile_load = [&](uint32_t t0) {
    TileIn d;
    const uint32_t t1 = t0 + 16 < pe ? t0 + 16 : pe;
    const int32_t ii = gi < (int)(t1 - t0) ? (int32_t)t0 + gi : (int32_t)t1 - 1;
    load_pos<float, DIM>(pos, ii, d.x);
    d.q = 0.0f;
#pragma unroll
    for (int v = 0; v < SMAX; ++v) d.m[v] = 0.0f;
    if constexpr (EXCH) {
      d.q = q[ii];
      load_mass<float, SMAX>(min_, ii, d.m);
    }
    d.cxa = (int)(a.skey[t0] - (uint32_t)rowbase);
    d.cxb = (int)(a.skey[t1 - 1] - (uint32_t)rowbase);
    const int xb = d.cxb + P.rx_own > nc0 - 1 ? nc0 - 1 : d.cxb + P.rx_own;
    d.own_je = cs[rowbase + xb + 1];
#pragma unroll
    for (int u = 0; u < NPRE; ++u) {
      d.fjb[u] = 0u;
      d.fje[u] = 0u;
      if (u < P.n_fwd && pre_cb[u] >= 0) {
        const int fa = d.cxa - pre_rx[u] < 0 ? 0 : d.cxa - pre_rx[u];
        const int fb = d.cxb + pre_rx[u] > nc0 - 1 ? nc0 - 1 : d.cxb + pre_rx[u];
        d.fjb[u] = cs[P.cell_off + pre_cb[u] + fa];
        d.fje[u] = cs[P.cell_off + pre_cb[u] + fb + 1];
      }
    }
    return d;
  };
  TileIn tin;
  if (pb < pe) tin = tile_load(pb);
  for (uint32_t t0 = pb; t0 < pe; t0 += 16) {
    const uint32_t t1 = t0 + 16 < pe ? t0 + 16 : pe;
    const int n_in = (int)(t1 - t0);
    const bool valid = gi < n_in;
    const int32_t ii = valid ? (int32_t)t0 + gi : (int32_t)t1 - 1;
    const TileIn cur_tile = tin;
    if (t1 < pe) tin = tile_load(t1);
    float xi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) xi[k] = cur_tile.x[k];
    // a lane past the tile's end: its separations overflow to +inf, weight 0
    if (!valid) xi[0] = -3.0e38f;
    const float qi = cur_tile.q;
    float Mi[SMAX];
#pragma unroll
    for (int v = 0; v < SMAX; ++v) Mi[v] = cur_tile.m[v];
    const int cxa = cur_tile.cxa, cxb = cur_tile.cxb;
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;

    // pairs inside the tile, from both ends: row g takes the rotations
    // 4g .. 4g + 3 of the tile's particles (all 16 over the four rows; the
    // rotation 0 is the particle itself, weight 1).  Evaluated once the first
    // chunk's loads are in flight, and added first.
    auto self_tile = [&]() {
      float part[V];
#pragma unroll
      for (int v = 0; v < V; ++v) part[v] = 0.0f;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int src = (lane & 48) | ((gi + 4 * gl + kk) & 15);
        float s2 = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const float dk = __shfl(xi[k], src) - xi[k];
          s2 = k == 0 ? dk * dk : __builtin_fmaf(dk, dk, s2);
        }
        float wgt = kweight(s2, esc);
        wgt = s2 <= rc2 ? wgt : 0.0f;
        if constexpr (EXCH) {
          const float pp = SYM ? wgt * (__shfl(qi, src) + qi) : wgt;
#pragma unroll
          for (int v = 0; v < SMAX; ++v) part[v] += pp * (__shfl(Mi[v], src) - Mi[v]);
        } else {
          part[0] += wgt;
        }
      }
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] += (double)part[v];
    };

    // forward candidates, 64 per chunk, the next chunk's loads issued before
    // the current chunk is computed
    struct Cand {
      float x[DIM], m[SMAX], q;
      float sl[V];  // the candidate's slot, read ahead (no other chunk of this tile touches it)
      int32_t j;
      int dix;
      bool has;
    };
    auto load = [&](int32_t j, bool has, int dix) {
      Cand d;
      {
        const float* __restrict__ sp = slots + ((int64_t)(npar * dix + par) * cap + (has ? j : 0)) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) d.sl[v] = has ? sp[v] : 0.0f;
      }
      load_pos<float, DIM>(pos, j, d.x);
      if (!has) d.x[0] = 3.0e38f;  // a dummy candidate: separation +inf, weight 0
      if constexpr (EXCH) {
        d.q = q[j];
        load_mass<float, SMAX>(min_, j, d.m);
      } else {
        d.q = 0.0f;
#pragma unroll
        for (int v = 0; v < SMAX; ++v) d.m[v] = 0.0f;
      }
      d.j = j;
      d.dix = dix;
      d.has = has;
      return d;
    };
    auto compute = [&](const Cand& d) {
      float ai[V], aj[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        ai[v] = 0.0f;
        aj[v] = 0.0f;
      }
      // every DPP operand below is read with all lanes active; no
      // contraction, so that the rotations fold into the adds and subtracts
      Steps<0, 16>::run([&](auto kc) {
#pragma clang fp contract(off)
        constexpr int K = decltype(kc)::value;
        float s2 = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const float dk = rror<K>(d.x[k]) - xi[k];
          s2 = k == 0 ? dk * dk : __builtin_fmaf(dk, dk, s2);
        }
        float wgt = kweight(s2, esc);
        wgt = s2 <= rc2 ? wgt : 0.0f;
        if constexpr (EXCH) {
          const float pp = SYM ? wgt * (rror<K>(d.q) + qi) : wgt;
#pragma unroll
          for (int v = 0; v < SMAX; ++v) {
            const float t = pp * (rror<K>(d.m[v]) - Mi[v]);
            ai[v] += t;
            aj[v] = (K == 0 ? -t : rror<1>(aj[v]) - t);
          }
        } else {
          ai[0] += wgt;
          aj[0] = (K == 0 ? wgt : rror<1>(aj[0]) + wgt);
        }
      });
#pragma unroll
      for (int v = 0; v < V; ++v) {
        acc[v] += (double)ai[v];
        aj[v] = rror<1>(aj[v]);  // the sum of this lane's own candidate
      }
      if (d.has) {
        float* __restrict__ sl = slots + ((int64_t)(npar * d.dix + par) * cap + d.j) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) sl[v] = d.sl[v] + aj[v];
      }
    };
    HalfCursor c;
    c.own_je = cur_tile.own_je;
#pragma unroll
    for (int u = 0; u < NPRE; ++u) {
      c.fjb[u] = cur_tile.fjb[u];
      c.fje[u] = cur_tile.fje[u];
    }
    c.k = -1;
    c.f = f_pre;
    c.p = 0;
    half_advance<NPRE>(c, P, a.st, cs, y, z, rowbase, cxa, cxb, t1);
    if (c.valid) {
      uint32_t vbase = 0;
      int32_t j;
      bool has;
      int dix;
      half_pick<NPRE>(c, P, a.st, cs, y, z, rowbase, cxa, cxb, t1, vbase, (int32_t)t0, j, has, dix);
      Cand cur = load(j, has, dix);
      self_tile();
      while (true) {
        const bool next = c.valid;
        Cand nxt = cur;
        if (next) {
          vbase += 64;
          half_pick<NPRE>(c, P, a.st, cs, y, z, rowbase, cxa, cxb, t1, vbase, (int32_t)t0, j, has, dix);
          nxt = load(j, has, dix);
        }
        compute(cur);
        if (!next) break;
        cur = nxt;
      }
    } else {
      self_tile();
    }
    // the particle's own sums over the four rows
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[v] += __shfl_xor(acc[v], 16);
      acc[v] += __shfl_xor(acc[v], 32);
    }
    if (gl == 0 && valid) {
#pragma unroll
      for (int v = 0; v < V; ++v) a.half_own[(int64_t)ii * V + v] = acc[v];
    }
  }
}

// Sum of particle i's slots of V values: for each direction in order (own row
// first, then the forward stencil rows whose source row exists) the segments
// of the source row whose windows reach i's cell (at most npar), ascending.
template <int V>
__device__ __forceinline__ void half_gather(const PairArgs& a, const RealParams& P, int32_t i, double (&acc)[V]) {
  const uint32_t lk = a.skey[i] - (uint32_t)P.cell_off;
  const int nc0 = P.nc[0], nc1 = P.nc[1], nc2 = P.nc[2];
  const int cx = (int)(lk % (uint32_t)nc0);
  const int rowi = (int)(lk / (uint32_t)nc0);
  const int y = rowi % nc1, z = rowi / nc1;
  const int W = P.seg_w, nseg = P.nseg, npar = P.npar;
  const float* __restrict__ slots = a.half_slots;
  const int64_t cap = a.half_cap;
  auto add = [&](int dix, int rx, bool own) {
    int slo = floordiv(cx - rx, W), shi = own ? cx / W : floordiv(cx + rx, W);
    slo = slo < 0 ? 0 : slo;
    shi = shi > nseg - 1 ? nseg - 1 : shi;
    for (int sg = slo; sg <= shi; ++sg) {
      const float* __restrict__ sl = slots + ((int64_t)(npar * dix + sg % npar) * cap + i) * V;
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] += (double)sl[v];
    }
  };
  add(0, P.rx_own, true);
  int nf = 0;
  for (int f = 0; f < P.n_stencil; ++f) {
    const StencilRow sr = a.st[P.stencil_off + f];
    if (!forward_row(sr)) continue;
    ++nf;
    const int sy = y - sr.dy, sz = z - sr.dz;
    if (sy < 0 || sy >= nc1 || sz < 0 || sz >= nc2) continue;
    add(nf, sr.rx, false);
  }
}

// Row sums of the half-stencil tiling: r_i = own sum + slots; q_i = 1 / r_i.
__global__ __launch_bounds__(kBlock) void k_half_rowsum_fin(PairArgs a) {
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(a.tiles, a.ntiles, tl, tile)) return;
  if (!tl.valid) return;
  const RealParams& P = a.rp[tile.real];
  double r[1] = {1.0};
  if (P.active && P.nseg > 0) {
    r[0] = a.half_own[tl.i];
    half_gather<1>(a, P, tl.i, r);
  }
  if (a.r_out) a.r_out[tl.i] = r[0];
  ((float*)a.q_out)[tl.i] = (float)(1.0 / r[0]);
}

// Exchange of the half-stencil tiling: the particle's sums of t over its
// neighbours (own sums + slots), then the explicit update, the reaction and
// the audit partials of the one-lane-per-particle tiles.
template <int SMAX>
__global__ __launch_bounds__(kBlock) void k_half_exchange_fin(PairArgs a) {
  TileLane tl;
  Tile tile;
  if (!tile_lane_setup<0>(a.tiles, a.ntiles, tl, tile)) return;
  const RealParams& P = a.rp[tile.real];
  const int32_t ii = tl.valid ? tl.i : tile.end - 1;
  float Mi[SMAX];
  load_mass<float, SMAX>((const float*)a.mass_in, ii, Mi);
  double acc[SMAX];
#pragma unroll
  for (int v = 0; v < SMAX; ++v) acc[v] = 0.0;
  double racc = 1.0;
  if (tl.valid && P.active && P.nseg > 0) {
#pragma unroll
    for (int v = 0; v < SMAX; ++v) acc[v] = a.half_own[(int64_t)ii * SMAX + v];
    half_gather<SMAX>(a, P, ii, acc);
    racc = a.norm == 0 ? 1.0 : a.r_out[ii];  // only the row normalisation divides by r_i
  }
  exchange_epilogue<float, SMAX, 64>(P, a.norm == 0, acc, racc, Mi, tl.valid, tl.i, (float*)a.mass_out, a.S,
                                     a.react_a, a.react_b, a.audit_part, wave_tile());
}

// ---------------------------------------------------------------------------
// Allocation-free transfer of one realisation held in caller arrays: set-up
// kernels that write the step's parameters, stencil, tiles and cleared cell
// counts from kernel arguments, convert the caller's layouts, and return the
// new masses in the caller's order.
// ---------------------------------------------------------------------------

// Parameters and stencil rows (one block): kernel arguments -> device memory.
__global__ __launch_bounds__(kBlock) void k_na_params(NoAllocParams a, RealParams* __restrict__ rp,
                                                      StencilRow* __restrict__ st, int64_t* __restrict__ real_start) {
  if (threadIdx.x == 0) {
    rp[0] = a.P;
    real_start[0] = a.P.p_begin;
    real_start[1] = a.P.p_end;
  }
  if ((int)threadIdx.x < a.n_st) st[threadIdx.x] = a.st[threadIdx.x];
}

// Grid-stride: ids 0..n-1, positions (n x DIM row-major) and masses (S x n
// species-major) into the particle-major layouts (unused species slots zero),
// tiles of G consecutive particles, the walk's per-block realisation table
// (all zero: one realisation) and cleared cell counts.
template <typename T, int DIM, int SP>
__global__ __launch_bounds__(kBlock) void k_na_load(int32_t n, int32_t S, const T* __restrict__ pos,
                                                    const T* __restrict__ mass, T* __restrict__ pos_out,
                                                    T* __restrict__ mass_out, uint32_t* __restrict__ id,
                                                    Tile* __restrict__ tiles, int32_t G, int32_t ntiles,
                                                    int32_t* __restrict__ blk_real, int32_t nblk,
                                                    uint32_t* __restrict__ cell_count, int64_t ncell) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t top = ncell > n ? ncell : n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < top; i += stride) {
    if (i < n) {
      id[i] = (uint32_t)i;
      T x[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) x[k] = pos[i * DIM + k];
      store_pos<T, DIM>(pos_out, i, x);
      T m[SP];
#pragma unroll
      for (int sp = 0; sp < SP; ++sp) m[sp] = sp < S ? mass[(int64_t)sp * n + i] : (T)0;
      store_mass<T, SP>(mass_out, i, m);
    }
    if (i < ntiles) {
      const int32_t b = (int32_t)i * G;
      tiles[i] = Tile{b, b + G < n ? b + G : n, 0, 0};
    }
    if (i < nblk) blk_real[i] = 0;
    if (i < ncell) cell_count[i] = 0u;
  }
}

// Sorted particle p's new masses to the caller's order (S x n species-major).
template <typename T, int SP>
__global__ __launch_bounds__(kBlock) void k_na_store(int32_t n, int32_t S, const T* __restrict__ mass_sorted,
                                                     const uint32_t* __restrict__ id, T* __restrict__ mass) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  T m[SP];
  load_mass<T, SP>(mass_sorted, p, m);
  const uint32_t o = id[p];
#pragma unroll
  for (int sp = 0; sp < SP; ++sp)
    if (sp < S) mass[(int64_t)sp * n + o] = m[sp];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
static inline unsigned canon_blocks_for(int64_t n) {
  return (unsigned)((n + kCanonItems * kBlock - 1) / (kCanonItems * kBlock));
}

hipError_t launch_walk_key(int fp64, int dim, const void* pos_in, void* pos_out,
                           const uint32_t* id, int32_t n, const RealParams* rp,
                           const int64_t* real_start, const int32_t* blk_real, int32_t n_real,
                           const uint64_t* step_ctr, uint64_t seed, int32_t do_walk, uint32_t* cell_count,
                           uint32_t* key, uint32_t* slot, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g(blocks_for(n)), b(kBlock);
#define RWPT_WK(T, D)                                                                             \
  hipLaunchKernelGGL((k_walk_key<T, D>), g, b, 0, s, (const T*)pos_in, (T*)pos_out, id, n, rp, \
                     real_start, blk_real, n_real, step_ctr, seed, do_walk, cell_count, key, slot)
  if (fp64) {
    if (dim == 1) RWPT_WK(double, 1);
    else if (dim == 2) RWPT_WK(double, 2);
    else RWPT_WK(double, 3);
  } else {
    if (dim == 1) RWPT_WK(float, 1);
    else if (dim == 2) RWPT_WK(float, 2);
    else RWPT_WK(float, 3);
  }
#undef RWPT_WK
  return hipGetLastError();
}

hipError_t launch_cell_scan(uint32_t* cell_count, uint32_t* cell_start, int64_t ncell,
                            uint32_t* partials, hipStream_t s) {
  const int64_t nb = (ncell + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, cell_count, ncell, partials);
  if (nb <= kScanDirectMax) {
    // each block sums the block partials before it, at most one per thread
    hipLaunchKernelGGL(k_scan_final<true>, dim3((unsigned)nb), dim3(kBlock), 0, s, cell_count, ncell, partials,
                       cell_start);
  } else {
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, partials, (int32_t)nb, cell_start, ncell);
    hipLaunchKernelGGL(k_scan_final<false>, dim3((unsigned)nb), dim3(kBlock), 0, s, cell_count, ncell, partials,
                       cell_start);
  }
  return hipGetLastError();
}

hipError_t launch_scatter(int32_t n, const uint32_t* key, const uint32_t* slot,
                          const uint32_t* cell_start, const uint32_t* id, uint32_t* tmp_src,
                          uint32_t* tmp_id, uint32_t* tmp_key, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, key, slot, cell_start, id,
                     tmp_src, tmp_id, tmp_key);
  return hipGetLastError();
}

hipError_t launch_canon(int fp64, int dim, int32_t n, const uint32_t* tmp_src,
                        const uint32_t* tmp_id, const uint32_t* tmp_key,
                        const uint32_t* cell_start, const void* pos_in, void* pos_out,
                        const void* mass_in, void* mass_out, int32_t S,
                        uint32_t* id_out, uint32_t* skey, uint32_t* src_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g(canon_blocks_for(n)), b(kBlock);
#define RWPT_CN(T, D)                                                                           \
  do {                                                                                          \
    if (S <= 2) RWPT_CN1(T, D, 2);                                                              \
    else if (S <= 4) RWPT_CN1(T, D, 4);                                                         \
    else RWPT_CN1(T, D, 8);                                                                     \
  } while (0)
#define RWPT_CN1(T, D, SM)                                                                      \
  do {                                                                                          \
    if (src_out)                                                                                \
      hipLaunchKernelGGL((k_canon<T, D, SM, false>), g, b, 0, s, n, tmp_src, tmp_id, tmp_key,     \
                         cell_start, (const T*)pos_in, (T*)pos_out, (const T*)mass_in,          \
                         (T*)mass_out, id_out, skey, src_out);                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_canon<T, D, SM, true>), g, b, 0, s, n, tmp_src, tmp_id, tmp_key,      \
                         cell_start, (const T*)pos_in, (T*)pos_out, (const T*)mass_in,          \
                         (T*)mass_out, id_out, skey, src_out);                               \
  } while (0)
  if (fp64) {
    if (dim == 1) RWPT_CN(double, 1);
    else if (dim == 2) RWPT_CN(double, 2);
    else RWPT_CN(double, 3);
  } else {
    if (dim == 1) RWPT_CN(float, 1);
    else if (dim == 2) RWPT_CN(float, 2);
    else RWPT_CN(float, 3);
  }
#undef RWPT_CN1
#undef RWPT_CN
  return hipGetLastError();
}

// Up to this many tiles, the row-broadcast kernels give each tile a whole
// block (its four waves take every fourth chunk of the candidates), so that a
// small ensemble still puts enough waves on the 1024 SIMDs to hide latency.
constexpr int32_t kSplitTiles = 4096;

static inline dim3 pair_grid(int32_t ntiles) {
  return dim3((unsigned)((ntiles + (kBlock / 64) - 1) / (kBlock / 64)));
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(T{}, IC<dim>{}, IC<log2l>{}) for the supported instantiations.
template <typename F>
static hipError_t dispatch_tdl(int fp64, int dim, int log2l, F&& f) {
  auto with_l = [&](auto t, auto d) -> hipError_t {
    switch (log2l) {
      case 0: f(t, d, IC<0>{}); break;
      case 2: f(t, d, IC<2>{}); break;
      case 3: f(t, d, IC<3>{}); break;
      case 4: f(t, d, IC<4>{}); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  auto with_d = [&](auto t) -> hipError_t {
    switch (dim) {
      case 1: return with_l(t, IC<1>{});
      case 2: return with_l(t, IC<2>{});
      case 3: return with_l(t, IC<3>{});
      default: return hipErrorInvalidValue;
    }
  };
  return fp64 ? with_d(double{}) : with_d(float{});
}

static hipError_t launch_half(int dim, bool exch, const PairArgs& a, hipStream_t s) {
  if (a.half_nitems > 0) {
    const dim3 g((unsigned)((a.half_nitems + kBlock / 64 - 1) / (kBlock / 64))), b(kBlock);
    auto go = [&](auto d, auto sm) {
      constexpr int D = decltype(d)::value, SM = decltype(sm)::value;
      if (!exch) hipLaunchKernelGGL((k_half_pairs<D, SM, false, true>), g, b, 0, s, a);
      else if (a.norm == 0) hipLaunchKernelGGL((k_half_pairs<D, SM, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_half_pairs<D, SM, true, false>), g, b, 0, s, a);
    };
    auto go_s = [&](auto d) {
      if (!exch || a.S <= 2) go(d, IC<2>{});
      else if (a.S <= 4) go(d, IC<4>{});
      else go(d, IC<8>{});
    };
    if (dim == 1) go_s(IC<1>{});
    else if (dim == 2) go_s(IC<2>{});
    else if (dim == 3) go_s(IC<3>{});
    else return hipErrorInvalidValue;
  }
  const dim3 g = pair_grid(a.ntiles), b(kBlock);
  if (!exch) {
    hipLaunchKernelGGL(k_half_rowsum_fin, g, b, 0, s, a);
  } else if (a.S <= 2) {
    hipLaunchKernelGGL(k_half_exchange_fin<2>, g, b, 0, s, a);
  } else if (a.S <= 4) {
    hipLaunchKernelGGL(k_half_exchange_fin<4>, g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL(k_half_exchange_fin<8>, g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_rowsum(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (log2l == kHalfPairs) return fp64 ? hipErrorInvalidValue : launch_half(dim, false, a, s);
  const dim3 g = pair_grid(a.ntiles), b(kBlock);
  if (log2l == kPrivateLists) {
    return dispatch_tdl(fp64, dim, 0, [&](auto t, auto d, auto) {
      using T = decltype(t);
      constexpr int D = decltype(d)::value;
#define RWPT_RSP_ARGS                                                                                 \
  (const T*)a.pos, a.cell_start, a.tiles, a.ntiles, a.rp, a.r_out, (T*)a.q_out, a.nb_meta, a.nb_idx, \
      (T*)a.nb_w, a.nb_src, a.src_of
      if (a.indirect) hipLaunchKernelGGL((k_rowsum_priv<T, D, true>), g, b, 0, s, RWPT_RSP_ARGS);
      else hipLaunchKernelGGL((k_rowsum_priv<T, D, false>), g, b, 0, s, RWPT_RSP_ARGS);
#undef RWPT_RSP_ARGS
    });
  }
  if (!fp64 && log2l == 2) {
    const bool split = a.ntiles <= kSplitTiles;
    const dim3 gs = split ? dim3((unsigned)a.ntiles) : g;
    auto go = [&](auto d) {
      constexpr int D = decltype(d)::value;
#define RWPT_RSD_ARGS \
  (const float*)a.pos, a.skey, a.cell_start, a.tiles, a.ntiles, a.rp, a.st, a.r_out, (float*)a.q_out
      if (split) hipLaunchKernelGGL((k_rowsum_dpp<D, kBlock / 64>), gs, b, 0, s, RWPT_RSD_ARGS);
      else hipLaunchKernelGGL((k_rowsum_dpp<D, 1>), gs, b, 0, s, RWPT_RSD_ARGS);
#undef RWPT_RSD_ARGS
    };
    if (dim == 1) go(IC<1>{});
    else if (dim == 2) go(IC<2>{});
    else if (dim == 3) go(IC<3>{});
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  return dispatch_tdl(fp64, dim, log2l, [&](auto t, auto d, auto l) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_rowsum<T, decltype(d)::value, decltype(l)::value>), g, b, 0, s, (const T*)a.pos,
                       a.skey, a.cell_start, a.tiles, a.ntiles, a.rp, a.st, a.r_out, (T*)a.q_out);
  });
}

hipError_t launch_exchange(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (a.S < 1 || a.S > 8) return hipErrorInvalidValue;
  if (log2l == kHalfPairs) return fp64 ? hipErrorInvalidValue : launch_half(dim, true, a, s);
  const dim3 g = pair_grid(a.ntiles), b(kBlock);
  if (log2l == kPrivateLists) {
    return dispatch_tdl(fp64, dim, 0, [&](auto t, auto d, auto) {
      using T = decltype(t);
      constexpr int D = decltype(d)::value;
#define RWPT_EXP_ARGS                                                                                  \
  (const T*)a.pos, (const T*)a.mass_in, (T*)a.mass_out, (const T*)a.q_in, a.r_out, a.skey,        \
      a.cell_start, a.tiles, a.ntiles, a.rp, a.st, a.S, a.react_a, a.react_b, a.norm, a.audit_part,      \
      a.nb_meta, a.nb_idx, (const T*)a.nb_w, a.nb_src, a.src_of
      auto go = [&](auto sm, auto ind) {
        hipLaunchKernelGGL((k_exchange_priv<T, D, decltype(sm)::value, decltype(ind)::value>), g, b, 0, s,
                           RWPT_EXP_ARGS);
      };
      auto go_s = [&](auto ind) {
        if (a.S <= 2) go(IC<2>{}, ind);
        else if (a.S <= 4) go(IC<4>{}, ind);
        else go(IC<8>{}, ind);
      };
      if (a.indirect) go_s(std::true_type{});
      else go_s(std::false_type{});
#undef RWPT_EXP_ARGS
    });
  }
  if (!fp64 && log2l == 2) {
    const bool split = a.ntiles <= kSplitTiles;
    const dim3 gs = split ? dim3((unsigned)a.ntiles) : g;
    auto go = [&](auto d) {
      constexpr int D = decltype(d)::value;
#define RWPT_EXD_ARGS                                                                                  \
  (const float*)a.pos, (const float*)a.mass_in, (float*)a.mass_out, (const float*)a.q_in, a.skey, \
      a.cell_start, a.tiles, a.ntiles, a.rp, a.st, a.S, a.react_a, a.react_b, a.norm, a.audit_part
      auto go_s = [&](auto sm) {
        constexpr int SM = decltype(sm)::value;
        if (split) hipLaunchKernelGGL((k_exchange_dpp<D, SM, kBlock / 64>), gs, b, 0, s, RWPT_EXD_ARGS);
        else hipLaunchKernelGGL((k_exchange_dpp<D, SM, 1>), gs, b, 0, s, RWPT_EXD_ARGS);
      };
      if (a.S <= 2) go_s(IC<2>{});
      else if (a.S <= 4) go_s(IC<4>{});
      else go_s(IC<8>{});
#undef RWPT_EXD_ARGS
    };
    if (dim == 1) go(IC<1>{});
    else if (dim == 2) go(IC<2>{});
    else if (dim == 3) go(IC<3>{});
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  return dispatch_tdl(fp64, dim, log2l, [&](auto t, auto d, auto l) {
    using T = decltype(t);
    constexpr int D = decltype(d)::value, L = decltype(l)::value;
#define RWPT_EX_ARGS                                                                          \
  (const T*)a.pos, (const T*)a.mass_in, (T*)a.mass_out, (const T*)a.q_in, a.skey, a.cell_start, \
      a.tiles, a.ntiles, a.rp, a.st, a.S, a.react_a, a.react_b, a.norm, a.audit_part
    if (a.S <= 2) hipLaunchKernelGGL((k_exchange<T, D, 2, L>), g, b, 0, s, RWPT_EX_ARGS);
    else if (a.S <= 4) hipLaunchKernelGGL((k_exchange<T, D, 4, L>), g, b, 0, s, RWPT_EX_ARGS);
    else hipLaunchKernelGGL((k_exchange<T, D, 8, L>), g, b, 0, s, RWPT_EX_ARGS);
#undef RWPT_EX_ARGS
  });
}

// The row-broadcast export/count kernels in the launch shape of the binary32
// four-lane pair kernels (one block per tile up to kSplitTiles tiles).
template <int MODE>
static hipError_t launch_nbr_dpp(int dim, const PairArgs& a, hipStream_t s) {
  const bool split = a.ntiles <= kSplitTiles;
  const dim3 g = split ? dim3((unsigned)a.ntiles) : pair_grid(a.ntiles), b(kBlock);
  auto go = [&](auto d) {
    constexpr int D = decltype(d)::value;
    if (split) hipLaunchKernelGGL((k_nbr_dpp<D, kBlock / 64, MODE>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_nbr_dpp<D, 1, MODE>), g, b, 0, s, a);
  };
  if (dim == 1) go(IC<1>{});
  else if (dim == 2) go(IC<2>{});
  else if (dim == 3) go(IC<3>{});
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_count(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (log2l == kHalfPairs) log2l = 0;  // same tiles of 64 particles
  const dim3 g = pair_grid(a.ntiles), b(kBlock);
  if (log2l == kPrivateLists) {  // same tiles of 64, one lane per particle
    return dispatch_tdl(fp64, dim, 0, [&](auto t, auto d, auto) {
      hipLaunchKernelGGL((k_count_priv<decltype(t), decltype(d)::value>), g, b, 0, s, a);
    });
  }
  if (!fp64 && log2l == 2) return launch_nbr_dpp<2>(dim, a, s);
  return dispatch_tdl(fp64, dim, log2l, [&](auto t, auto d, auto l) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_count<T, decltype(d)::value, decltype(l)::value>), g, b, 0, s, a);
  });
}

// The neighbour export enumerates the candidates exactly as the tiling the
// step launches: the row-broadcast chunks (binary32, four lanes), the own
// cutoff-box walk of the row-sum pass (one lane per particle), or the
// stencil rows of the vector-load tiles.
template <bool FILL>
static hipError_t launch_nbr(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (log2l == kHalfPairs) log2l = 0;  // same tiles of 64 particles
  const dim3 g = pair_grid(a.ntiles), b(kBlock);
  if (log2l == kPrivateLists) {
    return dispatch_tdl(fp64, dim, 0, [&](auto t, auto d, auto) {
      hipLaunchKernelGGL((k_nbr_priv<decltype(t), decltype(d)::value, FILL>), g, b, 0, s, a);
    });
  }
  if (!fp64 && log2l == 2) return launch_nbr_dpp<FILL ? 1 : 0>(dim, a, s);
  return dispatch_tdl(fp64, dim, log2l, [&](auto t, auto d, auto l) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_nbr<T, decltype(d)::value, decltype(l)::value, FILL>), g, b, 0, s, a);
  });
}

hipError_t launch_nbr_count(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  return launch_nbr<false>(fp64, dim, log2l, a, s);
}

hipError_t launch_nbr_fill(int fp64, int dim, int log2l, const PairArgs& a, hipStream_t s) {
  return launch_nbr<true>(fp64, dim, log2l, a, s);
}

hipError_t launch_noalloc_setup(int fp64, int dim, int S, const NoAllocParams& a, int32_t n, const void* pos,
                                const void* mass, void* pos_out, void* mass_out, uint32_t* id, Tile* tiles,
                                int32_t G, int32_t ntiles, RealParams* rp, StencilRow* st, int64_t* real_start,
                                int32_t* blk_real, uint32_t* cell_count, int64_t ncell, hipStream_t s) {
  if (a.n_st < 0 || a.n_st > kNoAllocStencil) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_na_params, dim3(1), dim3(kBlock), 0, s, a, rp, st, real_start);
  const int32_t nblk = (int32_t)blocks_for(n);
  const int64_t top = std::max<int64_t>(ncell, n);
  const unsigned g = (unsigned)std::min<int64_t>((top + kBlock - 1) / kBlock, 2048);
  auto go = [&](auto t, auto d, auto sp) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_na_load<T, decltype(d)::value, decltype(sp)::value>), dim3(g), dim3(kBlock), 0, s, n, S,
                       (const T*)pos, (const T*)mass, (T*)pos_out, (T*)mass_out, id, tiles, G, ntiles, blk_real,
                       nblk, cell_count, ncell);
  };
  auto with_s = [&](auto t, auto d) {
    if (S <= 2) go(t, d, IC<2>{});
    else if (S <= 4) go(t, d, IC<4>{});
    else go(t, d, IC<8>{});
  };
  auto with_d = [&](auto t) {
    if (dim == 1) with_s(t, IC<1>{});
    else if (dim == 2) with_s(t, IC<2>{});
    else with_s(t, IC<3>{});
  };
  if (fp64) with_d(double{});
  else with_d(float{});
  return hipGetLastError();
}

hipError_t launch_noalloc_store(int fp64, int S, int32_t n, const void* mass_sorted, const uint32_t* id,
                                void* mass, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  auto go = [&](auto t, auto sp) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_na_store<T, decltype(sp)::value>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, S,
                       (const T*)mass_sorted, id, (T*)mass);
  };
  auto with_s = [&](auto t) {
    if (S <= 2) go(t, IC<2>{});
    else if (S <= 4) go(t, IC<4>{});
    else go(t, IC<8>{});
  };
  if (fp64) with_s(double{});
  else with_s(float{});
  return hipGetLastError();
}

hipError_t launch_audit_reduce(const double* part, int32_t S1, const AuditChunk* chunks, int32_t nchunks,
                               double* chunk_part, const int32_t* chunk_start, int32_t n_real,
                               double* out, uint32_t* done, uint64_t* step_ctr, int32_t bump,
                               hipStream_t s) {
  if (n_real <= 0 || nchunks <= 0) return hipSuccess;
  if (S1 < 1 || S1 > kAuditValues) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_audit, dim3((unsigned)nchunks), dim3(kBlock), 0, s, part, S1, chunks, chunk_part,
                     chunk_start, out, done, step_ctr, bump);
  return hipGetLastError();
}

}  // namespace rwpt
