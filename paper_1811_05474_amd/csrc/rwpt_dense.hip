// rwpt_dense.hip -- full-matrix ("brute force", Sec. 1.1) mass transfer of
// one realisation on the matrix cores of gfx950.
//
// Pass 1 (VALU): r_i = sum_j w_ij over all j, q_i = 1 / r_i.
// Pass 2 (MFMA): with the symmetric normalisation
//   4 dM_i = sum_j w_ij (q_i + q_j)(M_j - M_i)
//          = q_i (W M)_i + (W (q M))_i - M_i (q_i (W 1)_i + (W q)_i),
// so one contraction C = W B with the columns B = [M_s, q M_s, q, 1] gives
// every species at once (row normalisation: 2 dM_i = (W M)_i / (W 1)_i - M_i).
// W tiles (16 rows x 32 columns) are generated on the VALU from the
// positions, split into three bf16 parts (w = w0 + w1 + w2 to about 24 bits),
// and multiplied with the three-part bf16 split of B by
// v_mfma_f32_16x16x32_bf16; the six products above 2^-24 of the leading
// term are kept.  Each tile's fp32 result is added into fp64 accumulators.
//
// Column tiles whose bounding box lies so far from the row tile's box that
// every weight is below 2^-40 are skipped; they change r_i by less than
// N 2^-40, far below binary32 rounding.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "rwpt_kernels.h"
#include "rwpt_layout.h"

namespace rwpt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kColTile = 32;   // columns (j) per MFMA K-step and per bounding box
constexpr int kRowTile = 16;   // rows (i) per block in the exchange pass
constexpr int kRowTileSum = 64;  // rows per block in the row-sum pass
// Waves that share one row tile, each taking every kSumWaves-th (kExWaves-th)
// near column tile, so that a 32768-particle matrix gives 8 waves per SIMD
// instead of one or two; their partial sums are added in wave order.
constexpr int kSumWaves = 16;  // row-sum pass: one block of 1024 threads per 64-row tile
constexpr int kExWaves = 4;    // exchange pass: one block of 256 threads per 16-row tile

__device__ __forceinline__ float bf16_to_f32(__bf16 v) { return (float)v; }

// w = p0 + p1 + p2 with each part a bf16 (residuals are exact in binary32).
__device__ __forceinline__ void split3(float w, __bf16& p0, __bf16& p1, __bf16& p2) {
  p0 = (__bf16)w;
  const float r1 = w - bf16_to_f32(p0);
  p1 = (__bf16)r1;
  const float r2 = r1 - bf16_to_f32(p1);
  p2 = (__bf16)r2;
}

template <int DIM>
__device__ __forceinline__ float sep2f(const float xi[DIM], const float xj[DIM]) {
#pragma clang fp contract(off)
  const float d0 = xj[0] - xi[0];
  float s = d0 * d0;
  if constexpr (DIM > 1) {
    const float d1 = xj[1] - xi[1];
    s = __builtin_fmaf(d1, d1, s);
  }
  if constexpr (DIM > 2) {
    const float d2 = xj[2] - xi[2];
    s = __builtin_fmaf(d2, d2, s);
  }
  return s;
}

// Squared distance between two axis-aligned boxes [lo, hi] (0 if they overlap).
template <int DIM>
__device__ __forceinline__ float box_dist2(const float* a, const float* b) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const float g = fmaxf(fmaxf(b[2 * k] - a[2 * k + 1], a[2 * k] - b[2 * k + 1]), 0.0f);
    s += g * g;
  }
  return s;
}

// Bounding box (min, max per axis) of every column tile of kColTile particles.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_tile_bbox(const float* __restrict__ pos, int32_t n,
                                                      float* __restrict__ bbox) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int j0 = t * kColTile;
  if (j0 >= n) return;
  const int j1 = j0 + kColTile < n ? j0 + kColTile : n;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    float lo = INFINITY, hi = -INFINITY;
    for (int j = j0; j < j1; ++j) {
      const float v = pos[pos_stride<DIM>() * j + k];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
    bbox[(int64_t)t * 2 * DIM + 2 * k] = lo;
    bbox[(int64_t)t * 2 * DIM + 2 * k + 1] = hi;
  }
}

// Walk the column tiles that may hold a weight >= 2^-40 for the row box:
// the wave tests 64 tiles at a time and visits the hits in order.
template <int DIM, typename Fn>
__device__ __forceinline__ void for_near_tiles(const float* __restrict__ bbox, int32_t ntile,
                                               const float rbox[2 * DIM], float skip_s2, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  for (int cb = 0; cb < ntile; cb += 64) {
    const int ct = cb + lane;
    bool near = false;
    if (ct < ntile) near = box_dist2<DIM>(rbox, bbox + (int64_t)ct * 2 * DIM) <= skip_s2;
    unsigned long long m = __ballot(near);
    while (m) {
      const int t = cb + __ffsll(m) - 1;
      m &= m - 1;
      fn(t);
    }
  }
}

template <int DIM>
__device__ __forceinline__ void load_box(const float* __restrict__ bbox, int t, float out[2 * DIM]) {
#pragma unroll
  for (int k = 0; k < 2 * DIM; ++k) out[k] = bbox[(int64_t)t * 2 * DIM + k];
}

// Pass 1: one lane per row, column tiles broadcast through scalar loads; the
// kSumWaves waves of a block share the block's 64 rows, wave w taking the
// near column tiles t = w mod kSumWaves.
template <int DIM>
__global__ __launch_bounds__(64 * kSumWaves) void k_dense_rowsum(const float* __restrict__ pos, const int32_t n, const float* __restrict__ bbox,
                                                         const int32_t ntile, const float escale,
                                                         const float skip_s2, double* __restrict__ r_out,
                                                         float* __restrict__ q_out) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rt = blockIdx.x;
  const int i0 = rt * kRowTileSum;  // < n: one block per row tile
  const int i = i0 + lane;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  float xi[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) xi[k] = pos[pos_stride<DIM>() * ii + k];
  // row box: union of the (up to) two column-tile boxes covering the rows
  float rbox[2 * DIM];
  load_box<DIM>(bbox, i0 / kColTile, rbox);
  const int t2 = i0 / kColTile + 1;
  if (t2 < ntile && t2 * kColTile < i0 + kRowTileSum) {
    float b2[2 * DIM];
    load_box<DIM>(bbox, t2, b2);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      rbox[2 * k] = fminf(rbox[2 * k], b2[2 * k]);
      rbox[2 * k + 1] = fmaxf(rbox[2 * k + 1], b2[2 * k + 1]);
    }
  }
  double acc = 0.0;
  for_near_tiles<DIM>(bbox, ntile, rbox, skip_s2, [&](int t) {
    if (t % kSumWaves != wave) return;  // another wave's tile
    const int j0 = t * kColTile;
    float a = 0.0f;
    if (j0 + kColTile <= n) {
#pragma unroll 8
      for (int u = 0; u < kColTile; ++u) {
        float xj[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xj[k] = pos[pos_stride<DIM>() * (j0 + u) + k];
        a += __builtin_amdgcn_exp2f(sep2f<DIM>(xi, xj) * escale);
      }
    } else {
      for (int j = j0; j < n; ++j) {
        float xj[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xj[k] = pos[pos_stride<DIM>() * j + k];
        a += __builtin_amdgcn_exp2f(sep2f<DIM>(xi, xj) * escale);
      }
    }
    acc += (double)a;
  });
  __shared__ double part[kSumWaves][64];
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kSumWaves; ++w) r += part[w][lane];
    if (valid) {
      r_out[i] = r;
      q_out[i] = (float)(1.0 / r);
    }
  }
}

// Columns of B, split into three bf16 parts, stored part-major then
// column-major: bparts[(p * NC + c) * cap + j].
__global__ __launch_bounds__(kBlock) void k_dense_prep_b(const float* __restrict__ mass, const float* __restrict__ q,
                                                         const int64_t cap, const int32_t n, const int32_t S,
                                                         const int32_t norm, const int32_t NC,
                                                         __bf16* __restrict__ bparts) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= cap) return;
  const bool in = j < n;
  const int64_t SP = species_slots(S);
  const float qj = in ? q[j] : 0.0f;
  for (int c = 0; c < NC; ++c) {
    float v = 0.0f;
    if (in) {
      if (norm == 0) {
        if (c < S) v = mass[SP * j + c];
        else if (c < 2 * S) v = qj * mass[SP * j + (c - S)];
        else if (c == 2 * S) v = qj;
        else if (c == 2 * S + 1) v = 1.0f;
      } else {
        if (c < S) v = mass[SP * j + c];
        else if (c == S) v = 1.0f;
      }
    }
    __bf16 p0, p1, p2;
    split3(v, p0, p1, p2);
    bparts[(0 * (int64_t)NC + c) * cap + j] = p0;
    bparts[(1 * (int64_t)NC + c) * cap + j] = p1;
    bparts[(2 * (int64_t)NC + c) * cap + j] = p2;
  }
}

// Pass 2: one block per 16-row tile, its kExWaves waves taking the near column
// tiles t = wave mod kExWaves; lane l generates the 8 weights
// W[i0 + l%16][32 t + 8 (l/16) + e], the A operand of the MFMA.  The waves'
// partial C tiles are added in wave order, and the first wave finishes.
template <int DIM, int NCB>
__global__ __launch_bounds__(kBlock) void k_dense_exchange(
    const float* __restrict__ pos, const int64_t cap, const int32_t n, const float* __restrict__ min_,
    float* __restrict__ mout, const float* __restrict__ q, const float* __restrict__ bbox,
    const int32_t ntile, const float escale, const float skip_s2, const __bf16* __restrict__ bparts,
    const int32_t S, const int32_t react_a, const int32_t react_b, const int32_t norm,
    double* __restrict__ audit_part) {
  constexpr int NC = 16 * NCB;
  static_assert(kExWaves == kBlock / 64, "one block of kExWaves waves per row tile");
  __shared__ double cpart[kExWaves - 1][NCB * 4][64];
  __shared__ double csh[kRowTile][NC];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rt = blockIdx.x;
  const int i0 = rt * kRowTile;
  const bool active = i0 < n;  // always: one block per row tile
  const int ri = lane & 15, kg = lane >> 4;
  const int i = i0 + ri;
  const bool valid_i = i < n;
  double acc[NCB][4];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[cb][e] = 0.0;
  if (active) {
  const int ii = valid_i ? i : n - 1;
  float xi[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) xi[k] = pos[pos_stride<DIM>() * ii + k];
  float rbox[2 * DIM];
  load_box<DIM>(bbox, i0 / kColTile, rbox);

  for_near_tiles<DIM>(bbox, ntile, rbox, skip_s2, [&](int t) {
    if (t % kExWaves != wave) return;  // another wave's tile
    const int jb = t * kColTile + 8 * kg;
    float w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = jb + e;
      float xj[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) xj[k] = pos[pos_stride<DIM>() * j + k];  // j < cap: rows past n are padding
      const float ww = __builtin_amdgcn_exp2f(sep2f<DIM>(xi, xj) * escale);
      w[e] = (valid_i && j < n) ? ww : 0.0f;
    }
    bf16x8 a0, a1, a2;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 p0, p1, p2;
      split3(w[e], p0, p1, p2);
      a0[e] = p0;
      a1[e] = p1;
      a2[e] = p2;
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = cb * 16 + ri;
      const bf16x8 b0 = *(const bf16x8*)(bparts + (0 * (int64_t)NC + c) * cap + jb);
      const bf16x8 b1 = *(const bf16x8*)(bparts + (1 * (int64_t)NC + c) * cap + jb);
      const bf16x8 b2 = *(const bf16x8*)(bparts + (2 * (int64_t)NC + c) * cap + jb);
      f32x4 tacc = {0.0f, 0.0f, 0.0f, 0.0f};
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, tacc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[cb][e] += (double)tacc[e];
    }
  });
  }  // active
  // the other waves' partial C tiles, added by the first in wave order
  if (wave > 0) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) cpart[wave - 1][cb * 4 + e][lane] = acc[cb][e];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 0; w < kExWaves - 1; ++w)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[cb][e] += cpart[w][cb * 4 + e][lane];
  // C[row 4 kg + e][col] lives in lane (col + 16 kg): gather rows through LDS
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) csh[4 * kg + e][cb * 16 + ri] = acc[cb][e];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  double tot[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) tot[s] = 0.0;
  if (active && lane < kRowTile && valid_i) {
    const double* C = csh[lane];
    const double qi = (double)q[i];
    double Mn[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s >= S) continue;
      const double Mi = (double)min_[species_slots(S) * (int64_t)i + s];
      double dm;
      if (norm == 0) dm = 0.25 * (qi * C[s] + C[S + s] - Mi * (qi * C[2 * S + 1] + C[2 * S]));
      else dm = 0.5 * (C[s] / C[S] - Mi);
      Mn[s] = Mi + dm;
    }
    if (react_a >= 0) {
      double m = fmin(Mn[react_a], Mn[react_b]);
      m = m > 0.0 ? m : 0.0;
      Mn[react_a] -= m;
      Mn[react_b] -= m;
    }
    double va = 0.0, vb = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s >= S) continue;
      const float v = (float)Mn[s];
      mout[species_slots(S) * (int64_t)i + s] = v;
      tot[s] = (double)v;
      if (s == react_a) va = (double)v;
      if (s == react_b) vb = (double)v;
    }
    tot[8] = va - vb;
  }
#pragma unroll
  for (int off = 1; off < kRowTile; off <<= 1)
#pragma unroll
    for (int s = 0; s < 9; ++s) tot[s] += __shfl_xor(tot[s], off);
  if (active && lane == 0) {
    double* part = audit_part + (int64_t)rt * (S + 1);
    for (int s = 0; s < S; ++s) part[s] = tot[s];
    part[S] = tot[8];
  }
}

hipError_t launch_dense_step(int dim, const DenseArgs& a, hipStream_t s) {
  const int32_t n = a.n;
  if (n <= 0) return hipSuccess;
  const int32_t ntile = (n + kColTile - 1) / kColTile;
  const dim3 b(kBlock);
  const int NC = 16 * a.ncb;
  if (a.ncb < 1 || a.ncb > 2 || dim < 1 || dim > 3) return hipErrorInvalidValue;
  const dim3 gbox((unsigned)((ntile + kBlock - 1) / kBlock));
  const dim3 gsum((unsigned)((n + kRowTileSum - 1) / kRowTileSum)), bsum(64 * kSumWaves);
  const dim3 gex((unsigned)((n + kRowTile - 1) / kRowTile));
  const dim3 gprep((unsigned)((a.cap + kBlock - 1) / kBlock));
  auto go = [&](auto d) {
    constexpr int D = decltype(d)::value;
    hipLaunchKernelGGL((k_tile_bbox<D>), gbox, b, 0, s, a.pos, n, a.bbox);
    hipLaunchKernelGGL((k_dense_rowsum<D>), gsum, bsum, 0, s, a.pos, n, a.bbox, ntile, a.escale,
                       a.skip_s2, a.r, a.q);
    hipLaunchKernelGGL(k_dense_prep_b, gprep, b, 0, s, a.mass_in, a.q, a.cap, n, a.S, a.norm, NC, a.bparts);
    if (a.ncb == 1)
      hipLaunchKernelGGL((k_dense_exchange<D, 1>), gex, b, 0, s, a.pos, a.cap, n, a.mass_in, a.mass_out, a.q,
                         a.bbox, ntile, a.escale, a.skip_s2, a.bparts, a.S, a.react_a, a.react_b, a.norm,
                         a.audit_part);
    else
      hipLaunchKernelGGL((k_dense_exchange<D, 2>), gex, b, 0, s, a.pos, a.cap, n, a.mass_in, a.mass_out, a.q,
                         a.bbox, ntile, a.escale, a.skip_s2, a.bparts, a.S, a.react_a, a.react_b, a.norm,
                         a.audit_part);
  };
  if (dim == 1) go(std::integral_constant<int, 1>{});
  else if (dim == 2) go(std::integral_constant<int, 2>{});
  else go(std::integral_constant<int, 3>{});
  return hipGetLastError();
}

}  // namespace rwpt
